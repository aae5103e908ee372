// Device-wide building blocks: fills, exclusive prefix sums and a stable LSD
// radix sort of 32-bit (key, value) pairs.  All stream-ordered, no host
// synchronisation, deterministic.
#include "common.hpp"

namespace lsl {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;   // 2048

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block.  Returns
// the exclusive prefix; *block_total receives the block's sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* smem4, T* block_total) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) smem4[w] = inc;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        T s = smem4[i];
        if (i < w) before += s;
        tot += s;
    }
    __syncthreads();
    *block_total = tot;
    return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T* __restrict__ in,
                                                              size_t n, T* __restrict__ sums) {
    __shared__ T sm[4];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    T tot;
    block_exclusive_scan(s, sm, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block sums in place, carry across chunks.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_top(T* __restrict__ sums, size_t nb,
                                                           T* __restrict__ total) {
    __shared__ T sm[4];
    T carry = 0;
    for (size_t c = 0; c < nb; c += kScanTile) {
        const size_t base = c + (size_t)threadIdx.x * kScanItems;
        T v[kScanItems];
        T s = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = (base + i < nb) ? sums[base + i] : T(0);
            s += v[i];
        }
        T tot;
        T pre = block_exclusive_scan(s, sm, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < nb) sums[base + i] = pre;
            pre += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const T* __restrict__ in,
                                                            T* __restrict__ out, size_t n,
                                                            const T* __restrict__ sums) {
    __shared__ T sm[4];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : T(0);
        s += v[i];
    }
    T tot;
    T pre = block_exclusive_scan(s, sm, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
}

template <typename T>
lsl_status scan_impl(const T* in, T* out, size_t n, T* tmp, T* total, hipStream_t st) {
    if (n == 0) {
        if (total) k_scan_top<T><<<1, kScanThreads, 0, st>>>(tmp, 0, total);
        LSL_HIP(hipGetLastError());
        return LSL_OK;
    }
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    k_scan_reduce<T><<<dim3((unsigned)nb), dim3(kScanThreads), 0, st>>>(in, n, tmp);
    k_scan_top<T><<<1, kScanThreads, 0, st>>>(tmp, nb, total);
    k_scan_down<T><<<dim3((unsigned)nb), dim3(kScanThreads), 0, st>>>(in, out, n, tmp);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

// --------------------------------------------------------------------------
// radix sort
// --------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;   // 4096 pairs per block

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             size_t n, int shift,
                                                             uint32_t* __restrict__ hist,
                                                             uint32_t nblocks) {
    __shared__ uint32_t h[4][256];
    const int w = threadIdx.x >> 6, lane = lane_id();
    for (int i = threadIdx.x; i < 4 * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kSortTile;
    const uint64_t lt = lanes_below(lane);
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = base + (size_t)r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        const uint32_t d = valid ? ((keys[i] >> shift) & 255u) : 0u;
        // lanes holding the same digit: one leader adds the group's size
        uint64_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot64(bit);
            peers &= bit ? bb : ~bb;
        }
        if (valid && (peers & lt) == 0) h[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    const int t = threadIdx.x;
    hist[(size_t)t * nblocks + blockIdx.x] = h[0][t] + h[1][t] + h[2][t] + h[3][t];
}

// Scatter with a stable in-block rank: the block's 4096 pairs are taken in
// 16 rounds of 256 in input order; within a round lanes of a wave are ranked
// by lane, waves by wave index.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, size_t n, int shift,
    const uint32_t* __restrict__ offs, uint32_t nblocks) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wc[4][256];
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    base[t] = offs[(size_t)t * nblocks + blockIdx.x];
    wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0;
    __syncthreads();
    const size_t tile0 = (size_t)blockIdx.x * kSortTile;
    const uint64_t lt = lanes_below(lane);
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = tile0 + (size_t)r * kSortThreads + t;
        const bool valid = i < n;
        uint32_t k = 0, v = 0;
        if (valid) {
            k = kin[i];
            v = vin[i];
        }
        const uint32_t d = (k >> shift) & 255u;
        uint64_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot64(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            const uint32_t c0 = wc[0][t], c1 = wc[1][t], c2 = wc[2][t], c3 = wc[3][t];
            const uint32_t b0 = base[t];
            wc[0][t] = b0;
            wc[1][t] = b0 + c0;
            wc[2][t] = b0 + c0 + c1;
            wc[3][t] = b0 + c0 + c1 + c2;
            base[t] = b0 + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wc[w][d] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0;
        __syncthreads();
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_bytes0(uint8_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_iota_u32(uint32_t* p, uint32_t base, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = base + (uint32_t)i;
}

unsigned grid_for(size_t n, unsigned threads) {
    size_t g = (n + threads - 1) / threads;
    if (g > 65536u * 4u) g = 65536u * 4u;
    return (unsigned)(g == 0 ? 1 : g);
}

}  // namespace

size_t scan_tmp_elems(size_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

lsl_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp,
                              uint32_t* total, hipStream_t st) {
    return scan_impl<uint32_t>(in, out, n, tmp, total, st);
}

lsl_status exclusive_scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp,
                              uint64_t* total, hipStream_t st) {
    return scan_impl<uint64_t>(in, out, n, tmp, total, st);
}

size_t radix_tmp_elems(size_t n) {
    const size_t nb = (n + kSortTile - 1) / kSortTile;
    const size_t h = 256 * (nb == 0 ? 1 : nb);
    return h + scan_tmp_elems(h);
}

lsl_status radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, size_t n,
                            int key_bits, uint32_t* tmp, int* which, hipStream_t st) {
    *which = 0;
    if (n <= 1 || key_bits <= 0) return LSL_OK;
    const size_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb > 0xffffffffull / 256) {
        set_error("radix sort: too many items");
        return LSL_EINTERNAL;
    }
    uint32_t* hist = tmp;
    uint32_t* stmp = tmp + 256 * nb;
    uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    for (int shift = 0; shift < key_bits; shift += 8) {
        k_radix_hist<<<dim3((unsigned)nb), dim3(kSortThreads), 0, st>>>(ki, n, shift, hist,
                                                                          (uint32_t)nb);
        LSL_TRY(exclusive_scan_u32(hist, hist, 256 * nb, stmp, nullptr, st));
        k_radix_scatter<<<dim3((unsigned)nb), dim3(kSortThreads), 0, st>>>(
            ki, vi, ko, vo, n, shift, hist, (uint32_t)nb);
        LSL_HIP(hipGetLastError());
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        *which ^= 1;
    }
    return LSL_OK;
}

lsl_status fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
    if (n == 0) return LSL_OK;
    k_fill_u32<<<grid_for(n, 256), 256, 0, st>>>(p, v, n);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status fill_bytes0(void* p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return LSL_OK;
    if (bytes % 4 == 0 && ((uintptr_t)p % 4) == 0)
        return fill_u32((uint32_t*)p, 0u, bytes / 4, st);
    k_fill_bytes0<<<grid_for(bytes, 256), 256, 0, st>>>((uint8_t*)p, bytes);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status iota_u32(uint32_t* p, uint32_t base, size_t n, hipStream_t st) {
    if (n == 0) return LSL_OK;
    k_iota_u32<<<grid_for(n, 256), 256, 0, st>>>(p, base, n);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
