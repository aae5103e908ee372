// Marching squares on the binary slice images (Sec. 4: rough boundary
// curves from the binary image), read as bit images (one bit per pixel), in
// two passes so that segments come out in row-major cell order with no
// atomics on the output:
//
//   count: case code and segment count (0, 1 or 2) per cell; per-block totals
//   scan : exclusive prefix over (plane, block) totals -> per-plane offsets
//   emit : re-derive the counts, rank them inside the block with wave ballots
//          (count bits 0 and 1 -> two ballots) and a per-wave LDS prefix, and
//          write each cell's segments at its offset.
//
// Cell (i, j) has corners (i,j), (i+1,j), (i+1,j+1), (i,j+1) -> bits b0..b3
// (the image's bits).  Segment ends are edge midpoints in grid units;
// the inside lies on the left of each segment; the saddles 5 and 10 keep the
// two inside corners apart.
#include "kernels.hpp"

namespace lsl {
namespace {

constexpr int kMThreads = 256;
constexpr int kMRounds = 8;
constexpr int kMTile = kMThreads * kMRounds;   // cells per block

// Per case: number of segments and up to two segments as
// (x0, y0, x1, y1) in half units of the cell.
__constant__ int8_t kSegCount[16] = {0, 1, 1, 1, 1, 2, 1, 1, 1, 1, 2, 1, 1, 1, 1, 0};
// edge midpoints in half units: B=(1,0) E=(2,1) T=(1,2) L=(0,1)
__constant__ int8_t kSeg[16][2][4] = {
    {{0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 0, 0, 1}, {0, 0, 0, 0}},   // 1: B -> L
    {{2, 1, 1, 0}, {0, 0, 0, 0}},   // 2: E -> B
    {{2, 1, 0, 1}, {0, 0, 0, 0}},   // 3: E -> L
    {{1, 2, 2, 1}, {0, 0, 0, 0}},   // 4: T -> E
    {{1, 0, 0, 1}, {1, 2, 2, 1}},   // 5: B -> L, T -> E
    {{1, 2, 1, 0}, {0, 0, 0, 0}},   // 6: T -> B
    {{1, 2, 0, 1}, {0, 0, 0, 0}},   // 7: T -> L
    {{0, 1, 1, 2}, {0, 0, 0, 0}},   // 8: L -> T
    {{1, 0, 1, 2}, {0, 0, 0, 0}},   // 9: B -> T
    {{2, 1, 1, 0}, {0, 1, 1, 2}},   // 10: E -> B, L -> T
    {{2, 1, 1, 2}, {0, 0, 0, 0}},   // 11: E -> T
    {{0, 1, 2, 1}, {0, 0, 0, 0}},   // 12: L -> E
    {{1, 0, 2, 1}, {0, 0, 0, 0}},   // 13: B -> E
    {{0, 1, 1, 0}, {0, 0, 0, 0}},   // 14: L -> B
    {{0, 0, 0, 0}, {0, 0, 0, 0}},
};

__device__ __forceinline__ uint32_t bit_at(const uint32_t* row, int i) {
    return (row[i >> 5] >> (i & 31)) & 1u;
}

// One plane of a binary image, row-major (BLK = false: `words` 32-bit words
// per row) or block-major (BLK = true: `words` 8x8-block words per block row).
template <bool BLK>
struct Img {
    const void* p;
    size_t words;
    __device__ __forceinline__ uint32_t at(int i, int j) const {
        if (BLK) {
            const uint64_t w = ((const uint64_t*)p)[(size_t)(j >> 3) * words + (size_t)(i >> 3)];
            return (uint32_t)(w >> (8 * (j & 7) + (i & 7))) & 1u;
        }
        return bit_at((const uint32_t*)p + (size_t)j * words, i);
    }
};

template <bool BLK>
__device__ __forceinline__ Img<BLK> plane_img(const void* bits, int32_t W, int32_t H, uint32_t k) {
    Img<BLK> m;
    if (BLK) {
        m.words = (size_t)(W + 7) / 8;
        m.p = (const uint64_t*)bits + (size_t)k * (size_t)((H + 7) / 8) * m.words;
    } else {
        m.words = (size_t)(W + 31) / 32;
        m.p = (const uint32_t*)bits + (size_t)k * (size_t)H * m.words;
    }
    return m;
}

// case code of cell (i, j)
template <bool BLK>
__device__ __forceinline__ int cell_case(const Img<BLK>& m, int i, int j) {
    return (int)(m.at(i, j) | (m.at(i + 1, j) << 1) | (m.at(i + 1, j + 1) << 2) |
                 (m.at(i, j + 1) << 3));
}

template <bool BLK>
__global__ __launch_bounds__(kMThreads) void k_ms_count(const void* bits, int32_t W,
                                                        int32_t H, uint32_t bps, uint8_t* codes,
                                                        unsigned long long* blk) {
    __shared__ uint32_t sm[4];
    const uint32_t k = blockIdx.x / bps, b = blockIdx.x % bps;
    const uint32_t cw = (uint32_t)(W - 1);
    const uint64_t cps = (uint64_t)cw * (uint64_t)(H - 1);
    const Img<BLK> f = plane_img<BLK>(bits, W, H, k);
    uint32_t cnt = 0;
    for (int r = 0; r < kMRounds; ++r) {
        const uint64_t c = (uint64_t)b * kMTile + (uint64_t)r * kMThreads + threadIdx.x;
        if (c < cps) {
            const int j = (int)(c / cw), i = (int)(c % cw);
            const int cs = cell_case<BLK>(f, i, j);
            cnt += (uint32_t)kSegCount[cs];
            if (codes) codes[(size_t)k * cps + c] = (uint8_t)cs;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, kWave);
    if (lane_id() == 0) sm[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

__global__ void k_ms_offsets(const unsigned long long* blk, uint32_t bps, int32_t nk,
                             const unsigned long long* base, int64_t* offsets) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= nk) offsets[k] = (int64_t)(blk[(size_t)k * bps] + (base ? *base : 0ull));
}

// base += this call's total (the segments of several calls share one array)
__global__ void k_ms_advance(unsigned long long* base, const unsigned long long* blk,
                             size_t nb) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += blk[nb];
}

template <bool BLK>
__global__ __launch_bounds__(kMThreads) void k_ms_emit(const void* bits, int32_t W, int32_t H,
                                                       uint32_t bps,
                                                       const unsigned long long* blk,
                                                       const unsigned long long* base,
                                                       float4* segs, int64_t capacity) {
    __shared__ uint32_t wsum[4];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const uint32_t k = blockIdx.x / bps, b = blockIdx.x % bps;
    const uint32_t cw = (uint32_t)(W - 1);
    const uint64_t cps = (uint64_t)cw * (uint64_t)(H - 1);
    const Img<BLK> f = plane_img<BLK>(bits, W, H, k);
    uint64_t run = blk[blockIdx.x] + (base ? *base : 0ull);
    const uint64_t lt = lanes_below(lane);
    for (int r = 0; r < kMRounds; ++r) {
        const uint64_t c = (uint64_t)b * kMTile + (uint64_t)r * kMThreads + threadIdx.x;
        int cs = 0, i = 0, j = 0;
        if (c < cps) {
            j = (int)(c / cw);
            i = (int)(c % cw);
            cs = cell_case<BLK>(f, i, j);
        }
        const int n = kSegCount[cs];
        const uint64_t m0 = ballot64(n & 1), m1 = ballot64(n >> 1);
        const uint32_t wtot = (uint32_t)(__popcll(m0) + 2 * __popcll(m1));
        const uint32_t pre = (uint32_t)(__popcll(m0 & lt) + 2 * __popcll(m1 & lt));
        if (lane == 0) wsum[w] = wtot;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int q = 0; q < 4; ++q) {
            before += q < w ? wsum[q] : 0u;
            tot += wsum[q];
        }
        const uint64_t o = run + before + pre;
        for (int s = 0; s < n; ++s) {
            if ((int64_t)(o + s) < capacity) {
                const int8_t* g = kSeg[cs][s];
                segs[o + s] = make_float4((float)i + 0.5f * g[0], (float)j + 0.5f * g[1],
                                          (float)i + 0.5f * g[2], (float)j + 0.5f * g[3]);
            }
        }
        run += tot;
        __syncthreads();
    }
}

uint32_t blocks_per_slice(int32_t W, int32_t H) {
    const uint64_t cps = (uint64_t)(W - 1) * (uint64_t)(H - 1);
    return (uint32_t)((cps + kMTile - 1) / kMTile);
}

}  // namespace

size_t contour_tmp_elems(int32_t nk, int32_t W, int32_t H) {
    const size_t n = (size_t)nk * blocks_per_slice(W, H) + 1;
    return n + scan_tmp_elems(n);
}

lsl_status launch_contours_count(const void* bits, bool blkl, int32_t nk, int32_t W, int32_t H,
                                 int64_t* offsets, uint8_t* codes, unsigned long long* tmp,
                                 const unsigned long long* base, hipStream_t st) {
    const uint32_t bps = blocks_per_slice(W, H);
    const size_t nb = (size_t)nk * bps;
    if (nb > 0x7fffffffull) {
        set_error("slice_contours: too many planes in one call");
        return LSL_EINVAL;
    }
    unsigned long long* blk = tmp;
    unsigned long long* stmp = tmp + nb + 1;
    if (blkl)
        k_ms_count<true><<<(unsigned)nb, kMThreads, 0, st>>>(bits, W, H, bps, codes, blk);
    else
        k_ms_count<false><<<(unsigned)nb, kMThreads, 0, st>>>(bits, W, H, bps, codes, blk);
    LSL_HIP(hipGetLastError());
    // exclusive scan over nb + 1 entries: the last one receives the total
    LSL_TRY(fill_bytes0(blk + nb, 8, st));
    LSL_TRY(exclusive_scan_u64((const uint64_t*)blk, (uint64_t*)blk, nb + 1, (uint64_t*)stmp,
                               nullptr, st));
    k_ms_offsets<<<(nk + 1 + 255) / 256, 256, 0, st>>>(blk, bps, nk, base, offsets);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_contours_emit(const void* bits, bool blkl, int32_t nk, int32_t W, int32_t H,
                                const unsigned long long* tmp, unsigned long long* base,
                                float* segs, int64_t capacity, hipStream_t st) {
    const uint32_t bps = blocks_per_slice(W, H);
    const size_t nb = (size_t)nk * bps;
    if (blkl)
        k_ms_emit<true><<<(unsigned)nb, kMThreads, 0, st>>>(bits, W, H, bps, tmp, base,
                                                            (float4*)segs, capacity);
    else
        k_ms_emit<false><<<(unsigned)nb, kMThreads, 0, st>>>(bits, W, H, bps, tmp, base,
                                                             (float4*)segs, capacity);
    if (base) k_ms_advance<<<1, 64, 0, st>>>(base, tmp, nb);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
