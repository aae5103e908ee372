// Bucket lists of one slab group.
//
// The active struts of the group [sa, sb] are the edge-list entries whose
// slab range meets it (Eq. (8) at slab granularity).  As the paper's sweep
// upward does (Sec. 4), a group following the previous one keeps the previous active
// list minus the struts that ended, then appends the edge-list range that
// starts in the new slabs.  Each active strut then emits one (bucket, strut)
// pair per (slab, tile) of its range; a stable radix sort by bucket keeps
// edge-list order inside every bucket, and the bucket offsets are the
// boundaries of the sorted keys.  The adjoint also needs each entry's
// emission index, which group_emi rebuilds from the key and the strut's box.
#include "kernels.hpp"

namespace lsl {
namespace {

constexpr int kCThreads = 256;
constexpr int kCItems = 8;
constexpr int kCTile = kCThreads * kCItems;

__device__ __forceinline__ uint32_t cand_at(const uint32_t* prev, uint32_t n_prev,
                                            uint32_t range_lo, size_t i) {
    return i < n_prev ? prev[i] : range_lo + (uint32_t)(i - n_prev);
}

// keep candidates whose last slab is >= sa
__global__ __launch_bounds__(kCThreads) void k_active_count(const uint32_t* prev, uint32_t n_prev,
                                                            uint32_t range_lo, size_t n_cand,
                                                            const SRange* rg, int32_t sa,
                                                            uint32_t* blk) {
    const size_t base = (size_t)blockIdx.x * kCTile;
    uint32_t c = 0;
    for (int r = 0; r < kCItems; ++r) {
        const size_t i = base + (size_t)r * kCThreads + threadIdx.x;
        if (i < n_cand) c += rg[cand_at(prev, n_prev, range_lo, i)].s1 >= sa ? 1u : 0u;
    }
    // block sum
    __shared__ uint32_t sm[4];
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
    if (lane_id() == 0) sm[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

__global__ __launch_bounds__(kCThreads) void k_active_write(const uint32_t* prev, uint32_t n_prev,
                                                            uint32_t range_lo, size_t n_cand,
                                                            const SRange* rg, int32_t sa,
                                                            const uint32_t* blk_off,
                                                            uint32_t* out, uint32_t cap) {
    __shared__ uint32_t wsum[4];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const size_t base = (size_t)blockIdx.x * kCTile;
    uint32_t run = blk_off[blockIdx.x];
    const uint64_t lt = lanes_below(lane);
    for (int r = 0; r < kCItems; ++r) {
        const size_t i = base + (size_t)r * kCThreads + threadIdx.x;
        uint32_t p = 0;
        bool keep = false;
        if (i < n_cand) {
            p = cand_at(prev, n_prev, range_lo, i);
            keep = rg[p].s1 >= sa;
        }
        const uint64_t m = ballot64(keep);
        if (lane == 0) wsum[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int k = 0; k < 4; ++k) {
            before += k < w ? wsum[k] : 0u;
            tot += wsum[k];
        }
        const uint32_t dst = run + before + (uint32_t)__popcll(m & lt);
        if (keep && dst < cap) out[dst] = p;
        run += tot;
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t pair_count(const SRange& r, int32_t sa, int32_t sb) {
    const int32_t s0 = r.s0 > sa ? r.s0 : sa;
    const int32_t s1 = r.s1 < sb ? r.s1 : sb;
    if (s1 < s0) return 0u;
    return (uint32_t)(s1 - s0 + 1) * (uint32_t)(r.tx1 - r.tx0 + 1) * (uint32_t)(r.ty1 - r.ty0 + 1);
}

__global__ void k_pair_counts(const uint32_t* active, uint32_t n, const SRange* rg, int32_t sa,
                              int32_t sb, uint32_t* counts) {
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) counts[a] = pair_count(rg[active[a]], sa, sb);
    if (a == n) counts[a] = 0u;
}

// One wave emits the pairs of 64 active struts, one strut at a time, the
// wave's lanes writing consecutive pairs (coalesced stores).  Each pair is
// (bucket key, the strut's edge-list position): after the stable sort the
// values are the bucket lists themselves.
__global__ __launch_bounds__(256) void k_emit(const uint32_t* active, uint32_t n,
                                              const SRange* rg, int32_t sa, int32_t sb,
                                              int32_t ntx, int32_t nty, const uint32_t* eoff,
                                              uint32_t* keys, uint32_t* vals, uint32_t cap) {
    const int lane = lane_id();
    const uint32_t a0 = (blockIdx.x * blockDim.x + threadIdx.x) & ~63u;
    if (a0 >= n) return;
    const uint32_t a = a0 + lane;
    SRange r{0, 0, 0, 0, 0, -1};
    uint32_t off = 0, pos = 0;
    if (a < n) {
        pos = active[a];
        r = rg[pos];
        off = eoff[a];
    }
    const int32_t s0 = r.s0 > sa ? r.s0 : sa;
    const uint32_t nx = (uint32_t)(r.tx1 - r.tx0 + 1), ny = (uint32_t)(r.ty1 - r.ty0 + 1);
    const uint32_t cnt = (a < n) ? eoff[a + 1] - off : 0u;
    const uint32_t per_slab = (uint32_t)ntx * (uint32_t)nty;
    const int m = (n - a0) < 64u ? (int)(n - a0) : 64;
    for (int s = 0; s < m; ++s) {
        const uint32_t c = __shfl(cnt, s, kWave);
        const uint32_t o = __shfl(off, s, kWave);
        const uint32_t p = __shfl(pos, s, kWave);
        const uint32_t bx = __shfl(nx, s, kWave), by = __shfl(ny, s, kWave);
        const uint32_t tx0 = __shfl((uint32_t)r.tx0, s, kWave);
        const uint32_t ty0 = __shfl((uint32_t)r.ty0, s, kWave);
        const uint32_t sr = (uint32_t)(__shfl(s0, s, kWave) - sa);
        for (uint32_t j = lane; j < c; j += kWave) {
            const uint32_t tx = j % bx;
            const uint32_t q = j / bx;
            const uint32_t ty = q % by;
            const uint32_t sl = q / by;
            const uint32_t e = o + j;
            if (e >= cap) break;
            keys[e] = (sr + sl) * per_slab + (ty0 + ty) * (uint32_t)ntx + tx0 + tx;
            vals[e] = p;
        }
    }
}

// offsets[b] = first sorted position whose key is >= b
__global__ void k_csr_offsets(const uint32_t* keys, uint32_t n, uint32_t n_buckets,
                              uint32_t* offsets) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const uint32_t kprev = i == 0 ? 0u : keys[i - 1] + 1u;   // first bucket after previous
    const uint32_t k = i == n ? n_buckets : keys[i];
    for (uint32_t b = kprev; b <= k && b <= n_buckets; ++b) offsets[b] = i;
}

__global__ void k_inverse(const uint32_t* active, uint32_t n, uint32_t* inv) {
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) inv[active[a]] = a;
}

// entry i: bucket key -> (slab, tile); its strut's emission began at eoff and
// ran over the strut's box slab-major, then tile row, then tile column
__global__ void k_emi(EmiArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_pairs) return;
    const uint32_t key = a.keys[i], p = a.ids[i];
    const uint32_t per_slab = (uint32_t)a.ntx * (uint32_t)a.nty;
    const uint32_t sl = key / per_slab, rem = key % per_slab;
    const uint32_t ty = rem / (uint32_t)a.ntx, tx = rem % (uint32_t)a.ntx;
    const SRange r = a.ranges[p];
    const int32_t s0 = r.s0 > a.sa ? r.s0 : a.sa;
    const uint32_t nx = (uint32_t)(r.tx1 - r.tx0 + 1), ny = (uint32_t)(r.ty1 - r.ty0 + 1);
    const uint32_t local = (((uint32_t)((int32_t)sl + a.sa - s0) * ny + (ty - r.ty0)) * nx) +
                           (tx - r.tx0);
    a.emi[i] = a.eoff[a.inv[p]] + local;
}

int bits_for(uint32_t n) {
    int b = 0;
    while (b < 32 && (1ull << b) < (uint64_t)n) ++b;
    return b;
}

}  // namespace

size_t group_tmp_elems(size_t n_pairs, size_t n_active, size_t n_cand) {
    size_t a = radix_tmp_elems(n_pairs);
    size_t b = scan_tmp_elems(n_active + 1);
    size_t c = scan_tmp_elems(n_cand / kCTile + 1);
    size_t m = a > b ? a : b;
    return (m > c ? m : c) + 16;
}

lsl_status bin_group(const GroupBuffers& g, hipStream_t st) {
    // 1. active list: kept part of the previous list plus the new range
    const size_t n_cand = (size_t)g.n_prev + (g.range_hi - g.range_lo);
    if (n_cand > 0) {
        const size_t nb = (n_cand + kCTile - 1) / kCTile;
        k_active_count<<<(unsigned)nb, kCThreads, 0, st>>>(g.prev_active, g.n_prev, g.range_lo,
                                                           n_cand, g.ranges, g.sa, g.blk);
        LSL_TRY(exclusive_scan_u32(g.blk, g.blk, nb, g.tmp, nullptr, st));
        k_active_write<<<(unsigned)nb, kCThreads, 0, st>>>(g.prev_active, g.n_prev, g.range_lo,
                                                           n_cand, g.ranges, g.sa, g.blk,
                                                           g.active, g.n_active);
        LSL_HIP(hipGetLastError());
    }
    // 2. pairs per active strut -> emission offsets
    k_pair_counts<<<(g.n_active + 1 + 255) / 256, 256, 0, st>>>(g.active, g.n_active, g.ranges,
                                                                g.sa, g.sb, g.eoff);
    LSL_TRY(exclusive_scan_u32(g.eoff, g.eoff, (size_t)g.n_active + 1, g.tmp, nullptr, st));
    if (g.n_pairs > 0) {
        // 3. emit (bucket, emission index) pairs in edge-list order
        const unsigned ge = (unsigned)(((size_t)g.n_active + 255) / 256);
        k_emit<<<ge, 256, 0, st>>>(g.active, g.n_active, g.ranges, g.sa, g.sb, g.ntx, g.nty,
                                   g.eoff, g.k0, g.v0, g.n_pairs);
        LSL_HIP(hipGetLastError());
        // 4. stable sort by bucket
        int which = 0;
        LSL_TRY(radix_sort_pairs(g.k0, g.v0, g.k1, g.v1, g.n_pairs, bits_for(g.n_buckets), g.tmp,
                                 &which, st));
        const uint32_t* ks = which ? g.k1 : g.k0;
        *g.keys_out = ks;
        *g.ids_out = which ? g.v1 : g.v0;
        // 5. bucket offsets: the boundaries of the sorted keys
        k_csr_offsets<<<(g.n_pairs + 1 + 255) / 256, 256, 0, st>>>(ks, g.n_pairs, g.n_buckets,
                                                                   g.offsets);
        LSL_HIP(hipGetLastError());
    } else {
        *g.keys_out = g.k0;
        *g.ids_out = g.v0;
        LSL_TRY(fill_u32(g.offsets, 0u, (size_t)g.n_buckets + 1, st));
    }
    return LSL_OK;
}

lsl_status group_emi(const EmiArgs& a, hipStream_t st) {
    if (a.n_active) k_inverse<<<(a.n_active + 255) / 256, 256, 0, st>>>(a.active, a.n_active, a.inv);
    if (a.n_pairs) k_emi<<<(a.n_pairs + 255) / 256, 256, 0, st>>>(a);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
