// Bucket lists of one slab group.
//
// The active struts of the group [sa, sb] are the edge-list entries whose
// slab range meets it (Eq. (8) at slab granularity).  As the paper's sweep
// upward does (Sec. 4), a group following the previous one keeps the previous active
// list minus the struts that ended, then appends the edge-list range that
// starts in the new slabs.  A bucket (slab, tile row, tile column) must list
// the struts that cover it in edge-list order.  A tile row's columns are
// grouped in segments of kSegTiles; each active strut emits one (cell,
// strut) item per (slab, tile row, column segment) its box meets, and a
// stable radix sort by cell gives every cell's struts in edge-list order.
// One wave per cell then counts the struts covering each of the cell's
// columns (the bucket sizes, scanned into the offsets) and writes them, in
// that order.  A strut's box is a few tiles wide, so the sort moves a
// fraction of the (slab, tile, strut) pairs, and a cell's columns are few.
// The adjoint also needs each entry's emission index (its position in the
// strut-major order of the pairs), which group_emi rebuilds from the entry's
// bucket and the strut's box.
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

// (slab, tile row, column segment) cells of a strut's box within the group
__device__ __forceinline__ uint32_t cell_count(const SRange& r, int32_t sa, int32_t sb) {
    const int32_t s0 = r.s0 > sa ? r.s0 : sa;
    const int32_t s1 = r.s1 < sb ? r.s1 : sb;
    if (s1 < s0) return 0u;
    return (uint32_t)(s1 - s0 + 1) * row_segments(r);
}

__global__ void k_pair_counts(const uint32_t* active, uint32_t n, const SRange* rg, int32_t sa,
                              int32_t sb, uint32_t* counts, uint32_t* rcounts) {
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) {
        const SRange r = rg[active[a]];
        counts[a] = pair_count(r, sa, sb);
        rcounts[a] = cell_count(r, sa, sb);
    }
    if (a == n) counts[a] = rcounts[a] = 0u;
}

// One wave emits the cells of 64 active struts, one strut at a time, the
// wave's lanes writing consecutive items (coalesced stores): (cell key
// ((slab - sa) nty + ty) nseg + column segment, the strut's edge-list
// position), slab-major, then tile row, then segment.
__global__ __launch_bounds__(256) void k_cell_emit(const uint32_t* active, uint32_t n,
                                                   const SRange* rg, int32_t sa, int32_t nty,
                                                   int32_t nseg, const uint32_t* toff,
                                                   uint32_t* keys, uint32_t* vals, uint32_t cap) {
    const int lane = lane_id();
    const uint32_t a0 = (blockIdx.x * blockDim.x + threadIdx.x) & ~63u;
    if (a0 >= n) return;
    const uint32_t a = a0 + lane;
    SRange r{0, 0, 0, 0, 0, -1};
    uint32_t off = 0, pos = 0, cnt = 0;
    if (a < n) {
        pos = active[a];
        r = rg[pos];
        off = toff[a];
        cnt = toff[a + 1] - off;
    }
    const int32_t s0 = r.s0 > sa ? r.s0 : sa;
    const uint32_t ny = (uint32_t)(r.ty1 - r.ty0 + 1);
    const uint32_t xs0 = (uint32_t)r.tx0 / kSegTiles;
    const uint32_t nxs = (uint32_t)r.tx1 / kSegTiles - xs0 + 1;
    const int m = (n - a0) < 64u ? (int)(n - a0) : 64;
    for (int s = 0; s < m; ++s) {
        const uint32_t c = __shfl(cnt, s, kWave);
        const uint32_t o = __shfl(off, s, kWave);
        const uint32_t p = __shfl(pos, s, kWave);
        const uint32_t by = __shfl(ny, s, kWave);
        const uint32_t bx = __shfl(nxs, s, kWave);
        const uint32_t x0 = __shfl(xs0, s, kWave);
        const uint32_t ty0 = __shfl((uint32_t)r.ty0, s, kWave);
        const uint32_t sr = (uint32_t)(__shfl(s0, s, kWave) - sa);
        for (uint32_t j = lane; j < c; j += kWave) {
            const uint32_t e = o + j;
            if (e >= cap) break;
            const uint32_t q = j / bx;
            keys[e] = ((sr + q / by) * (uint32_t)nty + ty0 + q % by) * (uint32_t)nseg + x0 + j % bx;
            vals[e] = p;
        }
    }
}

__device__ __forceinline__ int wave_min_i(int v) {
    for (int d = 32; d >= 1; d >>= 1) {
        const int o = __shfl_xor(v, d, kWave);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
    for (int d = 32; d >= 1; d >>= 1) {
        const int o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// One wave per cell (slab, tile row, column segment): the cell's struts
// (edge-list order) in chunks of 64, one per lane, lane l owning column
// kSegTiles xs + l of the segment.  For each column a chunk spans, the lanes
// whose strut covers it are ranked by a ballot.  FILL = false: count them
// into the bucket sizes; FILL = true: write them from the bucket's cursor
// on, in lane order.
template <bool FILL>
__global__ __launch_bounds__(256) void k_cell_buckets(const uint32_t* coffs, const uint32_t* cv,
                                                      const SRange* rg, uint32_t n_cells,
                                                      int32_t ntx, int32_t nseg,
                                                      uint32_t* counts, const uint32_t* offsets,
                                                      uint32_t* ids, uint32_t n_pairs) {
    const uint32_t cell = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (cell >= n_cells) return;
    const int lane = lane_id();
    const uint64_t lt = lanes_below(lane);
    const uint32_t beg = coffs[cell], end = coffs[cell + 1];
    const uint32_t row = cell / (uint32_t)nseg;
    const int w0 = (int)(cell % (uint32_t)nseg) * kSegTiles;
    const int w1 = w0 + kSegTiles - 1 < ntx - 1 ? w0 + kSegTiles - 1 : ntx - 1;
    const size_t b0 = (size_t)row * (size_t)ntx;
    const int tx_own = w0 + lane;
    const bool owner = lane < kSegTiles && tx_own <= w1;
    uint32_t cur = 0u;
    if (FILL && owner) cur = offsets[b0 + (size_t)tx_own];
    for (uint32_t c = beg; c < end; c += kWave) {
        const uint32_t i = c + (uint32_t)lane;
        uint32_t p = 0u;
        int t0 = 0x7fffffff, t1 = -1;                  // lanes past the cell cover nothing
        if (i < end) {
            p = cv[i];
            const SRange r = rg[p];
            t0 = r.tx0;
            t1 = r.tx1;
        }
        int lo = wave_min_i(t0), hi = wave_max_i(t1);
        lo = lo > w0 ? lo : w0;
        hi = hi < w1 ? hi : w1;
        for (int tx = lo; tx <= hi; ++tx) {
            const bool cov = t0 <= tx && tx <= t1;
            const uint64_t m = ballot64(cov);
            if (FILL) {
                const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)cur, tx - w0);
                const uint32_t pos = base + (uint32_t)__popcll(m & lt);
                if (cov && pos < n_pairs) ids[pos] = p;
            }
            if (lane == tx - w0) cur += (uint32_t)__popcll(m);
        }
    }
    if (!FILL && owner) counts[b0 + (size_t)tx_own] = cur;
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

// keys[i] = b for every entry i of bucket b: one wave per bucket, its lanes
// writing consecutive entries
__global__ __launch_bounds__(256) void k_expand_keys(const uint32_t* offsets, uint32_t n_buckets,
                                                     uint32_t* keys) {
    const uint32_t b = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (b >= n_buckets) return;
    const uint32_t e = offsets[b + 1];
    for (uint32_t i = offsets[b] + (uint32_t)lane_id(); i < e; i += kWave) keys[i] = b;
}

__global__ void k_inverse(const uint32_t* active, uint32_t n, uint32_t* inv) {
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) inv[active[a]] = a;
}

// entry i: bucket -> (slab, tile); its strut's emission began at eoff and ran
// over the strut's box slab-major, then tile row, then tile column
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

size_t group_tmp_elems(size_t n_pairs, size_t n_active, size_t n_cand, size_t n_buckets) {
    size_t a = radix_tmp_elems(n_pairs);
    size_t b = scan_tmp_elems(n_active + 1);
    size_t c = scan_tmp_elems(n_cand / kCTile + 1);
    size_t d = scan_tmp_elems(n_buckets + 1);
    size_t m = a > b ? a : b;
    m = m > c ? m : c;
    return (m > d ? m : d) + 16;
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
    // 2. pairs per active strut -> emission offsets (the adjoint's emission
    // index); cells per active strut -> their offsets
    k_pair_counts<<<(g.n_active + 1 + 255) / 256, 256, 0, st>>>(g.active, g.n_active, g.ranges,
                                                                g.sa, g.sb, g.eoff, g.toff);
    LSL_TRY(exclusive_scan_u32(g.eoff, g.eoff, (size_t)g.n_active + 1, g.tmp, nullptr, st));
    LSL_TRY(exclusive_scan_u32(g.toff, g.toff, (size_t)g.n_active + 1, g.tmp, nullptr, st));
    const uint32_t nseg = (uint32_t)((g.ntx + kSegTiles - 1) / kSegTiles);
    const uint32_t n_cells = (uint32_t)(g.sb - g.sa + 1) * (uint32_t)g.nty * nseg;
    if (g.n_pairs > 0 && g.n_cells > 0) {
        // 3. emit (cell, strut position) items in edge-list order
        const unsigned ge = (unsigned)(((size_t)g.n_active + 255) / 256);
        k_cell_emit<<<ge, 256, 0, st>>>(g.active, g.n_active, g.ranges, g.sa, g.nty, (int32_t)nseg,
                                        g.toff, g.k0, g.v0, g.n_cells);
        LSL_HIP(hipGetLastError());
        // 4. stable sort by cell, and the cells' CSR
        int which = 0;
        LSL_TRY(radix_sort_pairs(g.k0, g.v0, g.k1, g.v1, g.n_cells, bits_for(n_cells), g.tmp,
                                 &which, st));
        const uint32_t* ck = which ? g.k1 : g.k0;
        const uint32_t* cv = which ? g.v1 : g.v0;
        k_csr_offsets<<<(g.n_cells + 1 + 255) / 256, 256, 0, st>>>(ck, g.n_cells, n_cells,
                                                                   g.roffs);
        LSL_HIP(hipGetLastError());
        // 5. bucket sizes, scanned into the offsets
        const unsigned gr = (n_cells + 3) / 4;
        k_cell_buckets<false><<<gr, 256, 0, st>>>(g.roffs, cv, g.ranges, n_cells, g.ntx,
                                                  (int32_t)nseg, g.offsets, nullptr, nullptr, 0u);
        LSL_HIP(hipGetLastError());
        LSL_TRY(fill_u32(g.offsets + g.n_buckets, 0u, 1, st));
        LSL_TRY(exclusive_scan_u32(g.offsets, g.offsets, (size_t)g.n_buckets + 1, g.tmp, nullptr,
                                   st));
        // 6. the bucket lists, into the buffers not holding the sorted cells
        uint32_t* ids = which ? g.v0 : g.v1;
        k_cell_buckets<true><<<gr, 256, 0, st>>>(g.roffs, cv, g.ranges, n_cells, g.ntx,
                                                 (int32_t)nseg, nullptr, g.offsets, ids,
                                                 g.n_pairs);
        LSL_HIP(hipGetLastError());
        *g.ids_out = ids;
        *g.keys_out = which ? g.k0 : g.k1;
    } else {
        *g.keys_out = g.k0;
        *g.ids_out = g.v0;
        LSL_TRY(fill_u32(g.offsets, 0u, (size_t)g.n_buckets + 1, st));
    }
    return LSL_OK;
}

lsl_status group_emi(const EmiArgs& a, hipStream_t st) {
    if (a.n_pairs && a.n_buckets) {
        k_expand_keys<<<(a.n_buckets + 3) / 4, 256, 0, st>>>(a.offsets, a.n_buckets, a.keys);
        LSL_HIP(hipGetLastError());
    }
    if (a.n_active) k_inverse<<<(a.n_active + 255) / 256, 256, 0, st>>>(a.active, a.n_active, a.inv);
    if (a.n_pairs) k_emi<<<(a.n_pairs + 255) / 256, 256, 0, st>>>(a);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
