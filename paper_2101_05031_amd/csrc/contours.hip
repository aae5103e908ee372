// Marching squares on the binary slice images (Sec. 4: rough boundary
// curves from the binary image).  The images are block-major: one 64-bit
// word per 8x8 pixel block, bit 8 r + c = pixel (8 bx + c, 8 by + r).
//
// Cell (i, j) has corners (i,j), (i+1,j), (i+1,j+1), (i,j+1) -> bits b0..b3
// of its case code.  For the 64 cells of a block these are four 64-bit masks
// built from the block word and its right, lower and lower-right neighbours
// with shifts, so one lane finds all boundary cells of a block at once:
//   M = (b0|b1|b2|b3) & ~(b0&b1&b2&b3)       cells with one or two segments
//   S = saddles 5 and 10                        cells with two segments
// A wave takes one strip of 8 pixel rows of one plane (lane = block column):
//
//   count: popcount(M) + popcount(S) over the strip -> per-strip totals
//   scan : exclusive prefix over (plane, strip) -> per-plane offsets
//   emit : per-row totals of the strip, then per 64-block chunk a wave prefix
//          of the per-(row, block) counts, so every boundary cell knows its
//          rank in row-major cell order; each writes its segments there.
//
// Segment ends are edge midpoints in grid units; the inside lies on the left
// of each segment; the saddles 5 and 10 keep the two inside corners apart.
// Outputs are deterministic and written with no atomics.
#include <utility>

#include "kernels.hpp"

namespace lsl {
namespace {

constexpr int kMThreads = 256;
constexpr uint64_t kCol0 = 0x0101010101010101ull;   // column 0 of every row
constexpr uint64_t kCol7 = 0x8080808080808080ull;   // column 7 of every row

// Per case: number of segments and up to two segments as
// (x0, y0, x1, y1) in half units of the cell.  The tables are folded at
// compile time into register constants (kSegCountBits, kSegWord), so a
// lane's lookup by its own case is arithmetic, not a memory load.
constexpr int8_t kSegCountT[16] = {0, 1, 1, 1, 1, 2, 1, 1, 1, 1, 2, 1, 1, 1, 1, 0};
// edge midpoints in half units: B=(1,0) E=(2,1) T=(1,2) L=(0,1)
constexpr int8_t kSegT[16][2][4] = {
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

// 2 bits per case: the segment count
constexpr uint32_t seg_count_bits() {
    uint32_t r = 0;
    for (int c = 0; c < 16; ++c) r |= (uint32_t)kSegCountT[c] << (2 * c);
    return r;
}
// cases 4w .. 4w+3, 16 bits each: segment s in bits 8s .. 8s+7, its
// coordinates (each 0, 1 or 2) in 2 bits apiece, x0 lowest
constexpr uint64_t seg_word(int w) {
    uint64_t r = 0;
    for (int c = 0; c < 4; ++c)
        for (int s = 0; s < 2; ++s)
            for (int e = 0; e < 4; ++e)
                r |= (uint64_t)kSegT[4 * w + c][s][e] << (16 * c + 8 * s + 2 * e);
    return r;
}
constexpr uint32_t kSegCountBits = seg_count_bits();
constexpr uint64_t kSegWord[4] = {seg_word(0), seg_word(1), seg_word(2), seg_word(3)};

__device__ __forceinline__ int seg_count(int cs) { return (int)((kSegCountBits >> (2 * cs)) & 3u); }

// segment s of case cs as (x0, y0, x1, y1) in half units
__device__ __forceinline__ void seg_points(int cs, int s, int8_t g[4]) {
    const int w = cs >> 2;
    const uint64_t word = w == 0 ? kSegWord[0] : w == 1 ? kSegWord[1]
                        : w == 2 ? kSegWord[2] : kSegWord[3];
    const uint32_t b = (uint32_t)(word >> (16 * (cs & 3) + 8 * s)) & 0xffu;
#pragma unroll
    for (int e = 0; e < 4; ++e) g[e] = (int8_t)((b >> (2 * e)) & 3u);
}


// The four corner masks of the 64 cells of block (bx, by) of one plane, with
// the cells outside [0, W-1) x [0, H-1) cleared from M and S.
struct CellMasks {
    uint64_t b0, b1, b2, b3, m, s;
};

__device__ __forceinline__ CellMasks cell_masks(const uint64_t* P, int nbx, int nby, int bx,
                                                int by, int32_t W, int32_t H) {
    const size_t row = (size_t)by * (size_t)nbx;
    const bool right = bx + 1 < nbx, down = by + 1 < nby;
    const uint64_t w = P[row + bx];
    const uint64_t wr = right ? P[row + bx + 1] : 0ull;
    const uint64_t wd = down ? P[row + nbx + bx] : 0ull;
    const uint64_t wdr = (right && down) ? P[row + nbx + bx + 1] : 0ull;
    CellMasks c;
    c.b0 = w;
    c.b1 = ((w >> 1) & ~kCol7) | ((wr & kCol0) << 7);              // pixel (i+1, j)
    c.b3 = (w >> 8) | (wd << 56);                                   // pixel (i, j+1)
    const uint64_t b1d = ((wd >> 1) & ~kCol7) | ((wdr & kCol0) << 7);
    c.b2 = (c.b1 >> 8) | (b1d << 56);                               // pixel (i+1, j+1)
    int nc = W - 1 - 8 * bx, nr = H - 1 - 8 * by;                   // valid cell columns / rows
    nc = nc < 0 ? 0 : (nc > 8 ? 8 : nc);
    nr = nr < 0 ? 0 : (nr > 8 ? 8 : nr);
    const uint64_t cols = (uint64_t)((1u << nc) - 1u) * kCol0;
    const uint64_t rows = nr >= 8 ? ~0ull : ((1ull << (8 * nr)) - 1ull);
    const uint64_t valid = cols & rows;
    const uint64_t all = c.b0 & c.b1 & c.b2 & c.b3;
    const uint64_t any = c.b0 | c.b1 | c.b2 | c.b3;
    c.m = any & ~all & valid;
    c.s = ((c.b0 & c.b2 & ~c.b1 & ~c.b3) | (c.b1 & c.b3 & ~c.b0 & ~c.b2)) & valid;
    return c;
}

// v + v of the lane the DPP control selects (0 where it selects none)
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ uint32_t dpp_add(uint32_t acc, uint32_t v) {
    return acc + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, BANKS, false);
}

// inclusive prefix over the wave's lanes with DPP moves: within rows of 16
// (shifts by 1, 2, 3 of the inputs, then by 4 and 8 of the partial sums),
// then across rows (broadcasts of lanes 15 and 31)
__device__ __forceinline__ uint32_t wave_incl32(uint32_t v) {
    const uint32_t v0 = v;
    v = dpp_add<0x111, 0xf, 0xf>(v0, v0);          // row_shr:1
    v = dpp_add<0x112, 0xf, 0xf>(v, v0);           // row_shr:2
    v = dpp_add<0x113, 0xf, 0xf>(v, v0);           // row_shr:3
    v = dpp_add<0x114, 0xf, 0xe>(v, v);            // row_shr:4, lanes 4..15 of a row
    v = dpp_add<0x118, 0xf, 0xc>(v, v);            // row_shr:8, lanes 8..15
    v = dpp_add<0x142, 0xa, 0xf>(v, v);            // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc, 0xf>(v, v);            // row_bcast:31 into rows 2 and 3
    return v;
}

// the same for 64-bit words of packed counts whose fields never carry (the
// low halves' sums stay below 2^32)
__device__ __forceinline__ uint64_t wave_incl(uint64_t v, int) {
    return (uint64_t)wave_incl32((uint32_t)v) | ((uint64_t)wave_incl32((uint32_t)(v >> 32)) << 32);
}

__device__ __forceinline__ uint64_t wave_last(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), kWave - 1);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// total over the wave of packed counts that never carry
__device__ __forceinline__ uint64_t wave_total(uint64_t v) { return wave_last(wave_incl(v, 0)); }

// segments of row r (0..7) of a block: one per boundary cell, two per saddle
__device__ __forceinline__ uint32_t row_count(const CellMasks& c, int r) {
    return (uint32_t)(__popc((uint32_t)(c.m >> (8 * r)) & 0xffu) +
                      __popc((uint32_t)(c.s >> (8 * r)) & 0xffu));
}

// Segments per strip (tot) and per row of the strip (rows: two rows per
// word, 32 bits each, lower row in the low half).
__global__ __launch_bounds__(kMThreads) void k_strip_count(const uint64_t* img, int32_t nk,
                                                           int32_t W, int32_t H,
                                                           unsigned long long* tot,
                                                           unsigned long long* rows) {
    const int lane = lane_id();
    const int nbx = (W + 7) / 8, nby = (H + 7) / 8;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (wave >= (uint64_t)nk * (uint64_t)nby) return;
    const uint64_t k = wave / (uint64_t)nby;
    const int by = (int)(wave % (uint64_t)nby);
    const uint64_t* P = img + k * (uint64_t)nby * (uint64_t)nbx;
    uint64_t t2[4] = {0, 0, 0, 0};
    for (int bx = lane; bx < nbx; bx += kWave) {
        const CellMasks c = cell_masks(P, nbx, nby, bx, by, W, H);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            t2[q] += (uint64_t)row_count(c, 2 * q) | ((uint64_t)row_count(c, 2 * q + 1) << 32);
    }
    uint64_t cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        t2[q] = wave_total(t2[q]);
        cnt += (t2[q] & 0xffffffffull) + (t2[q] >> 32);
    }
    if (lane == 0) {
        tot[wave] = cnt;
#pragma unroll
        for (int q = 0; q < 4; ++q) rows[4 * wave + q] = t2[q];
    }
}

__global__ void k_ms_offsets(const unsigned long long* scan, uint32_t per_plane, int32_t nk,
                             const unsigned long long* base, int64_t* offsets) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= nk) offsets[k] = (int64_t)(scan[(size_t)k * per_plane] + (base ? *base : 0ull));
}

// base += this call's total (the segments of several calls share one array)
__global__ void k_ms_advance(unsigned long long* base, const unsigned long long* scan,
                             size_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += scan[n];
}

// Optional outputs of the emit pass for sub-pixel segments and chaining:
// endpoints interpolated on the field, each segment's start and end edge and
// its cell.  Edge ids per plane: 2 (y W + x) for the edge (x,y)-(x+1,y),
// 2 (y W + x) + 1 for (x,y)-(x,y+1).
struct SubPix {
    const void* field;                // [nk][H][W], T
    double C;
    uint32_t* edge_s;                 // [total] start edge of each segment
    uint32_t* edge_e;                 // [total] end edge
    uint32_t* cell;                   // [total] j (W-1) + i
};

// One end of a segment of cell (i, j) at table point g (half units): its
// edge id and, for SUB, the point where g - C interpolates to zero along the
// edge, from its lower-(j, i) grid point P to Q.
template <bool SUB, typename T>
__device__ __forceinline__ float2 seg_end(const int8_t* g, int i, int j, int32_t W, const T* f,
                                          T C, uint32_t* edge) {
    if (!SUB) return make_float2((float)i + 0.5f * g[0], (float)j + 0.5f * g[1]);   // midpoint
    if (!(g[1] & 1)) {                              // horizontal edge at y = j + g/2
        const int y = j + (g[1] >> 1);
        *edge = 2u * ((uint32_t)y * (uint32_t)W + (uint32_t)i);
        const T gp = f[(size_t)y * W + i], gq = f[(size_t)y * W + i + 1];
        return make_float2((float)((T)i + (C - gp) / (gq - gp)), (float)y);
    }
    const int x = i + (g[0] >> 1);                  // vertical edge at x = i + g/2
    *edge = 2u * ((uint32_t)j * (uint32_t)W + (uint32_t)x) + 1u;
    const T gp = f[(size_t)j * W + x], gq = f[(size_t)(j + 1) * W + x];
    return make_float2((float)x, (float)((T)j + (C - gp) / (gq - gp)));
}

// A boundary cell of the emit pass: its first segment's position, column,
// and row | case << 28.
struct MsItem {
    uint64_t o;
    uint32_t ci, cj;
};
constexpr uint32_t kItems = 128;       // items per wave and round

template <bool SUB, typename T>
__global__ __launch_bounds__(kMThreads) void k_strip_emit(const uint64_t* img, int32_t nk,
                                                          int32_t W, int32_t H,
                                                          const unsigned long long* scan,
                                                          const unsigned long long* rows,
                                                          const unsigned long long* base,
                                                          float4* segs, int64_t capacity,
                                                          SubPix sp) {
    const int lane = lane_id();
    const int nbx = (W + 7) / 8, nby = (H + 7) / 8;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (wave >= (uint64_t)nk * (uint64_t)nby) return;
    const uint64_t k = wave / (uint64_t)nby;
    const int by = (int)(wave % (uint64_t)nby);
    const uint64_t* P = img + k * (uint64_t)nby * (uint64_t)nbx;
    __shared__ MsItem s_items[kMThreads / kWave][kItems];

    uint64_t pos[8];                 // next free position of each row, for this lane
    {
        // the strip's per-row totals from the count pass
        uint64_t run = scan[wave] + (base ? *base : 0ull);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t t = rows[4 * wave + q];
            pos[2 * q] = run;
            run += t & 0xffffffffull;
            pos[2 * q + 1] = run;
            run += t >> 32;
        }
    }
    // per 64-block chunk: the boundary cells as items in LDS (each with its
    // case and the position of its first segment), then one item per lane
    MsItem* items = s_items[threadIdx.x / kWave];
    const T* f = SUB ? (const T*)sp.field + k * (uint64_t)W * (uint64_t)H : nullptr;
    for (int bx0 = 0; bx0 < nbx; bx0 += kWave) {
        const int bx = bx0 + lane;
        CellMasks c{};
        if (bx < nbx) c = cell_masks(P, nbx, nby, bx, by, W, H);
        // this chunk's per-row counts, four rows of 16 bits per word (a row
        // of a 64-block chunk holds at most 2 x 8 x 64 = 1024 segments),
        // their exclusive prefix over the lanes and their totals
        uint64_t ex[2], all[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            uint64_t v = 0;
#pragma unroll
            for (int h = 0; h < 4; ++h) v |= (uint64_t)row_count(c, 4 * q + h) << (16 * h);
            const uint64_t inc = wave_incl(v, lane);
            all[q] = wave_last(inc);
            ex[q] = inc - v;
        }
        if (ballot64(c.m != 0ull) != 0ull) {
            // the lane's cells are items exl .. exl + nl - 1 (lane-major)
            const uint32_t nl = (uint32_t)__popcll(c.m);
            const uint32_t incl = wave_incl32(nl);
            const uint32_t n_items = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
            const uint32_t exl = incl - nl;
            for (uint32_t R = 0; R < n_items; R += kItems) {
                uint64_t mb = c.m;
                uint32_t t = exl;
                int rcur = -1;
                uint64_t o = 0;
                while (mb) {
                    const int bit = __ffsll((unsigned long long)mb) - 1;
                    mb &= mb - 1ull;
                    const int r = bit >> 3;
                    if (r != rcur) {
                        o = pos[r] + ((ex[r >> 2] >> (16 * (r & 3))) & 0xffffull);
                        rcur = r;
                    }
                    const int cs = (int)(((c.b0 >> bit) & 1ull) | (((c.b1 >> bit) & 1ull) << 1) |
                                         (((c.b2 >> bit) & 1ull) << 2) |
                                         (((c.b3 >> bit) & 1ull) << 3));
                    if (t >= R && t < R + kItems)
                        items[t - R] = MsItem{o, (uint32_t)(8 * bx + (bit & 7)),
                                              (uint32_t)(8 * by + r) | ((uint32_t)cs << 28)};
                    o += (uint64_t)seg_count(cs);
                    ++t;
                }
                __builtin_amdgcn_wave_barrier();
                const uint32_t m = n_items - R < kItems ? n_items - R : kItems;
                for (uint32_t q = (uint32_t)lane; q < m; q += kWave) {
                    const MsItem it = items[q];
                    const int cs = (int)(it.cj >> 28);
                    const int ci = (int)it.ci, cj = (int)(it.cj & 0x0fffffffu);
                    const int n = seg_count(cs);
                    for (int sg = 0; sg < n; ++sg) {
                        const uint64_t os = it.o + (uint64_t)sg;
                        if ((int64_t)os < capacity) {
                            int8_t g[4];
                            seg_points(cs, sg, g);
                            uint32_t es = 0, ee = 0;
                            const float2 a = seg_end<SUB, T>(g, ci, cj, W, f, (T)sp.C, &es);
                            const float2 b = seg_end<SUB, T>(g + 2, ci, cj, W, f, (T)sp.C, &ee);
                            segs[os] = make_float4(a.x, a.y, b.x, b.y);
                            if (SUB) {
                                sp.edge_s[os] = es;
                                sp.edge_e[os] = ee;
                                sp.cell[os] = (uint32_t)cj * (uint32_t)(W - 1) + (uint32_t)ci;
                            }
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) pos[r] += (all[r >> 2] >> (16 * (r & 3))) & 0xffffull;
    }
}

// Case code of every cell, [nk][H-1][W-1] bytes (optional output).
__global__ __launch_bounds__(kMThreads) void k_ms_codes(const uint64_t* img, int32_t W, int32_t H,
                                                        uint8_t* codes) {
    const uint32_t k = blockIdx.y;
    const int nbx = (W + 7) / 8, nby = (H + 7) / 8;
    const uint64_t cw = (uint64_t)(W - 1), cps = cw * (uint64_t)(H - 1);
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cps) return;
    const int j = (int)(c / cw), i = (int)(c % cw);
    const uint64_t* P = img + (uint64_t)k * (uint64_t)nby * (uint64_t)nbx;
    auto at = [&](int x, int y) -> uint32_t {
        const uint64_t w = P[(size_t)(y >> 3) * (size_t)nbx + (size_t)(x >> 3)];
        return (uint32_t)(w >> (8 * (y & 7) + (x & 7))) & 1u;
    };
    codes[(uint64_t)k * cps + c] =
        (uint8_t)(at(i, j) | (at(i + 1, j) << 1) | (at(i + 1, j + 1) << 2) | (at(i, j + 1) << 3));
}

// Row-major copy of block-major images: word w of row j holds pixels
// 32 w .. 32 w + 31 (bit x % 32 is pixel x).  A thread reads the four block
// words of one output column and block row once and writes its eight rows
// (byte r of each block word is row r of the block).
__global__ __launch_bounds__(256) void k_bits_rows(const uint64_t* img, uint64_t n, int32_t W,
                                                   int32_t H, uint32_t* out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int words = (W + 31) / 32, nbx = (W + 7) / 8, nby = (H + 7) / 8;
    const int w = (int)(t % (uint64_t)words);
    const uint64_t kb = t / (uint64_t)words;
    const int by = (int)(kb % (uint64_t)nby);
    const uint64_t k = kb / (uint64_t)nby;
    const uint64_t* row = img + (k * (uint64_t)nby + (uint64_t)by) * (uint64_t)nbx;
    uint64_t q[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int bx = 4 * w + c;
        q[c] = bx < nbx ? row[bx] : 0ull;
    }
    uint32_t* o = out + (k * (uint64_t)H + (uint64_t)(8 * by)) * (uint64_t)words + (uint64_t)w;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (8 * by + r < H) {
            uint32_t v = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) v |= (uint32_t)((q[c] >> (8 * r)) & 0xffull) << (8 * c);
            o[(uint64_t)r * (uint64_t)words] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Chaining.  Segment s of plane k ends on edge e; the segment that starts on
// e lies in the cell across e, found by binary search of the plane's
// row-major cell indices, and follows s.  Chains and ranks then come from
// pointer jumping over all segments of the call at once:
//   1. X = succ (a tail points to itself), M = own index; K rounds of
//      M = min(M, M[X]), X = X[X] give every segment of a closed loop the
//      loop's smallest index, and leave a segment on an open chain pointing
//      at the chain's tail (succ[X] < 0).
//   2. Heads are segments with no predecessor and the smallest segment of
//      each loop; P = pred (a head points to itself), D = 0 at heads, else 1;
//      K rounds of D += D[P], P = P[P] give each segment its head and its
//      distance from it.
// K = 1 + ceil(log2(longest chain)).  All integer: bitwise deterministic.
__device__ __forceinline__ uint32_t plane_of(const int64_t* off, int32_t nk, uint64_t s) {
    int32_t lo = 0, hi = nk;                       // off[lo] <= s < off[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if ((uint64_t)off[mid] <= s) lo = mid; else hi = mid;
    }
    return (uint32_t)lo;
}

__global__ void k_poly_succ(const int64_t* off, int32_t nk, uint64_t total, int32_t W, int32_t H,
                            const uint32_t* edge_s, const uint32_t* edge_e, const uint32_t* cell,
                            int32_t* succ) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    const uint32_t k = plane_of(off, nk, s);
    const uint64_t lo = (uint64_t)off[k], hi = (uint64_t)off[k + 1];
    const uint32_t cw = (uint32_t)(W - 1);
    const uint32_t c = cell[s], i = c % cw, j = c / cw;
    const uint32_t e = edge_e[s], at = e >> 1;
    const int x = (int)(at % (uint32_t)W), y = (int)(at / (uint32_t)W);
    int ni = (int)i, nj = (int)j;
    if (e & 1u) ni = x == (int)i ? (int)i - 1 : (int)i + 1;     // vertical edge
    else nj = y == (int)j ? (int)j - 1 : (int)j + 1;            // horizontal edge
    int32_t r = -1;
    if (ni >= 0 && nj >= 0 && ni < W - 1 && nj < H - 1) {
        const uint32_t nc = (uint32_t)nj * cw + (uint32_t)ni;
        uint64_t a = lo, b = hi;                   // first position with cell >= nc
        while (a < b) {
            const uint64_t mid = (a + b) >> 1;
            if (cell[mid] < nc) a = mid + 1; else b = mid;
        }
        for (uint64_t q = a; q < hi && q < a + 2 && cell[q] == nc; ++q)
            if (edge_s[q] == e) r = (int32_t)q;
    }
    succ[s] = r;
}

__global__ void k_poly_pred(const int32_t* succ, uint64_t total, int32_t* pred) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < total && succ[s] >= 0) pred[succ[s]] = (int32_t)s;
}

__global__ void k_poly_init_min(const int32_t* succ, uint64_t total, int32_t* X, int32_t* M) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    X[s] = succ[s] < 0 ? (int32_t)s : succ[s];
    M[s] = (int32_t)s;
}

__global__ void k_poly_jump_min(const int32_t* X, const int32_t* M, uint64_t total, int32_t* X2,
                                int32_t* M2) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    const int32_t x = X[s];
    M2[s] = M[s] < M[x] ? M[s] : M[x];
    X2[s] = X[x];
}

__global__ void k_poly_heads(const int32_t* succ, const int32_t* pred, const int32_t* X,
                             const int32_t* M, uint64_t total, int32_t* P, int32_t* D) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    const bool on_loop = succ[X[s]] >= 0;
    const bool head = pred[s] < 0 || (on_loop && M[s] == (int32_t)s);
    P[s] = head ? (int32_t)s : pred[s];
    D[s] = head ? 0 : 1;
}

__global__ void k_poly_jump_rank(const int32_t* P, const int32_t* D, uint64_t total, int32_t* P2,
                                 int32_t* D2) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    const int32_t p = P[s];
    D2[s] = D[s] + D[p];
    P2[s] = P[p];
}

__global__ void k_poly_out(const int64_t* off, int32_t nk, uint64_t total, const int32_t* P,
                           const int32_t* D, int32_t* chain, int32_t* rank) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    const uint32_t k = plane_of(off, nk, s);
    chain[s] = P[s] - (int32_t)off[k];
    rank[s] = D[s];
}

}  // namespace

// tmp: per-strip totals (n + 1, scanned in place), the scan's scratch, then
// the per-row totals of every strip (4 words per strip)
size_t contour_tmp_elems(int32_t nk, int32_t W, int32_t H) {
    (void)W;
    const size_t n = (size_t)nk * (size_t)((H + 7) / 8);
    return (n + 1) + scan_tmp_elems(n + 1) + 4 * n;
}

namespace {
unsigned long long* strip_rows(unsigned long long* tmp, size_t n) {
    return tmp + (n + 1) + scan_tmp_elems(n + 1);
}
}  // namespace

lsl_status launch_contours_count(const uint64_t* img, int32_t nk, int32_t W, int32_t H,
                                 int64_t* offsets, uint8_t* codes, unsigned long long* tmp,
                                 const unsigned long long* base, hipStream_t st) {
    const uint32_t nby = (uint32_t)((H + 7) / 8);
    const size_t n = (size_t)nk * nby;
    if (n > 0x7fffffffull / 4) {
        set_error("slice_contours: too many planes in one call");
        return LSL_EINVAL;
    }
    unsigned long long* tot = tmp;
    unsigned long long* stmp = tmp + n + 1;
    if (W > 1 && H > 1)
        k_strip_count<<<(unsigned)((n + 3) / 4), kMThreads, 0, st>>>(img, nk, W, H, tot,
                                                                     strip_rows(tmp, n));
    else
        LSL_TRY(fill_bytes0(tot, n * 8, st));
    LSL_HIP(hipGetLastError());
    if (codes && W > 1 && H > 1) {
        const uint64_t cps = (uint64_t)(W - 1) * (uint64_t)(H - 1);
        const uint64_t words = (uint64_t)((H + 7) / 8) * (uint64_t)((W + 7) / 8);
        for (int32_t k = 0; k < nk; k += 65535) {        // grid y holds at most 65535 planes
            const int32_t m = nk - k < 65535 ? nk - k : 65535;
            const dim3 grid((unsigned)((cps + kMThreads - 1) / kMThreads), (unsigned)m);
            k_ms_codes<<<grid, kMThreads, 0, st>>>(img + (uint64_t)k * words, W, H,
                                                   codes + (uint64_t)k * cps);
        }
        LSL_HIP(hipGetLastError());
    }
    // exclusive scan over n + 1 entries: the last one receives the total
    LSL_TRY(fill_bytes0(tot + n, 8, st));
    LSL_TRY(exclusive_scan_u64((const uint64_t*)tot, (uint64_t*)tot, n + 1, (uint64_t*)stmp,
                               nullptr, st));
    k_ms_offsets<<<(nk + 1 + 255) / 256, 256, 0, st>>>(tot, nby, nk, base, offsets);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_contours_emit(const uint64_t* img, int32_t nk, int32_t W, int32_t H,
                                const unsigned long long* tmp, unsigned long long* base,
                                float* segs, int64_t capacity, hipStream_t st) {
    const uint32_t nby = (uint32_t)((H + 7) / 8);
    const size_t n = (size_t)nk * nby;
    if (W > 1 && H > 1)
        k_strip_emit<false, float><<<(unsigned)((n + 3) / 4), kMThreads, 0, st>>>(
            img, nk, W, H, tmp, strip_rows((unsigned long long*)tmp, n), base, (float4*)segs,
            capacity, SubPix{});
    if (base) k_ms_advance<<<1, 64, 0, st>>>(base, tmp, n);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_bits_rows(const uint64_t* img, int32_t nk, int32_t W, int32_t H,
                            uint32_t* bits, hipStream_t st) {
    const uint64_t n = (uint64_t)nk * (uint64_t)((H + 7) / 8) * (uint64_t)((W + 31) / 32);
    if (n == 0) return LSL_OK;
    k_bits_rows<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(img, n, W, H, bits);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_polylines(const uint64_t* img, const void* field, int dtype, double C,
                            int32_t nk, int32_t W, int32_t H, const unsigned long long* tmp,
                            const int64_t* offsets, uint64_t total, int32_t rounds, float* segs,
                            uint32_t* scratch, int32_t* chain, int32_t* rank, hipStream_t st) {
    if (total == 0 || W < 2 || H < 2) return LSL_OK;
    const uint32_t nby = (uint32_t)((H + 7) / 8);
    const size_t n = (size_t)nk * nby;
    SubPix sp;
    sp.field = field;
    sp.C = C;
    sp.edge_s = scratch;
    sp.edge_e = scratch + total;
    sp.cell = scratch + 2 * total;
    if (dtype == LSL_F32)
        k_strip_emit<true, float><<<(unsigned)((n + 3) / 4), kMThreads, 0, st>>>(
            img, nk, W, H, tmp, strip_rows((unsigned long long*)tmp, n), nullptr,
            (float4*)segs, (int64_t)total, sp);
    else
        k_strip_emit<true, double><<<(unsigned)((n + 3) / 4), kMThreads, 0, st>>>(
            img, nk, W, H, tmp, strip_rows((unsigned long long*)tmp, n), nullptr,
            (float4*)segs, (int64_t)total, sp);
    LSL_HIP(hipGetLastError());
    if (!chain || !rank) return LSL_OK;
    int32_t* succ = (int32_t*)(scratch + 3 * total);
    int32_t* pred = succ + total;
    int32_t* A0 = pred + total;                    // X | P
    int32_t* A1 = A0 + total;                      // M | D
    int32_t* B0 = A1 + total;
    int32_t* B1 = B0 + total;
    const unsigned g = (unsigned)((total + 255) / 256);
    k_poly_succ<<<g, 256, 0, st>>>(offsets, nk, total, W, H, sp.edge_s, sp.edge_e, sp.cell, succ);
    LSL_TRY(fill_u32((uint32_t*)pred, 0xffffffffu, total, st));
    k_poly_pred<<<g, 256, 0, st>>>(succ, total, pred);
    k_poly_init_min<<<g, 256, 0, st>>>(succ, total, A0, A1);
    for (int r = 0; r < rounds; ++r) {
        k_poly_jump_min<<<g, 256, 0, st>>>(A0, A1, total, B0, B1);
        std::swap(A0, B0);
        std::swap(A1, B1);
    }
    k_poly_heads<<<g, 256, 0, st>>>(succ, pred, A0, A1, total, B0, B1);
    std::swap(A0, B0);
    std::swap(A1, B1);
    for (int r = 0; r < rounds; ++r) {
        k_poly_jump_rank<<<g, 256, 0, st>>>(A0, A1, total, B0, B1);
        std::swap(A0, B0);
        std::swap(A1, B1);
    }
    k_poly_out<<<g, 256, 0, st>>>(offsets, nk, total, A0, A1, chain, rank);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

size_t polyline_scratch_elems(uint64_t total) { return (size_t)(9 * total + 16); }

}  // namespace lsl
