// Field evaluation (Eq. 6 with the closed form of Eq. 7, Sec. 4).
//
// The float32 kernel of the paper's kernel (field_q32.hpp) serves lattices
// whose planes may share reference planes; the method below (field_block.hpp)
// serves float64, the compact Gaussian and float32 lattices whose planes are
// coarse against the smallest support (every plane staged from float64).
//
// One wave owns an 8x8 pixel block of one tile and one slab of planes; the
// four waves of a workgroup take the four 8x8 blocks of a 16x16 tile (or
// four of the blocks of a larger tile).  The wave walks its tile's bucket
// list (edge-list order) 64 struts at a time.  Per strut and plane it stages,
// in float64, the foot F of the block centre c on the strut's line:
//
//   tc = (c - a).u,  m = a + tc u - c  (m is orthogonal to u),
//
// and drops the strut for that plane when no pixel of the block can be within
// R of the segment: with F* the segment's point nearest to c, D = |F* - c| and
// n = (F* - c)/D, the segment lies in n.(x - F*) >= 0, so a pixel c + d is at
// least D - n.d >= D - (3.5 dx |n_x| + 3.5 dy |n_y|) from it (the block is
// flat, so struts passing above or below it are dropped sooner than by a
// bounding circle).  The surviving struts are compacted into LDS with a
// ballot/mbcnt prefix.  For a pixel p = c + d (d in the plane) the
// arclength coordinates of the strut ends with origin at the foot of p are
//
//   alpha = -tc - d.u,   beta = (L - tc) - d.u,
//   H = R^2 - dist(p, line)^2 = (R^2 - |m|^2) + 2 m.d - |d|^2 + (d.u)^2,
//
// all formed from small quantities, and the term is
//
//   r/R^4 * integral over [clamp(alpha), clamp(beta)] of (H - t^2)^2 dt
//     = r/R^4 * (cb - ca) * (H^2 - 2/3 H S1 + S2/5),
//   S1 = ca^2 + ca cb + cb^2,  S2 = (ca^2 + cb^2) S1 - (ca cb)^2,
//   ca, cb = alpha, beta clamped to [-sqrt(H), sqrt(H)].
//
// Terms outside the support come out as exact zeros (cb - ca = 0).  A strut
// is a candidate of a block and plane only where it passes the distance test
// and its binned pixel and plane ranges cover them, so every tile size, slab
// depth and group split hands the block the same candidates in the same
// order.  Sums are compensated, s' = s + g, e += g - (s' - s): float32 adds
// each run of four consecutive candidates plainly, ((t0 + t1) + t2) + t3, and
// compensates once per run; float64 compensates every term.
#include <type_traits>

#include "field_block.hpp"
#include "field_q32.hpp"

namespace lsl {
namespace {

template <typename T, int SZ, bool STATS, int K, bool SR, bool PR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_field(FieldArgs a, uint32_t n_items) {
    const int wv = threadIdx.x >> 6;
    const uint32_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t item = blk * 4u + (uint32_t)wv;
    if (item >= n_items) return;
    // item -> (slab, tile, 8x8 block): blocks of a tile are consecutive
    const int nsub = a.tile / kBlockPix;
    uint32_t t = item;
    const int sub = (int)(t % (uint32_t)(nsub * nsub));
    t /= (uint32_t)(nsub * nsub);
    const int tx = (int)(t % (uint32_t)a.ntx);
    t /= (uint32_t)a.ntx;
    const int ty = (int)(t % (uint32_t)a.nty);
    t /= (uint32_t)a.nty;
    // float32, the paper's kernel, shared reference planes: field_q32.hpp;
    // otherwise (float64, the Gaussian, every plane its own reference)
    // field_block.hpp
    if constexpr (std::is_same<T, float>::value && K == LSL_KERNEL_QUARTIC && !PR) {
        __shared__ q32::Lds<SZ> lds[4];
        q32::field_block<SZ, STATS, SR>(a, a.s_lo + (int)t, tx, ty, sub, lds[wv]);
    } else {
        __shared__ Stage<T> stage[4][kWave];
        __shared__ T pend[4][fieldk::pend_elems<T, SZ>()];
        __shared__ double line[4][fieldk::kLineVals * kWave];
        fieldk::field_block<T, SZ, STATS, K, SR>(a, a.s_lo + (int)t, tx, ty, sub, stage[wv],
                                                 pend[wv], line[wv]);
    }
}

// Block-major binary image of a field: one wave takes 8 rows x 64 columns
// (8 blocks); each row's ballot gives one byte of each block's word.
template <typename T>
__global__ __launch_bounds__(256) void k_bits_blk(const T* field, int32_t nk, int32_t W,
                                                  int32_t H, T C, uint64_t* out) {
    const int lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nbx = (W + 7) / 8, nby = (H + 7) / 8;
    const int chunks = (W + 63) / 64;
    const uint64_t n = (uint64_t)nk * (uint64_t)nby * (uint64_t)chunks;
    if (wave >= n) return;
    const int c = (int)(wave % (uint64_t)chunks);
    const uint64_t kb = wave / (uint64_t)chunks;           // plane * nby + block row
    const int by = (int)(kb % (uint64_t)nby);
    const uint64_t k = kb / (uint64_t)nby;
    const T* f = field + k * (uint64_t)W * (uint64_t)H;
    const int i = c * 64 + lane;
    uint64_t word = 0;                                     // lane b < 8: block c*8 + b
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int j = by * 8 + r;
        const uint64_t m = ballot64(i < W && j < H && f[(size_t)j * W + i] >= C);
        word |= ((m >> (8 * (lane & 7))) & 0xffull) << (8 * r);
    }
    if (lane < 8 && c * 8 + lane < nbx) out[kb * (uint64_t)nbx + (uint64_t)(c * 8 + lane)] = word;
}

template <typename T, int SZ, int K, bool SR, bool PR>
lsl_status launch_tkp(const FieldArgs& a, bool stats, uint32_t n_items, hipStream_t st) {
    const unsigned blocks = (n_items + 3u) / 4u;
    if (stats)
        k_field<T, SZ, true, K, SR, PR><<<blocks, 256, 0, st>>>(a, n_items);
    else
        k_field<T, SZ, false, K, SR, PR><<<blocks, 256, 0, st>>>(a, n_items);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

// Coarse planes (every plane its own reference) matter to the float32
// kernel of the paper's kernel only.
template <typename T, int SZ, int K, bool SR>
lsl_status launch_tk(const FieldArgs& a, bool stats, uint32_t n_items, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value && K == LSL_KERNEL_QUARTIC) {
        if (a.plane_ref) return launch_tkp<T, SZ, K, SR, true>(a, stats, n_items, st);
    }
    return launch_tkp<T, SZ, K, SR, false>(a, stats, n_items, st);
}

template <typename T, int SZ>
lsl_status launch_t(const FieldArgs& a, bool stats, uint32_t n_items, hipStream_t st) {
    if (a.kernel == LSL_KERNEL_GAUSS)
        return a.strut_R ? launch_tk<T, SZ, LSL_KERNEL_GAUSS, true>(a, stats, n_items, st)
                         : launch_tk<T, SZ, LSL_KERNEL_GAUSS, false>(a, stats, n_items, st);
    return a.strut_R ? launch_tk<T, SZ, LSL_KERNEL_QUARTIC, true>(a, stats, n_items, st)
                     : launch_tk<T, SZ, LSL_KERNEL_QUARTIC, false>(a, stats, n_items, st);
}

template <typename T>
lsl_status launch_dt(const FieldArgs& a, bool stats, uint32_t n_items, hipStream_t st) {
    if (a.slab <= 1) return launch_t<T, 1>(a, stats, n_items, st);
    if (a.slab <= 2) return launch_t<T, 2>(a, stats, n_items, st);
    if (a.slab <= 4) return launch_t<T, 4>(a, stats, n_items, st);
    if (a.slab <= 8) return launch_t<T, 8>(a, stats, n_items, st);
    return launch_t<T, 16>(a, stats, n_items, st);
}

}  // namespace

lsl_status launch_field(int dtype, const FieldArgs& a, bool stats, hipStream_t st) {
    const int nsub = a.tile / kBlockPix;
    const uint64_t n_items = (uint64_t)(a.s_hi - a.s_lo + 1) * (uint64_t)a.ntx * (uint64_t)a.nty *
                             (uint64_t)(nsub * nsub);
    if (n_items == 0 || a.nk <= 0) return LSL_OK;
    if (n_items > 0xfffffff0ull) {
        set_error("slice_field: too many work items in one launch");
        return LSL_EINTERNAL;
    }
    if (dtype == LSL_F32) return launch_dt<float>(a, stats, (uint32_t)n_items, st);
    return launch_dt<double>(a, stats, (uint32_t)n_items, st);
}

lsl_status launch_bits_blk(int dtype, const void* field, int32_t nk, int32_t W, int32_t H,
                           double C, uint64_t* out, hipStream_t st) {
    const uint64_t waves = (uint64_t)nk * (uint64_t)((H + 7) / 8) * (uint64_t)((W + 63) / 64);
    if (waves == 0) return LSL_OK;
    const uint64_t blocks = (waves + 3) / 4;
    if (dtype == LSL_F32)
        k_bits_blk<float><<<(unsigned)blocks, 256, 0, st>>>((const float*)field, nk, W, H,
                                                            (float)C, out);
    else
        k_bits_blk<double><<<(unsigned)blocks, 256, 0, st>>>((const double*)field, nk, W, H, C,
                                                             out);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
