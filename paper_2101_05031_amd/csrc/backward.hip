// Adjoint of the field: dL/dr and dL/dv for a loss L of the sliced field,
// given G = dL/dg at the pixels of a plane range (the radius tuning of
// Sec. 5.3 changes exactly the strut weights r).
//
// Per pixel p and strut (a, b) with u = (b - a)/L, q = a - p, alpha = q.u,
// beta = alpha + L, H = R^2 - |q|^2 + alpha^2 (squared half chord), the
// clamped ends ca, cb and q_perp = q - alpha u (the offset of the line from
// p, |q_perp| < R):
//
//   I       = R^-4 (cb - ca) Q                         (the field term / r)
//   dI/dalpha = -phi(alpha), dI/dbeta = phi(beta),     phi(t) = R^-4 max(H - t^2, 0)^2
//   J = dI/dH = 2 R^-4 (cb - ca) (H - S1/3)
//   K = dI/dalpha + dI/dbeta + 2 alpha J
//
// and, through u = (b - a)/|b - a| and q,
//
//   dI/db = phi(beta) u + (K/L) q_perp
//   dI/da = -phi(alpha) u - (K/L + 2J) q_perp
//
// (the alpha-sized parts of K u and 2 J q cancel exactly, so every summed
// quantity stays of the size of R).  The loss gradient of a strut needs nine
// pixel sums: Aw = sum G I, Aa = sum G phi(alpha), Ab = sum G phi(beta),
// AKq = sum G K q_perp (3), AJq = sum G J q_perp (3):
//
//   dL/dr = Aw,  dL/db = r [Ab u + AKq / L],  dL/da = -r [Aa u + AKq / L + 2 AJq].
//
// Around the 8x8 block centre c, q_perp = m - d + (d.u) u with m = F - c the
// offset of the foot F of c (uniform per strut and plane) and d = p - c the
// pixel's offset (the same in every plane).  Within a slab m is affine in the
// plane index k, m_k = m_0 + k dm, so over the slab's planes
//   sum G K q_perp = (m_0 - d + (d.u) u) sum G K + dm sum k G K
// and likewise for J: each (pixel, strut, plane) adds to seven registers.
//
// Work split.  One wave takes one (tile, slab) bucket and walks the tile's
// 8x8 blocks in a fixed order.  For 32 list entries at a time it stages, per
// block and plane, the same block-centre quantities as the forward pass
// (m and tc), compacts the struts that reach the block in any
// plane of the slab, and then for each such strut loops over only the planes
// it reaches: every lane adds its pixel's contribution to seven registers,
// the wave sums them once per (strut, block), and one lane adds the sums into
// the entry's LDS slot.  The slots are written once per bucket entry, at the
// entry's emission index, so each (slab, tile, strut) pair gets exactly one
// partial, with no atomics, and a strut's pairs lie side by side.  The
// per-strut sums then run over each strut's pairs in emission order
// (slab, tile), and the nodes gather their struts' gradients through a node
// -> strut incidence list.  Every reduction has a fixed order.
#include "field_q32.hpp"
#include "kernels.hpp"

namespace lsl {
namespace {

constexpr int kChunk = 32;      // bucket entries staged at a time
constexpr int kParts = 9;       // pixel sums per (strut, bucket)

// per (strut, plane): the in-plane part of m = F - c, H0 = R^2 - |m|^2, and
// the ends -tc, L - tc
// (packed: 20 bytes in float32, so the wave's LDS keeps five waves per SIMD)
template <typename T>
struct BPlane {
    T mx, my, H0, ntc, nbtc;
};

template <typename T>
__device__ __forceinline__ T dsqrt(T x);
template <>
__device__ __forceinline__ float dsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ __forceinline__ double dsqrt<double>(double x) { return __builtin_sqrt(x); }

template <typename T>
__device__ __forceinline__ T dclamp(T v, T h);
template <>
__device__ __forceinline__ float dclamp<float>(float v, float h) {
    return __builtin_amdgcn_fmed3f(v, -h, h);
}
template <>
__device__ __forceinline__ double dclamp<double>(double v, double h) {
    return __builtin_fmin(__builtin_fmax(v, -h), h);
}

template <typename T>
__device__ __forceinline__ T dmax(T a, T b) {
    return __builtin_fmax(a, b);
}
template <>
__device__ __forceinline__ float dmax<float>(float a, float b) {
    return __builtin_fmaxf(a, b);
}

template <typename T>
__device__ __forceinline__ T dfma(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float dfma<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// Wave sums of the nine per-lane partials, added into one LDS slot row.
//
// float: a reduce-scatter.  v_permlane32_swap exchanges the upper half-wave
// of one register with the lower half-wave of another, so one swap and one
// add fold two values into one register (lanes 0-31 hold half sums of the
// first, lanes 32-63 of the second); v_permlane16_swap does the same for odd
// and even rows.  After the two folds, a row rotate by 8 pairs the half-rows,
// and three DPP steps finish each 8-lane group.  Lane group g = lane / 8
// then holds the total of value kScatter[g]; the ninth value takes a plain
// DPP reduction into lane 63.  The nine owner lanes add their totals to the
// slot, each at its own address, in a fixed order of operations.
constexpr int kSumLane = 63;

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_take(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}

__device__ __forceinline__ float fold32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float fold16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// value index whose total lane group g (= lane / 8) holds after reduce8
__device__ __forceinline__ int scatter_index(int lane) {
    const int g = lane >> 3, row = g >> 1;
    return 4 * (g & 1) + (((row & 1) << 1) | (row >> 1));
}

__device__ __forceinline__ float reduce8(float v0, float v1, float v2, float v3, float v4,
                                         float v5, float v6, float v7, int lane) {
    const float w0 = fold32(v0, v1), w1 = fold32(v2, v3), w2 = fold32(v4, v5),
                w3 = fold32(v6, v7);
    const float x0 = fold16(w0, w1), x1 = fold16(w2, w3);   // rows: values 0 2 1 3 | 4 6 5 7
    const float t0 = x0 + dpp_take<0x128, 0xF>(x0);          // row_ror:8
    const float t1 = x1 + dpp_take<0x128, 0xF>(x1);
    float y = (lane & 8) ? t1 : t0;
    y += dpp_take<0xB1, 0xF>(y);     // quad_perm [1,0,3,2]
    y += dpp_take<0x4E, 0xF>(y);     // quad_perm [2,3,0,1]
    y += dpp_take<0x141, 0xF>(y);    // row_half_mirror: every lane holds its group's total
    return y;
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_take<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v += dpp_take<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v += dpp_take<0x141, 0xF>(v);    // row_half_mirror
    v += dpp_take<0x140, 0xF>(v);    // row_mirror: every lane holds its row's sum
    v += dpp_take<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_take<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ void deposit(float* sl, const float (&v)[9], int lane, int own) {
    const float y = reduce8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], lane);
    const float z = wave_sum(v[8]);
    if (own >= 0) sl[own] += own == 8 ? z : y;
}

__device__ __forceinline__ void deposit(double* sl, const double (&v)[9], int lane, int) {
    double t[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        double x = v[q];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
        t[q] = x;
    }
    if (lane == kSumLane)
#pragma unroll
        for (int q = 0; q < 9; ++q) sl[q] += t[q];
}

// The slot entry this lane adds to in deposit (float), or -1.
__device__ __forceinline__ int deposit_owner(int lane) {
    if (lane == kSumLane) return 8;
    return (lane & 7) == 0 ? scatter_index(lane) : -1;
}

template <typename T, int SZ, bool SR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_backward(BackArgs a, uint32_t n_items) {
    // compacted list of the struts that reach the current block
    __shared__ T bs_ux[kChunk], bs_uy[kChunk], bs_uz[kChunk];
    __shared__ T bs_m0[3][kChunk], bs_dm[3][kChunk];   // m at the slab's first plane, step per plane
    __shared__ uint32_t bs_planes[kChunk], bs_pos[kChunk];
    __shared__ BPlane<T> bp[kChunk][SZ];
    __shared__ T slot[kChunk][kParts];

    const int lane = lane_id();
    const uint32_t item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= n_items) return;
    uint32_t t = item;
    const int tx = (int)(t % (uint32_t)a.ntx);
    t /= (uint32_t)a.ntx;
    const int ty = (int)(t % (uint32_t)a.nty);
    t /= (uint32_t)a.nty;
    const int slab = a.s_lo + (int)t;
    int kb = slab * a.slab, ke = kb + a.slab;
    if (kb < a.k0) kb = a.k0;
    if (ke > a.k0 + a.nk) ke = a.k0 + a.nk;
    const int nvalid = ke - kb;
    const uint32_t bucket = ((uint32_t)(slab - a.group_s0) * (uint32_t)a.nty + (uint32_t)ty) *
                                (uint32_t)a.ntx + (uint32_t)tx;
    uint32_t beg = a.offsets[bucket], end = a.offsets[bucket + 1];
    if (end > a.n_pairs) end = a.n_pairs;
    if (beg >= end) return;

    const int nsub = a.tile / kBlockPix;
    const int lx = lane & 7, ly = lane >> 3;
    const T dX = (T)(((double)lx - 3.5) * a.dx);
    const T dY = (T)(((double)ly - 3.5) * a.dy);
    const T d2 = dX * dX + dY * dY;
    const T dX2 = dX + dX, dY2 = dY + dY;
    // half extents of a block's pixel centres about its centre
    const double hx = 3.5 * a.dx, hy = 3.5 * a.dy;
    // one support: the (slightly widened) cull radius and R^2 are uniform
    const double Rc_u = a.R * (1.0 + 1e-7);
    const double Rc2_u = Rc_u * Rc_u;
    const double R2_u = a.R * a.R;
    const int own = deposit_owner(lane);
    const StrutRec<T>* recs = (const StrutRec<T>*)a.rec;
    const T* grad = (const T*)a.grad;
    T* part = (T*)a.partial;

    for (uint32_t cbase = beg; cbase < end; cbase += kChunk) {
        const int nent = (int)((end - cbase) < (uint32_t)kChunk ? (end - cbase) : (uint32_t)kChunk);
        for (int q = lane; q < kChunk * kParts; q += kWave) (&slot[0][0])[q] = T(0);
        __builtin_amdgcn_wave_barrier();

        // this chunk's strut records, one per lane (lanes >= nent idle)
        bool valid = lane < nent;
        uint32_t p = valid ? a.ids[cbase + (uint32_t)lane] : 0u;
        valid = valid && p < a.n_binned;
        const StrutRec<T> r = recs[valid ? p : 0u];
        const double ax = (double)r.ax, ay = (double)r.ay, az = (double)r.az;
        const Line ln = strut_line(r);
        const double L = ln.L, ux = ln.ux, uy = ln.uy, uz = ln.uz;

        for (int sub = 0; sub < nsub * nsub; ++sub) {
            const int i0 = tx * a.tile + (sub % nsub) * kBlockPix;
            const int j0 = ty * a.tile + (sub / nsub) * kBlockPix;
            if (i0 >= a.W || j0 >= a.H) continue;
            const int pi = i0 + lx, pj = j0 + ly;
            const bool pix = pi < a.W && pj < a.H;
            T G[SZ];
#pragma unroll
            for (int k = 0; k < SZ; ++k)
                G[k] = (pix && k < nvalid)
                           ? grad[((size_t)(kb + k - a.k0) * (size_t)a.H + (size_t)pj) *
                                      (size_t)a.W + (size_t)pi]
                           : T(0);
            const double cx = a.x0 + ((double)i0 + 4.0) * a.dx;
            const double cy = a.y0 + ((double)j0 + 4.0) * a.dy;
            const double wx = cx - ax, wy = cy - ay;
            const double txy = fma(wx, ux, wy * uy);

            // stage: which planes each strut reaches; per-plane data goes to
            // the lane's own row of bp (the compacted list keeps the row)
            uint32_t planes = 0;
#pragma unroll
            for (int k = 0; k < SZ; ++k) {
                if (k < nvalid) {
                    const double z = a.z0 + ((double)(kb + k) + 0.5) * a.dz;
                    const double wz = z - az;
                    const double tc = fma(wz, uz, txy);
                    const double mx = fma(tc, ux, -wx), my = fma(tc, uy, -wy),
                                 mz = fma(tc, uz, -wz);
                    const double m2 = fma(mx, mx, fma(my, my, mz * mz));
                    // the field kernel's reach test: with e = F* - c (F* the
                    // segment's point nearest to c), no pixel of the block is
                    // within R when D^2 - hx |e_x| - hy |e_y| >= R D
                    const double dt = fmin(fmax(tc, 0.0), L) - tc;
                    const double ex = fma(dt, ux, mx), ey = fma(dt, uy, my);
                    const double D2 = fma(dt, dt, m2);
                    const double q = D2 - fma(hx, fabs(ex), hy * fabs(ey));
                    // per-strut supports: the strut's cull radius and R^2
                    double Rc2 = Rc2_u, R2 = R2_u;
                    if (SR) {
                        const double Rs = (double)r.pad;
                        const double Rc = Rs * (1.0 + 1e-7);
                        Rc2 = Rc * Rc;
                        R2 = Rs * Rs;
                    }
                    if (valid && (q <= 0.0 || q * q < Rc2 * D2)) {
                        planes |= 1u << k;
                        BPlane<T> P;
                        P.mx = (T)mx;
                        P.my = (T)my;
                        P.H0 = (T)(R2 - m2);
                        P.ntc = (T)(-tc);
                        P.nbtc = (T)(L - tc);
                        bp[lane][k] = P;
                    }
                }
            }
            const uint64_t mask = ballot64(planes != 0u);
            if (mask == 0ull) continue;
            if (planes != 0u) {
                const int q = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                bs_ux[q] = (T)ux;
                bs_uy[q] = (T)uy;
                bs_uz[q] = (T)uz;
                bs_planes[q] = planes;
                bs_pos[q] = (uint32_t)lane;
                // m is affine in the plane index: m_k = m_0 + k dm
                const double wz0 = a.z0 + ((double)kb + 0.5) * a.dz - az;
                const double tc0 = fma(wz0, uz, txy);
                const double dtc = a.dz * uz;
                bs_m0[0][q] = (T)fma(tc0, ux, -wx);
                bs_m0[1][q] = (T)fma(tc0, uy, -wy);
                bs_m0[2][q] = (T)fma(tc0, uz, -wz0);
                bs_dm[0][q] = (T)(dtc * ux);
                bs_dm[1][q] = (T)(dtc * uy);
                bs_dm[2][q] = (T)fma(dtc, uz, -a.dz);
            }
            __builtin_amdgcn_wave_barrier();
            const int n = __popcll(mask);
            for (int j = 0; j < n; ++j) {
                const T bux = bs_ux[j], buy = bs_uy[j], buz = bs_uz[j];
                const uint32_t bpos = bs_pos[j];
                const uint32_t planes_s = __builtin_amdgcn_readfirstlane(bs_planes[j]);
                // sums over the planes: G I, G phi(alpha), G phi(beta), G K, k G K,
                // G J, k G J (k = plane index in the slab)
                T Aw = 0, Aa = 0, Ab = 0, AK = 0, AKk = 0, AJ = 0, AJk = 0;
                const T du = dfma(dX, bux, dY * buy);         // d.u: the same in every plane
                const T dd = dfma(du, du, -d2);               // (d.u)^2 - |d|^2
#pragma unroll
                for (int k = 0; k < SZ; ++k) {
                    if (k < nvalid && ((planes_s >> k) & 1u)) {
                        const BPlane<T> P = bp[bpos][k];
                        const T g = G[k];
                        const T al = P.ntc - du;
                        const T be = P.nbtc - du;
                        const T H = dfma(P.mx, dX2, dfma(P.my, dY2, P.H0 + dd));
                        const T Hc = dmax<T>(H, T(0));
                        const T h = dsqrt<T>(Hc);
                        const T ca = dclamp<T>(al, h), cb = dclamp<T>(be, h);
                        const T D = cb - ca;
                        const T x2 = ca * ca, y2 = cb * cb, xy = ca * cb;
                        const T q2 = x2 + y2;
                        const T S1 = q2 + xy;
                        const T S2 = dfma(q2, S1, -(xy * xy));
                        const T Q = dfma(H, dfma(T(-2.0 / 3.0), S1, H), T(0.2) * S2);
                        Aw = dfma(g * D, Q, Aw);
                        // phi at the ends: zero outside the chord, where the end
                        // is clamped to +-h, and off the strut's reach (Hc = 0)
                        T pa = Hc - x2;
                        pa = pa * pa;
                        T pb = Hc - y2;
                        pb = pb * pb;
                        Aa = dfma(g, pa, Aa);
                        Ab = dfma(g, pb, Ab);
                        const T J = T(2) * dfma(T(-1.0 / 3.0), S1, H) * D;   // J R^4
                        const T K = dfma(T(2) * al, J, pb - pa);               // K R^4
                        const T gK = g * K, gJ = g * J;
                        AK += gK;
                        AJ += gJ;
                        if (k > 0) {
                            AKk = dfma(gK, T(k), AKk);
                            AJk = dfma(gJ, T(k), AJk);
                        }
                    }
                }
                // sum G K q_perp over the planes, q_perp = m_k - d + (d.u) u and
                // m_k = m_0 + k dm:  (m_0 - d + (d.u) u) sum G K + dm sum k G K
                const T qx = dfma(du, bux, bs_m0[0][j] - dX), qy = dfma(du, buy, bs_m0[1][j] - dY),
                        qz = dfma(du, buz, bs_m0[2][j]);
                const T dmx = bs_dm[0][j], dmy = bs_dm[1][j], dmz = bs_dm[2][j];
                const T AKx = dfma(qx, AK, dmx * AKk), AKy = dfma(qy, AK, dmy * AKk),
                        AKz = dfma(qz, AK, dmz * AKk);
                const T AJx = dfma(qx, AJ, dmx * AJk), AJy = dfma(qy, AJ, dmy * AJk),
                        AJz = dfma(qz, AJ, dmz * AJk);
                const T v[9] = {Aw, Aa, Ab, AKx, AKy, AKz, AJx, AJy, AJz};
                deposit(slot[bpos], v, lane, own);
                __builtin_amdgcn_wave_barrier();
            }
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
        // each entry's sums go to its emission index (the strut's pairs are
        // then contiguous for the per-strut reduction)
        for (int q = lane; q < nent * kParts; q += kWave) {
            const uint32_t e = a.emi[cbase + (uint32_t)(q / kParts)];
            if (e < a.n_pairs) part[(size_t)e * kParts + (size_t)(q % kParts)] = (&slot[0][0])[q];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// float32 path
// ---------------------------------------------------------------------------
// One wave takes one (tile, slab) bucket, as above, but walks the tile in
// regions of 2x2 8x8 sub-blocks (16x16 pixels, one pixel of each sub-block
// per lane) -- or of one 8x8 block when the pixels are coarse against the
// smallest support (see below) -- and the slab in windows of at most 8
// planes.  For 64 bucket entries at a time (one per lane) and each window:
//
//  * region pre-test, per entry: which regions the strut's support may
//    reach at all (the distance from the region's box centre to the segment,
//    in float64, against R (1 + 1e-4) plus the box's half-diagonal); the
//    (entry, region) pairs that pass are compacted region-major, and the
//    rest, whose terms would all be exact zeros, are never staged;
//  * staging, one pair per lane, 64 at a time: the strut's line around its
//    region's centre c (float64), its values per plane, and the reach test
//    of the field kernel for every (sub-block, plane), in float32 against
//    the support widened by 1e-5 relative (so that no strut that reaches a
//    pixel is dropped; one that does not adds exact zeros);
//  * evaluation, per staged pair that reaches its region: every lane adds
//    its pixels' terms over the (sub-block, plane) pairs the strut reaches,
//    and the wave sums the nine pixel sums once per (strut, region) into the
//    entry's slot, in region order.
//
// Lengths are in units of the strut's support R (hats): H^ = 1 - |q_perp|^2
// / R^2 <= 1, the ends alpha^ = A_k - d.u^ and beta^ = B_k - d.u^ (A_k =
// -tc_k / R, B_k = (L - tc_k) / R).  As in the field kernel, a reference
// plane r carries the strut's values and from plane r to plane k the foot
// moves by (k - r) dz u_z along the strut:  A_k = A_r - (k - r) dz^ u_z and
// H^_k = G_k + E + (k - r) c1 (d.u^), with G_k = 1 - |m_k|^2 / R^2 (per
// plane, from float64), E = 2 m_r^.d^ - |d^|^2 + (d.u^)^2 and c1 = 2 dz^ u_z.
// Here r is the middle of the planes of the window that the strut reaches,
// so the shifts stay small and m_r is of the size of R.  For a coarse plane
// pitch (the field kernel's rule) every plane carries its own A_k, B_k and
// m_k instead.  With s = ca + cb and D = cb - ca of the clamped ends, A' =
// H^ - s^2/4 - D^2/12:
//
//   I / R        = D Q,            Q = A'^2 + D^2 (s^2/12 + D^2/180)
//   phi(alpha)   = (H^ - ca^2)^2,  phi(beta) = (H^ - cb^2)^2
//   J R          = 2 D A'          (the H-derivative of the integral; the
//                                   clamped ends add nothing, the integrand
//                                   vanishes there)
//
// and the two ends' weights of q_perp, K_b = K and K_a = K + 2 J L:
//
//   K_b = phi(beta) - phi(alpha) + 4 alpha^ D A'
//   K_a = phi(beta) - phi(alpha) + 4 beta^ D A'
//   dI/db = phi(beta) u + (K_b / L) q_perp,  dI/da = -phi(alpha) u - (K_a / L) q_perp
//
// (summing K and J apart would cancel in K / L + 2 J for pixels near one end
// of a strut much longer than its support).  K and phi are dimensionless;
// the loop keeps 16 D Q and 4 D A', and takes out the power of two before
// the wave sums.  The q_perp weights
// follow from q_perp = m_k - d + (d.u) u with m_k = m_r + (k - r) dm: each
// lane keeps, per (strut, region), sum G K, sum (k - r) G K, and sum G K
// over its right-hand and lower sub-blocks (whose d is 8 dx, 8 dy larger),
// for K_b and K_a, and forms the three components once before the wave sums.
// The partials are then (sum G I / R, sum G phi(alpha), sum G phi(beta), sum
// G K_b q_perp, sum G K_a q_perp): k_reduce scales them by R and 1/L.
//
// The rounding of H^ grows with |d| / R (its pieces 2 m^.d^ and |d^|^2 grow
// while H^ <= 1), so the 16x16 regions are used only while their farthest
// pixel, 7.5 |(dx, dy)| from the centre, stays within the smallest support;
// otherwise d is measured from each 8x8 block's centre and H^ = 1 -
// |q_perp^|^2 is formed from q_perp^ = m_k^ - (d^ - (d.u^) u) itself, whose
// components are of the size of the support (three more operations per
// pair; for pixels coarse against the support this halves the error of the
// node gradients).
namespace b32 {

template <int SZ, bool PR, int CH>
struct Lds;
template <int SZ, int CH>
struct Lds<SZ, false, CH> {
    float pg[SZ][CH];         // per plane: G_k
    float4 gr[CH];            // A_0, B_0, 2 m_0,x / R^2, 2 m_0,y / R^2
    float4 e[CH];             // u_x / R, u_y / R, c1, 1 / R^2
    float dl[CH];             // -dz u_z / R
    float4 m0[CH];            // m_0 (x, y, z), R
    float4 u4[CH];            // u (x, y, z), dz u_z
    uint32_t mask[CH];        // reach bits: sub-block s, plane k at bit s SZ + k
    uint32_t cand[CH];        // staged lane | entry << 8 | region << 16
    float slot[CH][kParts];   // per bucket entry of the chunk
    uint8_t pairs[256];       // (entry, region) pairs: entry | region in group << log2(CH)
};
template <int SZ, int CH>
struct Lds<SZ, true, CH> {
    float4 pl[SZ][CH];        // per plane: A_k, B_k, G_k, 2 m_k,x / R^2
    float pmy[SZ][CH];        // per plane: 2 m_k,y / R^2
    float4 e[CH];
    float4 m0[CH];
    float4 u4[CH];
    float rk[CH];             // the reference plane r (window index)
    uint32_t mask[CH];
    uint32_t cand[CH];
    float slot[CH][kParts];
    uint8_t pairs[256];
};

// MODE 0: 16x16 regions, shared reference planes; 1: 16x16 regions, every
// plane its own reference; 2: 8x8 regions, every plane its own reference
// and H^ = 1 - |q_perp^|^2 formed from q_perp itself (coarse pixels against
// the support: the pieces of H^ above would be large).  Every plane its own
// reference with 8-plane windows holds 16.6 KB of LDS per wave, so at most 9
// waves fit a compute unit: that mode asks for three waves per SIMD (up to
// 168 registers) rather than four, which it could not reach.
template <int SZ, bool SR, int MODE>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(MODE == 1 && SZ == 8 ? 3 : 4))) void k_backward32(
    BackArgs a, uint32_t n_items) {
    constexpr int NS = MODE == 2 ? 1 : 2;     // sub-blocks per region side
    constexpr bool PR = MODE != 0;            // per-plane values in LDS
    constexpr bool QD = MODE == 2;            // H^ from q_perp
    constexpr int kSub = NS * NS;             // 8x8 sub-blocks of a region
    constexpr int kEdge = 8 * NS;             // region edge in pixels
    // bucket entries staged at a time: the per-plane values of 8x8 regions
    // take 32 entries, which keeps the LDS of four waves per SIMD
    constexpr int kCh = MODE == 2 ? 32 : kWave;
    __shared__ Lds<SZ, PR, kCh> L;
    const int lane = lane_id();
    const uint32_t item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= n_items) return;
    uint32_t t = item;
    const int tx = (int)(t % (uint32_t)a.ntx);
    t /= (uint32_t)a.ntx;
    const int ty = (int)(t % (uint32_t)a.nty);
    t /= (uint32_t)a.nty;
    const int slab = a.s_lo + (int)t;
    int kb = slab * a.slab, ke = kb + a.slab;
    if (kb < a.k0) kb = a.k0;
    if (ke > a.k0 + a.nk) ke = a.k0 + a.nk;
    const uint32_t bucket = ((uint32_t)(slab - a.group_s0) * (uint32_t)a.nty + (uint32_t)ty) *
                                (uint32_t)a.ntx + (uint32_t)tx;
    uint32_t beg = a.offsets[bucket], end = a.offsets[bucket + 1];
    if (end > a.n_pairs) end = a.n_pairs;
    if (beg >= end) return;

    const int lx = lane & 7, ly = lane >> 3;
    // the lane's pixel of sub-block s = sx + NS sy lies at d = ((8 sx + lx +
    // 1/2 - kEdge/2) dx, (8 sy + ly + 1/2 - kEdge/2) dy) from the region centre
    const double dxa = ((double)lx + 0.5 - 0.5 * kEdge) * a.dx, dxb = dxa + 8.0 * a.dx;
    const double dya = ((double)ly + 0.5 - 0.5 * kEdge) * a.dy, dyb = dya + 8.0 * a.dy;
    const float Dx[2] = {(float)dxa, (float)dxb};
    const float Dy[2] = {(float)dya, (float)dyb};
    float nd2[kSub];
    for (int s = 0; s < kSub; ++s) {
        const double ex = (s % NS) ? dxb : dxa, ey = (s / NS) ? dyb : dya;
        nd2[s] = (float)(-(ex * ex + ey * ey));
    }
    const float hxf = (float)(3.5 * a.dx), hyf = (float)(3.5 * a.dy);
    const float dzf = (float)a.dz, dxf = (float)a.dx, dyf = (float)a.dy;
    const int nreg = a.tile >= kEdge ? a.tile / kEdge : 1;
    const int ti1 = (tx + 1) * a.tile < a.W ? (tx + 1) * a.tile : a.W;
    const int tj1 = (ty + 1) * a.tile < a.H ? (ty + 1) * a.tile : a.H;
    const int own = deposit_owner(lane);
    const StrutRec<float>* recs = (const StrutRec<float>*)a.rec;
    const float* grad = (const float*)a.grad;
    float* part = (float*)a.partial;

    const bool st_ok = lane < kCh;            // the lane stages an entry
    // regions whose (region, entry) pairs are compacted together, and the
    // bits of an entry index in a pair
    constexpr int kGrp = 256 / kCh;
    constexpr int kEntBits = kCh == 64 ? 6 : 5;
    const int nrg = nreg * nreg;
    // half extents of a region's pixel centres
    const double hxr = 0.5 * (kEdge - 1) * fabs(a.dx), hyr = 0.5 * (kEdge - 1) * fabs(a.dy);
    for (uint32_t cbase = beg; cbase < end; cbase += kCh) {
        const int nent = (int)((end - cbase) < (uint32_t)kCh ? (end - cbase) : (uint32_t)kCh);
        for (int q = lane; q < kCh * kParts; q += kWave) (&L.slot[0][0])[q] = 0.0f;
        const uint32_t idx = cbase + (uint32_t)lane;
        bool valid = st_ok && idx < end;
        const uint32_t pid = valid ? a.ids[idx] : 0u;
        valid = valid && pid < a.n_binned;
        const uint32_t p = valid ? pid : 0u;

        for (int w0 = kb; w0 < ke; w0 += SZ) {
            const int nw = ke - w0 < SZ ? ke - w0 : SZ;
            // the window's plane centres: mid-plane and half extent
            const double czm = a.z0 + ((double)w0 + 0.5 * (double)nw) * a.dz;
            const double hzr = 0.5 * (double)(nw - 1) * fabs(a.dz);
            const double hd = sqrt(fma(hxr, hxr, fma(hyr, hyr, hzr * hzr)));
            for (int g0 = 0; g0 < nrg; g0 += kGrp) {
                const int ng = nrg - g0 < kGrp ? nrg - g0 : kGrp;
                // ------------------------------------- region pre-test
                // bit q: some pixel centre of region g0 + q, on some plane of
                // the window, may lie within the support of the entry's
                // segment.  Every pixel centre lies within hd of the
                // region's box centre c, so none does when dist(c, segment)
                // >= R (1 + 1e-4) + hd (the margin keeps every pair whose
                // float32 terms could be nonzero).
                uint32_t near = 0u;
                if (valid) {
                    const StrutRec<float> r = recs[p];
                    const double4 ln = a.line[p];
                    const double Rs = SR ? (double)r.pad : a.R;
                    const double thr = fma(Rs, 1.0 + 1e-4, hd), thr2 = thr * thr;
                    const double wz = czm - (double)r.az;
                    for (int q = 0; q < ng; ++q) {
                        const int rg = g0 + q;
                        const int i0 = tx * a.tile + (rg % nreg) * kEdge;
                        const int j0 = ty * a.tile + (rg / nreg) * kEdge;
                        if (i0 >= ti1 || j0 >= tj1) continue;
                        const double wx = a.x0 + ((double)i0 + 0.5 * kEdge) * a.dx - (double)r.ax;
                        const double wy = a.y0 + ((double)j0 + 0.5 * kEdge) * a.dy - (double)r.ay;
                        double tt = fma(wx, ln.x, fma(wy, ln.y, wz * ln.z));
                        tt = tt < 0.0 ? 0.0 : (tt > ln.w ? ln.w : tt);
                        const double ex = fma(-tt, ln.x, wx), ey = fma(-tt, ln.y, wy),
                                     ez = fma(-tt, ln.z, wz);
                        if (fma(ex, ex, fma(ey, ey, ez * ez)) < thr2) near |= 1u << q;
                    }
                }
                // (entry, region) pairs, region-major and in entry order
                // within a region, so every entry's slot receives its
                // regions' sums in region order
                int npair = 0;
                for (int q = 0; q < ng; ++q) {
                    const bool on = (near >> q) & 1u;
                    const uint64_t bm = ballot64(on);
                    if (on) {
                        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
                        L.pairs[npair + (int)rank] = (uint8_t)((uint32_t)lane | ((uint32_t)q << kEntBits));
                    }
                    npair += __popcll(bm);
                }
                __builtin_amdgcn_wave_barrier();

                for (int pb = 0; pb < npair; pb += kCh) {
                    // this lane stages pair pb + lane
                    const bool has = st_ok && pb + lane < npair;
                    const uint32_t pr8 = has ? (uint32_t)L.pairs[pb + lane] : 0u;
                    const uint32_t ent = pr8 & (uint32_t)(kCh - 1);
                    const int rgl = g0 + (int)(pr8 >> kEntBits);
                    const uint32_t ps = has ? a.ids[cbase + ent] : 0u;
                    const int i0 = tx * a.tile + (rgl % nreg) * kEdge;
                    const int j0 = ty * a.tile + (rgl / nreg) * kEdge;
                    uint32_t sub_ok = 0u;
                    for (int s = 0; s < kSub; ++s)
                        if (i0 + 8 * (s % NS) < ti1 && j0 + 8 * (s / NS) < tj1) sub_ok |= 1u << s;
                    const double cx = a.x0 + ((double)i0 + 0.5 * kEdge) * a.dx;
                    const double cy = a.y0 + ((double)j0 + 0.5 * kEdge) * a.dy;
                    // ------------------------------------------------ staging
                    int n_cand = 0;
                    {
                        // read the entry afresh for every pass: what follows from
                        // it would otherwise stay in registers through the
                        // evaluation
                        uint32_t pr = ps;
                        asm volatile("" : "+v"(pr));
                        const StrutRec<float> r = recs[pr];
                        const double4 ln = a.line[pr];
                        const double Rs = SR ? (double)r.pad : a.R;
                        const double iR = 1.0 / Rs, iR2 = iR * iR;
                        const float Rc2f = (float)(Rs * Rs * (1.0 + 2e-5));
                        const double wx = cx - (double)r.ax, wy = cy - (double)r.ay;
                        const double txy = fma(wx, ln.x, wy * ln.y);
                        const double wz = a.z0 + ((double)w0 + 0.5) * a.dz - (double)r.az;
                        const double tc0 = fma(wz, ln.z, txy);
                        const double mx = fma(tc0, ln.x, -wx), my = fma(tc0, ln.y, -wy),
                                     mz = fma(tc0, ln.z, -wz);
                        const double m20 = fma(mx, mx, fma(my, my, mz * mz));
                        const double dzuz = a.dz * ln.z;
                        // m_k = m_0 + k dz (u_z u - e_z) is orthogonal to u:
                        // |m_k|^2 = |m_0|^2 - 2 k dz m_0,z + k^2 dz^2 (1 - u_z^2)
                        const double c1d = -2.0 * a.dz * mz, c2 = a.dz * a.dz * (1.0 - ln.z * ln.z);
                        // sub-block centres c + delta_s: the foot moves by
                        // delta.u along u, the offset m by (delta.u) u - delta
                        float dus[kSub], cxs[kSub], cys[kSub], css[kSub], tdx[kSub], tdy[kSub];
                        for (int s = 0; s < kSub; ++s) {
                            const double ddx = (8.0 * (s % NS) + 4.0 - 0.5 * kEdge) * a.dx;
                            const double ddy = (8.0 * (s / NS) + 4.0 - 0.5 * kEdge) * a.dy;
                            const double du = fma(ddx, ln.x, ddy * ln.y);
                            dus[s] = (float)du;
                            cxs[s] = (float)fma(du, ln.x, -ddx);
                            cys[s] = (float)fma(du, ln.y, -ddy);
                            css[s] = (float)(ddx * ddx + ddy * ddy - du * du);
                            tdx[s] = (float)(-2.0 * ddx);
                            tdy[s] = (float)(-2.0 * ddy);
                        }
                        const float uxf = (float)ln.x, uyf = (float)ln.y, Lf = (float)ln.w;
                        const float mxf0 = (float)mx, myf0 = (float)my;
                        const float vxf = (float)(dzuz * ln.x), vyf = (float)(dzuz * ln.y);
                        uint32_t mask = 0u;
    #pragma unroll 1
                        for (int k = 0; k < nw; ++k) {
                            const double kd = (double)k;
                            const double tc = fma(kd, dzuz, tc0);
                            const double m2 = fma(kd * kd, c2, fma(kd, c1d, m20));
                            const float tcf = (float)tc, m2f = (float)m2, kf = (float)k;
                            const float mxf = __builtin_fmaf(kf, vxf, mxf0);
                            const float myf = __builtin_fmaf(kf, vyf, myf0);
                            uint32_t bits = 0u;
    #pragma unroll
                            for (int s = 0; s < kSub; ++s) {
                                // e = F* - c_s, F* the segment's point nearest to
                                // the sub-block centre; no pixel of the sub-block
                                // is within R when D^2 - hx |e_x| - hy |e_y| >= R D
                                const float tcs = tcf + dus[s];
                                const float dt = __builtin_amdgcn_fmed3f(tcs, 0.0f, Lf) - tcs;
                                const float ex = __builtin_fmaf(dt, uxf, mxf + cxs[s]);
                                const float ey = __builtin_fmaf(dt, uyf, myf + cys[s]);
                                const float m2s =
                                    __builtin_fmaf(tdx[s], mxf, __builtin_fmaf(tdy[s], myf, m2f + css[s]));
                                const float D2 = __builtin_fmaf(dt, dt, m2s);
                                const float q = D2 - __builtin_fmaf(hxf, fabsf(ex), hyf * fabsf(ey));
                                const uint32_t pass =
                                    ((sub_ok >> s) & 1u) &
                                    ((uint32_t)(q <= 0.0f) | (uint32_t)(q * q < Rc2f * D2));
                                bits |= pass << (s * SZ);
                            }
                            mask |= bits << k;
                            if constexpr (QD) {
                                // m_k / R
                                const double mxk = fma(kd, dzuz * ln.x, mx), myk = fma(kd, dzuz * ln.y, my),
                                             mzk = fma(kd, fma(dzuz, ln.z, -a.dz), mz);
                                if (st_ok) L.pl[k][lane] = make_float4((float)(-tc * iR), (float)((ln.w - tc) * iR),
                                                            (float)(mxk * iR), (float)(myk * iR));
                                if (st_ok) L.pmy[k][lane] = (float)(mzk * iR);
                            } else if constexpr (PR) {
                                const double mxk = fma(kd, dzuz * ln.x, mx), myk = fma(kd, dzuz * ln.y, my);
                                if (st_ok) L.pl[k][lane] = make_float4((float)(-tc * iR), (float)((ln.w - tc) * iR),
                                                            (float)fma(-m2, iR2, 1.0), (float)(2.0 * mxk * iR2));
                                if (st_ok) L.pmy[k][lane] = (float)(2.0 * myk * iR2);
                            } else {
                                if (st_ok) L.pg[k][lane] = (float)fma(-m2, iR2, 1.0);
                            }
                        }
                        if (!has) mask = 0u;
                        if (st_ok) L.mask[lane] = mask;
                        // the reference plane r: the middle of the planes the
                        // strut reaches, so that the shifts k - r and the offsets
                        // m_r stay small (m_k = m_r + (k - r) dm, dm = dz (u_z u -
                        // e_z), grows without bound along a steep strut)
                        uint32_t pm = 0u;
                        for (int s = 0; s < kSub; ++s) pm |= (mask >> (s * SZ)) & ((1u << SZ) - 1u);
                        // (shared reference planes: the window's first plane, as
                        // fine planes keep (k - r) dz small against R)
                        const int rr = (MODE != 0 && pm) ? (__builtin_ctz(pm) + 31 - __builtin_clz(pm)) >> 1 : 0;
                        const double rd = (double)rr;
                        const double tcr = fma(rd, dzuz, tc0);
                        const double mxr = fma(rd, dzuz * ln.x, mx), myr = fma(rd, dzuz * ln.y, my),
                                     mzr = fma(rd, fma(dzuz, ln.z, -a.dz), mz);
                        if constexpr (PR) {
                            if (st_ok) L.rk[lane] = (float)rr;
                        }
                        if (st_ok) L.e[lane] = make_float4((float)(ln.x * iR), (float)(ln.y * iR),
                                                (float)(2.0 * dzuz * iR), (float)(QD ? iR : iR2));
                        if constexpr (!PR) {
                            if (st_ok) L.dl[lane] = (float)(-dzuz * iR);
                            if (st_ok) L.gr[lane] = make_float4((float)(-tcr * iR), (float)((ln.w - tcr) * iR),
                                                     (float)(2.0 * mxr * iR2), (float)(2.0 * myr * iR2));
                        }
                        if (st_ok) L.m0[lane] = make_float4((float)mxr, (float)myr, (float)mzr, (float)Rs);
                        if (st_ok) L.u4[lane] = make_float4(uxf, uyf, (float)ln.z, (float)dzuz);
                        const uint64_t cm = ballot64(mask != 0u);
                        if (mask != 0u) {
                            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(cm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
                            L.cand[rank] = (uint32_t)lane | (ent << 8) | ((uint32_t)rgl << 16);
                        }
                        n_cand = __popcll(cm);
                    }
                    __builtin_amdgcn_wave_barrier();
                    const int n = n_cand;

                    // --------------------------------------------- evaluation
                    // dL/dg at the lane's pixels of the candidate's region, loaded
                    // when the region changes
                    float Gv[kSub][SZ];
                    int cur = -1;
    #pragma unroll 1
                    for (int j = 0; j < n; ++j) {
                        const uint32_t c = __builtin_amdgcn_readfirstlane(L.cand[j]);
                        const uint32_t e = c & 0xffu;
                        const int crg = (int)(c >> 16);
                        if (crg != cur) {
                            cur = crg;
                            const int ri = tx * a.tile + (crg % nreg) * kEdge;
                            const int rj = ty * a.tile + (crg / nreg) * kEdge;
                            q32::for_planes<0, kSub>([&](auto sc) {
                                constexpr int s = decltype(sc)::value;
                                const int pi = ri + 8 * (s % NS) + lx, pj = rj + 8 * (s / NS) + ly;
                                const bool pix = pi < ti1 && pj < tj1;
                                q32::for_planes<0, SZ>([&](auto kc) {
                                    constexpr int k = decltype(kc)::value;
                                    Gv[s][k] = (pix && k < nw)
                                                   ? grad[((size_t)(w0 + k - a.k0) * (size_t)a.H + (size_t)pj) *
                                                              (size_t)a.W + (size_t)pi]
                                                   : 0.0f;
                                });
                            });
                        }
                        const uint32_t mask = __builtin_amdgcn_readfirstlane(L.mask[e]);
                        const float4 E = L.e[e];
                        const float4 U = L.u4[e];
                        float rf = 0.0f;
                        if constexpr (PR) rf = L.rk[e];
                        float nD = 0.0f;
                        float4 Rg = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                        float Gk[SZ];
                        if constexpr (!PR) {
                            nD = L.dl[e];
                            Rg = L.gr[e];
                            q32::for_planes<0, SZ>([&](auto kc) {
                                constexpr int k = decltype(kc)::value;
                                Gk[k] = L.pg[k][e];
                            });
                        }
                        // per lane: sum G I, G phi(alpha), G phi(beta); sum G K, sum
                        // (k - r) G K and sum G K over the right-hand (sx = 1) and
                        // lower (sy = 1) sub-blocks, whose pixels lie 8 dx, 8 dy
                        // further (likewise for J)
                        float Aw = 0.0f, Aa = 0.0f, Ab = 0.0f, ABk = 0.0f, AAk = 0.0f;
                        float Bs[kSub], As[kSub];                 // per sub-block
                        q32::for_planes<0, kSub>([&](auto sc) {
                            constexpr int s = decltype(sc)::value;
                            Bs[s] = As[s] = 0.0f;
                        });
                        const float du0 = __builtin_fmaf(Dx[0], E.x, Dy[0] * E.y);
                        const float e8x = NS == 2 ? 8.0f * dxf * E.x : 0.0f;
                        const float e8y = NS == 2 ? 8.0f * dyf * E.y : 0.0f;
                        q32::for_planes<0, kSub>([&](auto sc) {
                            constexpr int s = decltype(sc)::value;
                            const uint32_t ms = (mask >> (s * SZ)) & ((1u << SZ) - 1u);
                            if (ms == 0u) return;
                            // one plane's values at a time (not all planes kept
                            // in registers across the four sub-blocks)
                            uint32_t es = e;
                            if constexpr (PR) asm volatile("" : "+v"(es));
                            const float dX = Dx[s % NS], dY = Dy[s / NS];
                            // d.u^ (d of sub-block (sx, sy) = d_00 + 8 (sx dx, sy dy))
                            float du = du0;
                            if constexpr (s % NS != 0) du += e8x;
                            if constexpr (s / NS != 0) du += e8y;
                            float ndd = 0.0f, vx = 0.0f, vy = 0.0f, vz = 0.0f;
                            if constexpr (QD) {
                                // q_perp^ = m_k^ - v, v = d^ - (d.u^) u
                                vx = __builtin_fmaf(-du, U.x, dX * E.w);
                                vy = __builtin_fmaf(-du, U.y, dY * E.w);
                                vz = -du * U.z;
                            } else {
                                ndd = nd2[s] * E.w;                                  // -|d^|^2
                            }
                            float ar = 0.0f, br = 0.0f, Eg = 0.0f, P1 = 0.0f;
                            if constexpr (!PR) {
                                ar = Rg.x - du;
                                br = Rg.y - du;
                                Eg = __builtin_fmaf(du, du,
                                                    __builtin_fmaf(Rg.z, dX, __builtin_fmaf(Rg.w, dY, ndd)));
                                P1 = E.z * du;
                            }
                            q32::for_planes<0, SZ>([&](auto kc) {
                                constexpr int k = decltype(kc)::value;
                                if (!((ms >> k) & 1u)) return;
                                // k - r (r = 0 with shared reference planes)
                                const float kap = MODE == 0 ? (float)k : (float)k - rf;
                                float al, be, Hp;
                                if constexpr (QD) {
                                    const float4 P = L.pl[k][es];
                                    const float qz = L.pmy[k][es] - vz;
                                    const float qx = P.z - vx, qy = P.w - vy;
                                    al = P.x - du;
                                    be = P.y - du;
                                    Hp = 1.0f - __builtin_fmaf(qx, qx, __builtin_fmaf(qy, qy, qz * qz));
                                } else if constexpr (PR) {
                                    const float4 P = L.pl[k][es];
                                    const float my2 = L.pmy[k][es];
                                    al = P.x - du;
                                    be = P.y - du;
                                    Hp = __builtin_fmaf(du, du,
                                                        __builtin_fmaf(P.w, dX, __builtin_fmaf(my2, dY, ndd + P.z)));
                                } else if constexpr (k == 0) {
                                    al = ar;
                                    be = br;
                                    Hp = Gk[0] + Eg;
                                } else {
                                    al = __builtin_fmaf(kap, nD, ar);
                                    be = __builtin_fmaf(kap, nD, br);
                                    Hp = __builtin_fmaf(kap, P1, Gk[k] + Eg);
                                }
                                const float H = __builtin_amdgcn_fmed3f(Hp, 0.0f, 1.0f);
                                const float h = __builtin_amdgcn_sqrtf(H);
                                const float ca = __builtin_amdgcn_fmed3f(al, -h, h);
                                const float cb = __builtin_amdgcn_fmed3f(be, -h, h);
                                const float sm = ca + cb, D = cb - ca;
                                const float s2 = sm * sm, D2 = D * D;
                                const float A4 = __builtin_fmaf(D2, -1.0f / 3.0f, __builtin_fmaf(H, 4.0f, -s2));
                                const float V16 = __builtin_fmaf(s2, 4.0f / 3.0f, D2 * (4.0f / 45.0f));
                                const float Q16 = __builtin_fmaf(A4, A4, D2 * V16);
                                const float g = Gv[s][k];
                                const float gD = g * D;
                                Aw = __builtin_fmaf(gD, Q16, Aw);
                                const float Jq = gD * A4;                    // 2 G J R
                                const float xa = __builtin_fmaf(-ca, ca, H), xb = __builtin_fmaf(-cb, cb, H);
                                const float pa = xa * xa, pb = xb * xb;
                                Aa = __builtin_fmaf(g, pa, Aa);
                                Ab = __builtin_fmaf(g, pb, Ab);
                                const float gd = g * (pb - pa);
                                // (shared reference planes, fine pixels: J itself
                                // instead of K_a, one operation less)
                                const float gKb = __builtin_fmaf(al, Jq, gd);
                                const float gKa = MODE == 0 ? Jq : __builtin_fmaf(be, Jq, gd);
                                Bs[s] += gKb;
                                As[s] += gKa;
                                if (MODE != 0 || k != 0) {
                                    ABk = __builtin_fmaf(kap, gKb, ABk);
                                    AAk = __builtin_fmaf(kap, gKa, AAk);
                                }
                            });
                        });
                        // over all sub-blocks, the right-hand ones and the lower ones
                        const float4 M = L.m0[e];
                        const float dmx = U.w * U.x, dmy = U.w * U.y, dmz = __builtin_fmaf(U.w, U.z, -dzf);
                        const float rux = M.w * U.x, ruy = M.w * U.y, ruz = M.w * U.z;
                        // sum G K q_perp = m_r sum G K + dm sum (k - r) G K - sum G K d
                        // + R u sum G K (d.u^), dm = dz u_z u - dz e_z, for K_b and K_a
                        float v[kParts];
                        v[0] = Aw * (1.0f / 16.0f);
                        v[1] = Aa;
                        v[2] = Ab;
                        if constexpr (NS == 2) {
                            // over all sub-blocks, the right-hand and the lower ones
                            // (d of sub-block (sx, sy) = d_00 + 8 (sx dx, sy dy))
                            const float SXB = Bs[1] + Bs[3], SXA = As[1] + As[3];
                            const float SYB = Bs[2] + Bs[3], SYA = As[2] + As[3];
                            const float AB = (Bs[0] + Bs[2]) + SXB, AA = (As[0] + As[2]) + SXA;
                            const float ABx = __builtin_fmaf(8.0f * dxf, SXB, Dx[0] * AB);
                            const float ABy = __builtin_fmaf(8.0f * dyf, SYB, Dy[0] * AB);
                            const float ABu = __builtin_fmaf(e8x, SXB, __builtin_fmaf(e8y, SYB, du0 * AB));
                            const float AAx = __builtin_fmaf(8.0f * dxf, SXA, Dx[0] * AA);
                            const float AAy = __builtin_fmaf(8.0f * dyf, SYA, Dy[0] * AA);
                            const float AAu = __builtin_fmaf(e8x, SXA, __builtin_fmaf(e8y, SYA, du0 * AA));
                            v[3] = __builtin_fmaf(M.x, AB, __builtin_fmaf(dmx, ABk, __builtin_fmaf(rux, ABu, -ABx)));
                            v[4] = __builtin_fmaf(M.y, AB, __builtin_fmaf(dmy, ABk, __builtin_fmaf(ruy, ABu, -ABy)));
                            v[5] = __builtin_fmaf(M.z, AB, __builtin_fmaf(dmz, ABk, ruz * ABu));
                            v[6] = __builtin_fmaf(M.x, AA, __builtin_fmaf(dmx, AAk, __builtin_fmaf(rux, AAu, -AAx)));
                            v[7] = __builtin_fmaf(M.y, AA, __builtin_fmaf(dmy, AAk, __builtin_fmaf(ruy, AAu, -AAy)));
                            v[8] = __builtin_fmaf(M.z, AA, __builtin_fmaf(dmz, AAk, ruz * AAu));
                        } else {
                            // one sub-block: the lane's q_perp at plane r, m_r - d + (d.u) u,
                            // weights both ends' sums
                            const float qx = __builtin_fmaf(rux, du0, M.x - Dx[0]);
                            const float qy = __builtin_fmaf(ruy, du0, M.y - Dy[0]);
                            const float qz = __builtin_fmaf(ruz, du0, M.z);
                            v[3] = __builtin_fmaf(qx, Bs[0], dmx * ABk);
                            v[4] = __builtin_fmaf(qy, Bs[0], dmy * ABk);
                            v[5] = __builtin_fmaf(qz, Bs[0], dmz * ABk);
                            v[6] = __builtin_fmaf(qx, As[0], dmx * AAk);
                            v[7] = __builtin_fmaf(qy, As[0], dmy * AAk);
                            v[8] = __builtin_fmaf(qz, As[0], dmz * AAk);
                        }
                        if constexpr (MODE == 0) {
                            // K_a = K_b + 2 J L: the second sums carried J
                            const float Lh = Rg.y - Rg.x;
                            v[6] = __builtin_fmaf(Lh, v[6], v[3]);
                            v[7] = __builtin_fmaf(Lh, v[7], v[4]);
                            v[8] = __builtin_fmaf(Lh, v[8], v[5]);
                        }
                        deposit(L.slot[(c >> 8) & 0xffu], v, lane, own);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        // each entry's sums go to its emission index
        for (int q = lane; q < nent * kParts; q += kWave) {
            const uint32_t e = a.emi[cbase + (uint32_t)(q / kParts)];
            if (e < a.n_pairs) part[(size_t)e * kParts + (size_t)(q % kParts)] = (&L.slot[0][0])[q];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int SZ, bool SR>
void launch_sz(const BackArgs& a, uint32_t n_items, hipStream_t st) {
    if (!a.wide)
        k_backward32<SZ, SR, 2><<<n_items, 64, 0, st>>>(a, n_items);
    else if (a.plane_ref)
        k_backward32<SZ, SR, 1><<<n_items, 64, 0, st>>>(a, n_items);
    else
        k_backward32<SZ, SR, 0><<<n_items, 64, 0, st>>>(a, n_items);
}

template <int SZ>
void launch_sr(const BackArgs& a, uint32_t n_items, hipStream_t st) {
    if (a.strut_R)
        launch_sz<SZ, true>(a, n_items, st);
    else
        launch_sz<SZ, false>(a, n_items, st);
}

lsl_status launch(const BackArgs& a, uint32_t n_items, hipStream_t st) {
    if (a.slab <= 1)
        launch_sr<1>(a, n_items, st);
    else if (a.slab <= 2)
        launch_sr<2>(a, n_items, st);
    else if (a.slab <= 4)
        launch_sr<4>(a, n_items, st);
    else
        launch_sr<8>(a, n_items, st);      // longer slabs: windows of 8 planes
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace b32

// Per active strut: sum its pairs of the slabs [s_lo, s_hi] in emission
// order, then form the strut's gradient and add it to acc (float64).
template <typename T>
__global__ void k_reduce(ReduceArgs a, const SRange* ranges, int32_t sa, int32_t s_lo,
                         int32_t s_hi, uint32_t n_pairs, uint32_t n_binned) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_active) return;
    const uint32_t p = a.active[i];
    if (p >= n_binned) return;
    const SRange rg = ranges[p];
    const int32_t s0 = rg.s0 > sa ? rg.s0 : sa;
    const uint32_t nxy = (uint32_t)(rg.tx1 - rg.tx0 + 1) * (uint32_t)(rg.ty1 - rg.ty0 + 1);
    const int32_t lo = s_lo > s0 ? s_lo : s0;
    const int32_t hi = s_hi < rg.s1 ? s_hi : rg.s1;
    if (hi < lo) return;
    const uint32_t e0 = a.eoff[i] + (uint32_t)(lo - s0) * nxy;
    uint32_t e1 = a.eoff[i] + (uint32_t)(hi - s0 + 1) * nxy;
    double s[kParts];
    for (int q = 0; q < kParts; ++q) s[q] = 0.0;
    const T* part = (const T*)a.partial;
    if (e1 > n_pairs) e1 = n_pairs;
    for (uint32_t e = e0; e < e1; ++e)
        for (int q = 0; q < kParts; ++q) s[q] += (double)part[(size_t)e * kParts + q];
    const StrutRec<T> r = ((const StrutRec<T>*)a.rec)[p];
    const double w = (double)((const T*)a.w)[p];
    const double Rs = a.strut_R ? (double)r.pad : a.R;
    const double R4 = Rs * Rs * Rs * Rs;
    const Line ln = strut_line(r);
    const double u[3] = {ln.ux, ln.uy, ln.uz};
    double* acc = a.acc + (size_t)p * 7;
    if (a.normalized) {
        // partials in units of R: sum G I / R; phi and the end weights K_b,
        // K_a dimensionless
        acc[0] += s[0] * Rs;
        for (int c = 0; c < 3; ++c) {
            acc[1 + c] -= w * (s[1] * u[c] + s[6 + c] / ln.L);   // dL/da
            acc[4 + c] += w * (s[2] * u[c] + s[3 + c] / ln.L);   // dL/db
        }
        return;
    }
    const double cw = w / R4;
    acc[0] += s[0] / R4;
    for (int c = 0; c < 3; ++c) {
        const double kq = s[3 + c] / ln.L;
        acc[1 + c] -= cw * (s[1] * u[c] + kq + 2.0 * s[6 + c]);     // dL/da
        acc[4 + c] += cw * (s[2] * u[c] + kq);                       // dL/db
    }
}

__global__ void k_node_keys(const int2* ends, int64_t n, uint32_t* keys, uint32_t* vals) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int2 e = ends[p];
    keys[2 * p] = (uint32_t)e.x;
    vals[2 * p] = (uint32_t)(2 * p);
    keys[2 * p + 1] = (uint32_t)e.y;
    vals[2 * p + 1] = (uint32_t)(2 * p + 1);
}

__global__ void k_node_offsets(const uint32_t* keys, uint32_t n, uint32_t n_nodes,
                               uint32_t* off) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const uint32_t kprev = i == 0 ? 0u : keys[i - 1] + 1u;
    const uint32_t k = i == n ? n_nodes : keys[i];
    for (uint32_t b = kprev; b <= k && b <= n_nodes; ++b) off[b] = i;
}

template <typename T>
__global__ void k_scatter_weight(ScatterArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_binned) return;
    T* gw = (T*)a.grad_weight;
    const uint32_t e = a.perm[p];
    const T v = (T)a.acc[(size_t)p * 7];
    gw[e] = a.accumulate ? gw[e] + v : v;
}

template <typename T>
__global__ void k_scatter_nodes(ScatterArgs a) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.n_nodes) return;
    double g[3] = {0.0, 0.0, 0.0};
    const uint32_t i0 = a.node_off[n], i1 = a.node_off[n + 1];
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t inc = a.node_inc[i];
        const uint32_t p = inc >> 1, end = inc & 1u;
        if ((int64_t)p >= a.n_binned) continue;
        const double* s = a.acc + (size_t)p * 7 + 1 + 3 * end;
        g[0] += s[0];
        g[1] += s[1];
        g[2] += s[2];
    }
    T* gn = (T*)a.grad_nodes + (size_t)n * 3;
    for (int c = 0; c < 3; ++c) gn[c] = a.accumulate ? gn[c] + (T)g[c] : (T)g[c];
}

template <typename T>
__global__ void k_fill_t(T* p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <typename T, int SZ>
lsl_status launch_b(const BackArgs& a, uint32_t n_items, hipStream_t st) {
    if (a.strut_R)
        k_backward<T, SZ, true><<<n_items, 64, 0, st>>>(a, n_items);
    else
        k_backward<T, SZ, false><<<n_items, 64, 0, st>>>(a, n_items);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

template <typename T>
lsl_status launch_bt(const BackArgs& a, uint32_t n_items, hipStream_t st) {
    if (a.slab <= 1) return launch_b<T, 1>(a, n_items, st);
    if (a.slab <= 2) return launch_b<T, 2>(a, n_items, st);
    if (a.slab <= 4) return launch_b<T, 4>(a, n_items, st);
    if (a.slab <= 8) return launch_b<T, 8>(a, n_items, st);
    return launch_b<T, 16>(a, n_items, st);
}

}  // namespace

lsl_status launch_backward(int dtype, const BackArgs& a, hipStream_t st) {
    const uint64_t n_items = (uint64_t)(a.s_hi - a.s_lo + 1) * (uint64_t)a.ntx * (uint64_t)a.nty;
    if (n_items == 0 || a.nk <= 0) return LSL_OK;
    if (n_items > 0x7fffffffull) {
        set_error("slice_field_backward: too many work items in one launch");
        return LSL_EINTERNAL;
    }
    if (dtype == LSL_F32) return b32::launch(a, (uint32_t)n_items, st);
    return launch_bt<double>(a, (uint32_t)n_items, st);
}

lsl_status launch_reduce(int dtype, const ReduceArgs& a, const SRange* ranges, int32_t sa,
                         int32_t s_lo, int32_t s_hi, uint32_t n_pairs, uint32_t n_binned,
                         hipStream_t st) {
    if (a.n_active == 0) return LSL_OK;
    const unsigned g = (a.n_active + 255) / 256;
    if (dtype == LSL_F32)
        k_reduce<float><<<g, 256, 0, st>>>(a, ranges, sa, s_lo, s_hi, n_pairs, n_binned);
    else
        k_reduce<double><<<g, 256, 0, st>>>(a, ranges, sa, s_lo, s_hi, n_pairs, n_binned);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_node_keys(const int2* ends, int64_t n_binned, uint32_t* keys, uint32_t* vals,
                            hipStream_t st) {
    if (n_binned == 0) return LSL_OK;
    k_node_keys<<<(unsigned)((n_binned + 255) / 256), 256, 0, st>>>(ends, n_binned, keys, vals);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_node_offsets(const uint32_t* sorted_keys, size_t n, int64_t n_nodes,
                               uint32_t* node_off, hipStream_t st) {
    k_node_offsets<<<(unsigned)((n + 1 + 255) / 256), 256, 0, st>>>(sorted_keys, (uint32_t)n,
                                                                    (uint32_t)n_nodes, node_off);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_scatter(int dtype, const ScatterArgs& a, hipStream_t st) {
    const size_t es = dtype == LSL_F64 ? 8 : 4;
    if (a.grad_weight) {
        if (!a.accumulate && a.n_edges > 0) {
            if (dtype == LSL_F32)
                k_fill_t<float><<<(unsigned)((a.n_edges + 255) / 256), 256, 0, st>>>(
                    (float*)a.grad_weight, (size_t)a.n_edges);
            else
                k_fill_t<double><<<(unsigned)((a.n_edges + 255) / 256), 256, 0, st>>>(
                    (double*)a.grad_weight, (size_t)a.n_edges);
        }
        if (a.n_binned > 0) {
            const unsigned g = (unsigned)((a.n_binned + 255) / 256);
            if (dtype == LSL_F32)
                k_scatter_weight<float><<<g, 256, 0, st>>>(a);
            else
                k_scatter_weight<double><<<g, 256, 0, st>>>(a);
        }
    }
    if (a.grad_nodes && a.n_nodes > 0) {
        const unsigned g = (unsigned)((a.n_nodes + 255) / 256);
        if (dtype == LSL_F32)
            k_scatter_nodes<float><<<g, 256, 0, st>>>(a);
        else
            k_scatter_nodes<double><<<g, 256, 0, st>>>(a);
    }
    (void)es;
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
