// Per-block field evaluation shared by the plain and the persistent field
// kernels (see field.hip for the method).
#pragma once

#include "kernels.hpp"

namespace lsl {
namespace fieldk {

template <typename T>
struct Num;

template <>
struct Num<float> {
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float clamp_(float v, float lo, float hi) {
        return __builtin_amdgcn_fmed3f(v, lo, hi);
    }
    static __device__ __forceinline__ float fma_(float a, float b, float c) {
        return __builtin_fmaf(a, b, c);
    }
    static __device__ __forceinline__ float max_(float a, float b) { return __builtin_fmaxf(a, b); }
    static __device__ __forceinline__ float erf_(float x) { return erff(x); }
    static __device__ __forceinline__ float exp_(float x) { return expf(x); }
};

template <>
struct Num<double> {
    static __device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
    static __device__ __forceinline__ double clamp_(double v, double lo, double hi) {
        return __builtin_fmin(__builtin_fmax(v, lo), hi);
    }
    static __device__ __forceinline__ double fma_(double a, double b, double c) {
        return __builtin_fma(a, b, c);
    }
    static __device__ __forceinline__ double max_(double a, double b) { return __builtin_fmax(a, b); }
    static __device__ __forceinline__ double erf_(double x) { return erf(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
};

// One (pixel, strut) term of the field.
template <typename T>
__device__ __forceinline__ T eval_term(const Stage<T>& e, T dX, T dY, T d2) {
    using N = Num<T>;
    const T du = N::fma_(dX, e.ux, dY * e.uy);                 // d.u
    const T al = e.ntc - du;                                     // alpha
    const T be = e.nbtc - du;                                    // beta
    const T H = N::fma_(du, du, N::fma_(e.mx2, dX, N::fma_(e.my2, dY, e.H0 - d2)));
    const T h = N::sqrt_(N::max_(H, T(0)));
    const T ca = N::clamp_(al, -h, h);
    const T cb = N::clamp_(be, -h, h);
    const T D = cb - ca;
    const T x2 = ca * ca, y2 = cb * cb, xy = ca * cb;
    const T q2 = x2 + y2;
    const T S1 = q2 + xy;
    const T S2 = N::fma_(q2, S1, -(xy * xy));
    const T u = N::fma_(T(-2.0 / 3.0), S1, H);
    const T Q = N::fma_(H, u, T(0.2) * S2);
    return (e.wq * D) * Q;
}

// The Gaussian variant's term: with the same H, h and clamped ends,
//   wq [exp(H k2) c0 (erf(cb k1) - erf(ca k1)) - (cb - ca)],
// wq = r exp(-R^2 k2), k1 = 1/(sigma sqrt 2), k2 = 1/(2 sigma^2),
// c0 = sigma sqrt(pi/2): exp(H k2) wq / r = exp(-dist(p, line)^2 k2).  An
// empty interval gives erf(x) - erf(x) = 0 and cb - ca = 0: an exact zero.
template <typename T>
__device__ __forceinline__ T eval_term_gauss(const Stage<T>& e, T dX, T dY, T d2, T k1, T k2,
                                             T c0) {
    using N = Num<T>;
    const T du = N::fma_(dX, e.ux, dY * e.uy);
    const T al = e.ntc - du;
    const T be = e.nbtc - du;
    const T H = N::fma_(du, du, N::fma_(e.mx2, dX, N::fma_(e.my2, dY, e.H0 - d2)));
    const T h = N::sqrt_(N::max_(H, T(0)));
    const T ca = N::clamp_(al, -h, h);
    const T cb = N::clamp_(be, -h, h);
    const T E = N::erf_(cb * k1) - N::erf_(ca * k1);
    return e.wq * N::fma_(N::exp_(H * k2) * c0, E, ca - cb);
}

template <typename T>
__device__ __forceinline__ void comp_add(T t, T& s, T& c) {
    const T sn = s + t;
    c += t - (sn - s);
    s = sn;
}

// Terms per compensated add.  float32 adds each run of four consecutive
// candidates of a (block, plane) plainly, ((t0 + t1) + t2) + t3, and
// compensates once per run; float64 compensates every term, and so does the
// Gaussian term (two erf and one exp per pair dwarf the sum, and the runs'
// extra registers would spill).  Runs are counted
// over the whole candidate sequence of the (block, plane), across the 64-entry
// chunks of the bucket list: a run left open at the end of a chunk waits in
// LDS (`pend`, [SZ][64] per wave) for the next one.
template <typename T>
struct Group {
    static constexpr int n = 1;
};
template <>
struct Group<float> {
    static constexpr int n = 4;
};
template <typename T, int SZ>
constexpr int pend_elems() {
    return Group<T>::n > 1 ? SZ * kWave : 1;
}

// Between the planes of a chunk each lane keeps six float64 values of its
// strut's line (a_z, the xy part of tc, c - a in x and y, u_x, u_y) in LDS,
// [kLineVals][64] per wave, instead of in registers across the evaluation
// loops: 12 registers fewer per lane, and with the stage and the open runs
// a workgroup of four waves stays under 32 KB of LDS (five per CU).
constexpr int kLineVals = 6;

// One wave evaluates the 8x8 block `sub` of tile (tx, ty) over the planes of
// `slab` that lie in [k0, k0+nk); `stage` is the wave's 64-entry LDS area,
// `pend` its pend_elems<T, SZ>() open-run sums and `line` its
// kLineVals * 64 line values.  K: LSL_KERNEL_QUARTIC or LSL_KERNEL_GAUSS;
// SR: per-strut supports (in the record's pad) instead of one support R.
template <typename T, int SZ, bool STATS, int K, bool SR>
__device__ __forceinline__ void field_block(const FieldArgs& a, int slab, int tx, int ty, int sub,
                                            Stage<T>* stage, T* pend, double* line) {
    constexpr int G = K == LSL_KERNEL_GAUSS ? 1 : Group<T>::n;
    const int lane = lane_id();
    const uint32_t n_binned = a.n_binned, n_pairs = a.n_pairs;
    const int nsub = a.tile / kBlockPix;
    const int i0 = tx * a.tile + (sub % nsub) * kBlockPix;
    const int j0 = ty * a.tile + (sub / nsub) * kBlockPix;
    if (i0 >= a.W || j0 >= a.H) return;
    int kb = slab * a.slab, ke = kb + a.slab;
    if (kb < a.k0) kb = a.k0;
    if (ke > a.k0 + a.nk) ke = a.k0 + a.nk;
    const int nvalid = ke - kb;

    const uint32_t bucket = ((uint32_t)(slab - a.group_s0) * (uint32_t)a.nty + (uint32_t)ty) *
                                (uint32_t)a.ntx + (uint32_t)tx;
    uint32_t beg = a.offsets[bucket], end = a.offsets[bucket + 1];
    if (end > n_pairs) end = n_pairs;
    if (beg > end) beg = end;

    const int lx = lane & 7, ly = lane >> 3;
    const int pi = i0 + lx, pj = j0 + ly;
    const bool pix = pi < a.W && pj < a.H;
    const double cx = a.x0 + ((double)i0 + 4.0) * a.dx;     // centre of the 8x8 centres
    const double cy = a.y0 + ((double)j0 + 4.0) * a.dy;
    const T dX = (T)(((double)lx - 3.5) * a.dx);
    const T dY = (T)(((double)ly - 3.5) * a.dy);
    const T d2 = dX * dX + dY * dY;
    // half extents of the block's pixel centres about c
    const double hx = 3.5 * a.dx, hy = 3.5 * a.dy;
    // one support: the (slightly widened) cull radius and R^2 are uniform
    const double Rc_u = a.R * (1.0 + 1e-7);
    const double Rc2_u = Rc_u * Rc_u;
    const double R2_u = a.R * a.R;
    const T gk1 = (T)a.gk1, gk2 = (T)a.gk2, gc0 = (T)a.gc0;

    // the block's pixel columns and rows (for the range test)
    const int ie = i0 + 7 < a.W - 1 ? i0 + 7 : a.W - 1;
    const int je = j0 + 7 < a.H - 1 ? j0 + 7 : a.H - 1;

    T acc_s[SZ], acc_c[SZ];
    int open[SZ];                       // terms in each plane's open run (wave-uniform)
#pragma unroll
    for (int k = 0; k < SZ; ++k) {
        acc_s[k] = acc_c[k] = T(0);
        open[k] = 0;
    }
    unsigned long long n_cand = 0, n_useful = 0;

    const StrutRec<T>* recs = (const StrutRec<T>*)a.rec;
    for (uint32_t cbase = beg; cbase < end; cbase += kWave) {
        const uint32_t idx = cbase + (uint32_t)lane;
        bool valid = idx < end;
        uint32_t p = valid ? a.ids[idx] : 0u;
        valid = valid && p < n_binned;
        const StrutRec<T> r = recs[valid ? p : 0u];
        // The strut is a candidate of this block and plane only where its
        // binned pixel and plane ranges cover them: then every tile size,
        // slab depth and group split hands the block the same candidates in
        // the same order, and the runs of four are the same.
        uint32_t zmask = 0u;            // bit k: plane kb + k within the strut's planes
        {
            const PRange pr = a.pranges[valid ? p : 0u];
            valid = valid && (int)pr.i0 <= ie && (int)pr.i1 >= i0 && (int)pr.j0 <= je &&
                    (int)pr.j1 >= j0;
            const int klo = pr.k0 - kb > 0 ? pr.k0 - kb : 0;
            const int khi = pr.k1 - kb < SZ - 1 ? pr.k1 - kb : SZ - 1;
            zmask = klo <= khi ? (2u << khi) - (1u << klo) : 0u;
        }
        const double ax = (double)r.ax, ay = (double)r.ay, az = (double)r.az;
        double* cl = line + lane;
        const Line ln = strut_line(r);
        const double L = ln.L, uz = ln.uz;
        {
            const double wx = cx - ax, wy = cy - ay;
            cl[0 * kWave] = az;
            cl[1 * kWave] = fma(wx, ln.ux, wy * ln.uy);
            cl[2 * kWave] = wx;
            cl[3 * kWave] = wy;
            cl[4 * kWave] = ln.ux;
            cl[5 * kWave] = ln.uy;
        }
#pragma unroll
        for (int k = 0; k < SZ; ++k) {
            if (k < nvalid) {
                // the line is read back from LDS for each plane (the empty
                // asm keeps the compiler from holding it in registers)
                asm volatile("" ::: "memory");
                const double az = cl[0 * kWave], txy = cl[1 * kWave], wx = cl[2 * kWave],
                             wy = cl[3 * kWave], ux = cl[4 * kWave], uy = cl[5 * kWave];
                const double z = a.z0 + ((double)(kb + k) + 0.5) * a.dz;
                const double wz = z - az;
                const double tc = fma(wz, uz, txy);
                const double mx = fma(tc, ux, -wx), my = fma(tc, uy, -wy), mz = fma(tc, uz, -wz);
                const double m2 = fma(mx, mx, fma(my, my, mz * mz));
                // e = F* - c, F* the point of the segment nearest to c, and
                // D = |e|.  The segment lies in the half-space n.(x - F*) >= 0
                // (n = e / D), so a pixel c + d of the block is at least
                // D - n.d >= D - (hx |e_x| + hy |e_y|) / D from it: the strut
                // reaches no pixel when D^2 - hx |e_x| - hy |e_y| >= R D.
                const double dt = fmin(fmax(tc, 0.0), L) - tc;
                const double ex = fma(dt, ux, mx), ey = fma(dt, uy, my);
                const double D2 = fma(dt, dt, m2);
                const double q = D2 - fma(hx, fabs(ex), hy * fabs(ey));
                // per-strut supports: the strut's cull radius and R^2, formed
                // here to keep no doubles live across the evaluation loop
                double Rc2 = Rc2_u, R2 = R2_u;
                if (SR) {
                    const double Rs = (double)r.pad;
                    const double Rc = Rs * (1.0 + 1e-7);
                    Rc2 = Rc * Rc;
                    R2 = Rs * Rs;
                }
                const bool pass = valid && ((zmask >> k) & 1u) && (q <= 0.0 || q * q < Rc2 * D2);
                const uint64_t mask = ballot64(pass);
                if (mask == 0ull) continue;
                if (pass) {
                    Stage<T> s;
                    s.mx2 = (T)(2.0 * mx);
                    s.my2 = (T)(2.0 * my);
                    s.ux = (T)ux;
                    s.uy = (T)uy;
                    s.ntc = (T)(-tc);
                    s.nbtc = (T)(L - tc);
                    s.H0 = (T)(R2 - m2);
                    s.wq = r.wq;
                    // rank among the passing lanes: set bits of mask below this lane
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                    stage[rank] = s;
                }
                __builtin_amdgcn_wave_barrier();
                const int n = __popcll(mask);
                T s_ = acc_s[k], c_ = acc_c[k];
                auto term_at = [&](int j) -> T {
                    const T t = K == LSL_KERNEL_GAUSS
                                    ? eval_term_gauss<T>(stage[j], dX, dY, d2, gk1, gk2, gc0)
                                    : eval_term<T>(stage[j], dX, dY, d2);
                    if (STATS) n_useful += t > T(0) ? 1ull : 0ull;
                    return t;
                };
                if (G == 1) {
                    for (int j = 0; j < n; ++j) comp_add(term_at(j), s_, c_);
                } else {
                    T* pk = pend + k * kWave + lane;
                    int q = open[k];
                    int j = 0;
                    if (q != 0) {               // complete the run left open
                        T g = *pk;
                        for (; j < n && q < G; ++j, ++q) g += term_at(j);
                        if (q == G) {
                            comp_add(g, s_, c_);
                            q = 0;
                        } else {
                            *pk = g;
                        }
                    }
#pragma unroll 1
                    for (; j + G <= n; j += G) {
                        T g = term_at(j);
#pragma unroll
                        for (int i = 1; i < G; ++i) g += term_at(j + i);
                        comp_add(g, s_, c_);
                    }
                    if (j < n) {                // open a run with the rest
                        T g = term_at(j);
                        for (q = 1, ++j; j < n; ++j, ++q) g += term_at(j);
                        *pk = g;
                    }
                    open[k] = q;
                }
                if (STATS) n_cand += pix ? (unsigned long long)n : 0ull;
                acc_s[k] = s_;
                acc_c[k] = c_;
                __builtin_amdgcn_wave_barrier();
            }
        }
    }

    if (G > 1) {
#pragma unroll
        for (int k = 0; k < SZ; ++k)
            if (open[k] != 0) comp_add(pend[k * kWave + lane], acc_s[k], acc_c[k]);
    }

    if (STATS) {
        if (!pix) n_useful = 0;
        for (int d = 32; d >= 1; d >>= 1) {
            n_cand += __shfl_xor(n_cand, d, kWave);
            n_useful += __shfl_xor(n_useful, d, kWave);
        }
        const unsigned long long npx = (unsigned long long)__popcll(ballot64(pix)) * nvalid;
        if (lane == 0) {
            atomicAdd(&a.stats[0], n_cand);
            atomicAdd(&a.stats[1], n_useful);
            atomicAdd(&a.stats[2], npx);
        }
        return;
    }
    if (pix && a.field) {
        T* out = (T*)a.field;
#pragma unroll
        for (int k = 0; k < SZ; ++k)
            if (k < nvalid)
                out[((size_t)(kb + k - a.k0) * (size_t)a.H + (size_t)pj) * (size_t)a.W + (size_t)pi] =
                    acc_s[k] + acc_c[k];
    }
    if (a.bits_blk) {
        // binary image, block-major: the block's ballot is its word
        const size_t nbx = (size_t)(a.W + 7) / 8, nby = (size_t)(a.H + 7) / 8;
        const T C = (T)a.C;
#pragma unroll
        for (int k = 0; k < SZ; ++k) {
            if (k < nvalid) {
                const uint64_t m = ballot64(pix && acc_s[k] + acc_c[k] >= C);
                if (lane == 0)
                    a.bits_blk[((size_t)(kb + k - a.k0) * nby + (size_t)(j0 >> 3)) * nbx +
                               (size_t)(i0 >> 3)] = m;
            }
        }
    }
}


}  // namespace fieldk
}  // namespace lsl
