// The float32 field kernel of the paper's quartic kernel (Eqs. 5-7), with the
// planes of a slab evaluated strut by strut.
//
// A wave owns an 8x8 pixel block over one slab of planes.  It walks the
// block's bucket list 64 entries at a time.  Staging (one lane per entry, in
// float64): the strut's line, the reach test of every plane of the slab (the
// block's support function, as in field_block.hpp) and, per plane, the two
// numbers the pixels need, written to LDS; the entries that reach the block
// at some plane are compacted with a ballot/mbcnt prefix.  Evaluation: for
// each candidate strut, every lane forms what does not depend on the plane
// once, then adds the strut's term to each plane the strut reaches.
//
// Lengths are in units of R_j / rho_j (hats below), R_j the strut's support
// and rho_j = (r_j R_j)^(1/5) / 2^e with one e per lattice chosen so that
// rho_j <= 1.  In those units the strut's term r_j/R_j^4 * integral(...) is
// the bare integral times 2^(5e): the closed form is homogeneous of degree 5
// in length, so the weight folds into the unit, and the sums are scaled by
// the power of two once at the end (exactly).  For a pixel p = c + d of
// plane k (c the block centre, d in the plane), with t measured along the
// strut's direction u from the foot of p on the line,
//
//   alpha = (A_r - d.u^) - kappa_k dz^ u_z,  beta = (B_r - d.u^) - kappa_k dz^ u_z,
//   H     = rho^2 (1 - dist(p, line)^2 / R^2)
//         = G_k + E + kappa_k * c1 * (d.u^),
//
// where r is a reference plane and kappa_k = k - r, A_r = -tc_r^ and
// B_r = L^ - tc_r^ (tc the position of the foot of c along the strut; each
// rounded once from float64, so that long struts lose nothing to
// cancellation), G_k = rho^2 - |m_k^|^2 (m_k = F_k - c, F_k the foot of c on
// the line at plane k, formed per plane in float64), E = 2 m_r^.d^ - |d^|^2 +
// (d.u^)^2 and c1 = 2 dz^ u_z: from plane r to plane k the foot moves by
// (k - r) dz u_z along the strut and the foot offset by (k - r) dz (u_z u -
// e_z), so 2 m.d grows by 2 (k - r) dz u_z (d.u).  The reference planes are the multiples of 8 (r = 8 floor(k / 8)),
// so a plane's value does not depend on how planes are grouped into slabs.
// The shift costs accuracy once 7 dz |d| is no longer small against R^2 (the
// pieces of H grow while H stays small): such lattices (a choice made once
// per lattice and grid) are sliced by the kernel of field_block.hpp, which
// stages every plane from float64.
// H <= rho^2 <= 1, so the clamp to [0, 1] is the max(H, 0) the square root
// needs.
//
// The term: with h = sqrt(H), ca, cb = alpha, beta clamped to [-h, h],
// s = ca + cb, D = cb - ca (the clamped interval, centre s/2, half-width D/2),
//
//   integral over [ca, cb] of (H - t^2)^2 dt = D Q,
//   Q = (H - s^2/4 - D^2/12)^2 + D^2 (s^2/12 + D^2/180),
//
// (expand (H - (s/2 + x)^2)^2 and integrate over x in [-D/2, D/2]; every
// piece is a square or a product of squares, so nothing cancels).  An
// interval outside the support gives D = 0: an exact zero.
//
// Sums: each plane's candidates are added in runs of eight consecutive
// candidates, g = fma(D, Q, g), and each run is added to a compensated sum
// (s' = s + g, e += g - (s' - s)).  A strut is a candidate of a block and
// plane when its binned pixel and plane ranges cover them and the reach test
// passes -- a function of the strut, the block and the plane alone -- and
// the strut order is the bucket list's (edge-list) order, so every tile size,
// slab depth and group split gives a pixel the same terms in the same runs:
// the field is bitwise the same.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace lsl {
namespace q32 {

constexpr int kRun = 8;         // terms per compensated add

// Per-wave LDS of the staging, indexed by the staged lane (bucket entry):
// pg, per plane G_k; gr, per reference group (A_r, B_r, 2 m_r,x^, 2 m_r,y^)
// with m^ = m / unit^2; e: (u_x^, u_y^, c1, 1 / unit^2); dl: -dz^ u_z;
// cand: the compacted candidates, lane | plane mask << 8.
template <int SZ>
struct Lds {
    float pg[SZ][kWave];
    float4 gr[SZ >= 16 ? 3 : (SZ >= 2 ? 2 : 1)][kWave];
    float4 e[kWave];
    float dl[kWave];
    uint32_t cand[kWave];
};

// (float)k for k in 0..7, formed with integer operations so that a uniform
// k stays in a scalar register (the float conversion is a vector operation)
__device__ __forceinline__ float kappa(int k) {
    // high and second-highest bytes of the float32 encodings of 0..7
    const uint32_t hi = (uint32_t)(0x4040404040403f00ull >> (8 * k)) & 0xffu;
    const uint32_t lo = (uint32_t)(0xe0c0a08040008000ull >> (8 * k)) & 0xffu;
    return __uint_as_float((hi << 24) | (lo << 16));
}

// Calls f(std::integral_constant<int, k>) for k = K .. N-1: the per-plane
// registers are indexed by constants from the start, so they stay separate
// scalars rather than one vector that every conditional update copies whole.
template <int K, int N, typename F>
__device__ __forceinline__ void for_planes(F&& f) {
    if constexpr (K < N) {
        f(std::integral_constant<int, K>{});
        for_planes<K + 1, N>(f);
    }
}

// A wave-uniform float64 value moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ void comp_add(float g, float& s, float& c) {
    const float sn = s + g;
    c += g - (sn - s);
    s = sn;
}

// The terms of one candidate strut (staging lane e, planes `mask`, uniform;
// E, nD and the planes' G_k its staged values) at the pixel d = (dX, dY) of each plane it
// reaches, added to the open runs of the planes of the slab that starts at
// plane kb (reference group gb).
template <int SZ, bool STATS>
__device__ __forceinline__ void add_candidate(const Lds<SZ>& L, uint32_t e,
                                              uint32_t mask, float4 E, float nD, int kb, int gb,
                                              const float (&Gk)[SZ], float dX, float dY,
                                              float nd2, bool pix, float (&acc_s)[SZ],
                                              float (&acc_c)[SZ], float (&run)[SZ],
                                              int (&open)[SZ], unsigned long long& n_cand,
                                              unsigned long long& n_useful) {
    const float du = __builtin_fmaf(dX, E.x, dY * E.y);        // d.u^
    const float P1 = E.z * du;
    const float ndd = nd2 * E.w;                                // -|d^|^2
    float Eg = 0.0f, ar = 0.0f, br = 0.0f;
    int gcur = -1;
    for_planes<0, SZ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (!((mask >> k) & 1u)) return;
        const int g = ((kb + k) >> 3) - gb;
        if (g != gcur) {
            const float4 Rg = L.gr[g][e];
            ar = Rg.x - du;
            br = Rg.y - du;
            Eg = __builtin_fmaf(du, du, __builtin_fmaf(Rg.z, dX, __builtin_fmaf(Rg.w, dY, ndd)));
            gcur = g;
        }
        const float kap = kappa((kb + k) & 7);
        const float al = __builtin_fmaf(kap, nD, ar);
        const float be = __builtin_fmaf(kap, nD, br);
        const float H = __builtin_amdgcn_fmed3f(__builtin_fmaf(kap, P1, Gk[k] + Eg), 0.0f, 1.0f);
        const float h = __builtin_amdgcn_sqrtf(H);
        const float ca = __builtin_amdgcn_fmed3f(al, -h, h);
        const float cb = __builtin_amdgcn_fmed3f(be, -h, h);
        const float s = ca + cb, D = cb - ca;
        const float s2 = s * s, D2 = D * D;
        const float A = __builtin_fmaf(D2, -1.0f / 12.0f, __builtin_fmaf(s2, -0.25f, H));
        const float V = __builtin_fmaf(s2, 1.0f / 12.0f, D2 * (1.0f / 180.0f));
        const float Q = __builtin_fmaf(A, A, D2 * V);
        if (STATS) {
            n_cand += pix ? 1ull : 0ull;
            n_useful += (pix && D * Q > 0.0f) ? 1ull : 0ull;
        }
        run[k] = __builtin_fmaf(D, Q, run[k]);
        if (++open[k] == kRun) {
            comp_add(run[k], acc_s[k], acc_c[k]);
            run[k] = 0.0f;
            open[k] = 0;
        }
    });}

// One wave: the 8x8 block `sub` of tile (tx, ty) over the planes of `slab`
// in [k0, k0+nk).
template <int SZ, bool STATS, bool SR>
__device__ __forceinline__ void field_block(const FieldArgs& a, int slab, int tx, int ty, int sub,
                                            Lds<SZ>& L) {
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
    const int gb = kb >> 3;                     // first reference group

    const uint32_t bucket = ((uint32_t)(slab - a.group_s0) * (uint32_t)a.nty + (uint32_t)ty) *
                                (uint32_t)a.ntx + (uint32_t)tx;
    uint32_t beg = a.offsets[bucket], end = a.offsets[bucket + 1];
    if (end > n_pairs) end = n_pairs;
    if (beg > end) beg = end;

    const int lx = lane & 7, ly = lane >> 3;
    const int pi = i0 + lx, pj = j0 + ly;
    const bool pix = pi < a.W && pj < a.H;
    // centre of the 8x8 centres (uniform: held in scalar registers)
    const double cx = uniform(a.x0 + ((double)i0 + 4.0) * a.dx);
    const double cy = uniform(a.y0 + ((double)j0 + 4.0) * a.dy);
    // d in grid units; the strut's values carry its length unit (so one
    // support given per strut is bitwise the same computation as one R)
    const double dXd = ((double)lx - 3.5) * a.dx, dYd = ((double)ly - 3.5) * a.dy;
    const float dX = (float)dXd, dY = (float)dYd;
    const float nd2 = (float)(-(dXd * dXd + dYd * dYd));
    const float hxf = (float)(3.5 * a.dx), hyf = (float)(3.5 * a.dy);
    const int ie = i0 + 7 < a.W - 1 ? i0 + 7 : a.W - 1;
    const int je = j0 + 7 < a.H - 1 ? j0 + 7 : a.H - 1;

    float acc_s[SZ], acc_c[SZ], run[SZ];
    int open[SZ];                               // terms in each plane's open run (uniform)
    for_planes<0, SZ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        acc_s[k] = acc_c[k] = run[k] = 0.0f;
        open[k] = 0;
    });
    unsigned long long n_cand = 0, n_useful = 0;

    const StrutRec<float>* recs = (const StrutRec<float>*)a.rec;
    // the bucket entries of the next chunk are read one chunk ahead, and all
    // of an entry's records at once: one memory round trip per chunk
    // (read unconditionally from a clamped index, so that the wait for this
    // chunk's records does not wait for them; lanes past the end are
    // invalid whatever they read)
    uint32_t p_next = 0u;
    if (beg < end) p_next = a.ids[beg + (uint32_t)lane < end ? beg + (uint32_t)lane : end - 1u];
    for (uint32_t cbase = beg; cbase < end; cbase += kWave) {
        // ---------------------------------------------------------- staging
        const uint32_t idx = cbase + (uint32_t)lane;
        bool valid = idx < end;
        const uint32_t p = p_next;
        valid = valid && p < n_binned;
        const uint32_t q = valid ? p : 0u;
        const StrutRec<float> r = recs[q];
        // (one 16-byte load: i0 | i1 << 16, j0 | j1 << 16, k0, k1)
        const uint4 pr = reinterpret_cast<const uint4*>(a.pranges)[q];
        // the strut's direction and length (float64, from the binning)
        const double4 ln = a.line[q];
        // lengths in units of R / rho (rho <= 1: the weight folded into the
        // closed form, which scales with the fifth power of length)
        const double rho = (double)a.rho[q];
        p_next = a.ids[idx + kWave < end ? idx + kWave : end - 1u];
        uint32_t zmask = 0u;
        {
            valid = valid && (int)(pr.x & 0xffffu) <= ie && (int)(pr.x >> 16) >= i0 &&
                    (int)(pr.y & 0xffffu) <= je && (int)(pr.y >> 16) >= j0;
            const int pk0 = (int)pr.z, pk1 = (int)pr.w;
            const int klo = pk0 - kb > 0 ? pk0 - kb : 0;
            const int khi = pk1 - kb < SZ - 1 ? pk1 - kb : SZ - 1;
            zmask = valid && klo <= khi ? (2u << khi) - (1u << klo) : 0u;
        }
        const double ax = (double)r.ax, ay = (double)r.ay, az = (double)r.az;
        const double Rs = SR ? (double)r.pad : a.R;
        const double iR = rho / Rs, iR2 = iR * iR;
        // the reach test below runs in float32 against a support widened by
        // 1e-5 relative, far above its rounding, so it never drops a strut
        // that reaches a pixel
        const float Rc2f = (float)(Rs * Rs * (1.0 + 2e-5));
        const double wx = cx - ax, wy = cy - ay;
        const double txy = fma(wx, ln.x, wy * ln.y);
        const float uxf = (float)ln.x, uyf = (float)ln.y, Lf = (float)ln.w;
        // per plane, the foot offset moves by dz (u_z u - e_z)
        const float vxf = (float)(a.dz * ln.z * ln.x), vyf = (float)(a.dz * ln.z * ln.y);
        const double c2 = a.dz * a.dz * (1.0 - ln.z * ln.z);
        uint32_t pmask = 0u;
        double tcr = 0.0, m2r = 0.0, c1 = 0.0;
        float mxr = 0.0f, myr = 0.0f;
        int grp = -1, rref = 0;
        // one plane at a time: the float64 temporaries of several planes in
        // flight would cost registers the evaluation needs
#pragma unroll 1
        for (int k = 0; k < nvalid; ++k) {
            const int ka = kb + k;
            const int g = ka >> 3;
            if (g != grp) {
                // the group's reference plane, in float64
                grp = g;
                rref = g << 3;
                const double z = a.z0 + ((double)rref + 0.5) * a.dz;
                const double wz = z - az;
                tcr = fma(wz, ln.z, txy);
                const double mx = fma(tcr, ln.x, -wx), my = fma(tcr, ln.y, -wy),
                             mz = fma(tcr, ln.z, -wz);
                m2r = fma(mx, mx, fma(my, my, mz * mz));
                c1 = -2.0 * a.dz * mz;
                mxr = (float)mx;
                myr = (float)my;
                L.gr[g - gb][lane] = make_float4((float)(-tcr * iR), (float)((ln.w - tcr) * iR),
                                                 (float)(2.0 * mx * iR2), (float)(2.0 * my * iR2));
            }
            // plane ka from the reference: tc and |m|^2 (m is orthogonal to u,
            // so |m_k|^2 = |m_r|^2 - 2 kappa dz m_r,z + kappa^2 dz^2 (1 - u_z^2))
            const int kap = ka - rref;
            const double kd = (double)kap;
            const double tc = fma(kd * a.dz, ln.z, tcr);
            const double m2 = fma(kd * kd, c2, fma(kd, c1, m2r));
            // reach test of field_block.hpp: the segment's point F* nearest
            // to c, e = F* - c, D = |e|; no pixel is within R when
            // D^2 - hx |e_x| - hy |e_y| >= R D
            const float tcf = (float)tc, kf = (float)kap;
            const float mxf = __builtin_fmaf(kf, vxf, mxr), myf = __builtin_fmaf(kf, vyf, myr);
            const float dt = __builtin_amdgcn_fmed3f(tcf, 0.0f, Lf) - tcf;
            const float ex = __builtin_fmaf(dt, uxf, mxf), ey = __builtin_fmaf(dt, uyf, myf);
            const float D2 = __builtin_fmaf(dt, dt, (float)m2);
            const float q = D2 - __builtin_fmaf(hxf, fabsf(ex), hyf * fabsf(ey));
            // evaluated without branches: both compares and the range bit
            const uint32_t pass = ((zmask >> k) & 1u) &
                                  ((uint32_t)(q <= 0.0f) | (uint32_t)(q * q < Rc2f * D2));
            pmask |= pass << k;
            L.pg[k][lane] = (float)(rho * rho - m2 * iR2);
        }
        L.e[lane] = make_float4((float)(ln.x * iR), (float)(ln.y * iR),
                                (float)(2.0 * a.dz * ln.z * iR), (float)iR2);
        L.dl[lane] = (float)(-a.dz * ln.z * iR);
        const uint64_t cm = ballot64(pmask != 0u);
        if (pmask != 0u) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(cm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
            L.cand[rank] = (uint32_t)lane | (pmask << 8);
        }
        __builtin_amdgcn_wave_barrier();
        const int n = __popcll(cm);

        // ------------------------------------------------------- evaluation
        // The next candidate's values are read while this one is evaluated.
        uint32_t c = L.cand[0];
        float4 E = L.e[c & 63u];
        float nD = L.dl[c & 63u];
#pragma unroll 1
        for (int j = 0; j < n; ++j) {
            const uint32_t e = c & 63u;
            const uint32_t mask = __builtin_amdgcn_readfirstlane(c >> 8);
            float Gk[SZ];
            for_planes<0, SZ>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                Gk[k] = L.pg[k][e];
            });
            const uint32_t cn = L.cand[j + 1 < n ? j + 1 : j];
            const float4 En = L.e[cn & 63u];
            const float nDn = L.dl[cn & 63u];
            add_candidate<SZ, STATS>(L, e, mask, E, nD, kb, gb, Gk, dX, dY, nd2, pix,
                                                acc_s, acc_c, run, open, n_cand, n_useful);
            c = cn;
            E = En;
            nD = nDn;
        }
        __builtin_amdgcn_wave_barrier();
    }

    for_planes<0, SZ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (open[k] != 0) comp_add(run[k], acc_s[k], acc_c[k]);
    });

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
        float* out = (float*)a.field;
        for_planes<0, SZ>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if (k < nvalid)
                out[((size_t)(kb + k - a.k0) * (size_t)a.H + (size_t)pj) * (size_t)a.W + (size_t)pi] =
                    __builtin_ldexpf(acc_s[k] + acc_c[k], 5 * a.wexp);
        });
    }
    if (a.bits_blk) {
        const size_t nbx = (size_t)(a.W + 7) / 8, nby = (size_t)(a.H + 7) / 8;
        const float C = (float)a.C;
        for_planes<0, SZ>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if (k < nvalid) {
                const uint64_t m =
                    ballot64(pix && __builtin_ldexpf(acc_s[k] + acc_c[k], 5 * a.wexp) >= C);
                if (lane == 0)
                    a.bits_blk[((size_t)(kb + k - a.k0) * nby + (size_t)(j0 >> 3)) * nbx +
                               (size_t)(i0 >> 3)] = m;
            }
        });
    }
}

}  // namespace q32
}  // namespace lsl
