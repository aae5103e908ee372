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
// pixel's offset, so sum G K q_perp = sum G K m - d sum G K + u sum G K (d.u):
// each pair adds to thirteen registers without forming q_perp.
//
// Work split.  One wave takes one (tile, slab) bucket and walks the tile's
// 8x8 blocks in a fixed order.  For 32 list entries at a time it stages, per
// block and plane, the same block-centre quantities as the forward pass
// (m and tc), compacts the struts that reach the block in any
// plane of the slab, and then for each such strut loops over only the planes
// it reaches: every lane adds its pixel's contribution to thirteen registers,
// the wave sums them once per (strut, block), and one lane adds the sums into
// the entry's LDS slot.  The slots are written once per bucket entry, so each
// (slab, tile, strut) pair gets exactly one partial, with no atomics.
// The per-strut sums then run over the pairs of each strut in emission order
// (slab, tile), and the nodes gather their struts' gradients through a node
// -> strut incidence list.  Every reduction has a fixed order.
#include "kernels.hpp"

namespace lsl {
namespace {

constexpr int kChunk = 32;      // bucket entries staged at a time
constexpr int kParts = 9;       // pixel sums per (strut, bucket)

template <typename T>
struct alignas(16) BStrut {
    T ux, uy, uz, pad;
    uint32_t planes;            // bit k: the strut reaches the block in plane k
    uint32_t pos;               // entry index within the chunk
};

template <typename T>
struct alignas(16) BPlane {
    T mx2, my2, ntc, H0;        // as in the forward pass
    T mx, my, mz, nbtc;         // m = F - c; L - tc
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

// Sum over the wave, complete in lane 63 (kSumLane).  float: DPP row
// operations only (quad swaps, half-row and row mirrors, then the row
// broadcasts of lanes 15 and 31 into the following rows), no LDS traffic.
constexpr int kSumLane = 63;

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_take(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <typename T, int SZ>
__global__ __launch_bounds__(64) void k_backward(BackArgs a, uint32_t n_items) {
    __shared__ BStrut<T> bs[kChunk];
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
    const double rb = 3.5 * sqrt(a.dx * a.dx + a.dy * a.dy);
    const double thr = (a.R + rb) * (1.0 + 1e-7);
    const double thr2 = thr * thr;
    const double R2 = a.R * a.R;
    const uint64_t lt = lanes_below(lane);
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
                    const double ex = tc < 0.0 ? -tc : (tc > L ? tc - L : 0.0);
                    if (valid && fma(ex, ex, m2) < thr2) {
                        planes |= 1u << k;
                        BPlane<T> P;
                        P.mx2 = (T)(2.0 * mx);
                        P.my2 = (T)(2.0 * my);
                        P.ntc = (T)(-tc);
                        P.H0 = (T)(R2 - m2);
                        P.mx = (T)mx;
                        P.my = (T)my;
                        P.mz = (T)mz;
                        P.nbtc = (T)(L - tc);
                        bp[lane][k] = P;
                    }
                }
            }
            const uint64_t mask = ballot64(planes != 0u);
            if (mask == 0ull) continue;
            if (planes != 0u) {
                BStrut<T> b;
                b.ux = (T)ux;
                b.uy = (T)uy;
                b.uz = (T)uz;
                b.pad = T(0);
                b.planes = planes;
                b.pos = (uint32_t)lane;
                bs[__popcll(mask & lt)] = b;
            }
            __builtin_amdgcn_wave_barrier();
            const int n = __popcll(mask);
            for (int j = 0; j < n; ++j) {
                const BStrut<T> b = bs[j];
                const uint32_t planes_s = __builtin_amdgcn_readfirstlane(b.planes);
                T Aw = 0, Aa = 0, Ab = 0, AK = 0, AKx = 0, AKy = 0, AKz = 0, AKd = 0, AJ = 0,
                  AJx = 0, AJy = 0, AJz = 0, AJd = 0;
#pragma unroll
                for (int k = 0; k < SZ; ++k) {
                    if (k < nvalid && ((planes_s >> k) & 1u)) {
                        const BPlane<T> P = bp[b.pos][k];
                        const T g = G[k];
                        const T du = dfma(dX, b.ux, dY * b.uy);
                        const T al = P.ntc - du;
                        const T be = P.nbtc - du;
                        const T H = dfma(du, du, dfma(P.mx2, dX, dfma(P.my2, dY, P.H0 - d2)));
                        const T h = dsqrt<T>(H > T(0) ? H : T(0));
                        const T ca = dclamp<T>(al, h), cb = dclamp<T>(be, h);
                        const T D = cb - ca;
                        const T x2 = ca * ca, y2 = cb * cb, xy = ca * cb;
                        const T q2 = x2 + y2;
                        const T S1 = q2 + xy;
                        const T S2 = dfma(q2, S1, -(xy * xy));
                        const T Q = dfma(H, dfma(T(-2.0 / 3.0), S1, H), T(0.2) * S2);
                        Aw = dfma(g * D, Q, Aw);
                        T pa = dmax<T>(dfma(-al, al, H), T(0));
                        pa = pa * pa;
                        T pb = dmax<T>(dfma(-be, be, H), T(0));
                        pb = pb * pb;
                        Aa = dfma(g, pa, Aa);
                        Ab = dfma(g, pb, Ab);
                        const T J = T(2) * dfma(T(-1.0 / 3.0), S1, H) * D;   // J R^4
                        const T K = dfma(T(2) * al, J, pb - pa);               // K R^4
                        const T gK = g * K, gJ = g * J;
                        AK += gK;
                        AKx = dfma(gK, P.mx, AKx);
                        AKy = dfma(gK, P.my, AKy);
                        AKz = dfma(gK, P.mz, AKz);
                        AKd = dfma(gK, du, AKd);
                        AJ += gJ;
                        AJx = dfma(gJ, P.mx, AJx);
                        AJy = dfma(gJ, P.my, AJy);
                        AJz = dfma(gJ, P.mz, AJz);
                        AJd = dfma(gJ, du, AJd);
                    }
                }
                // sum G K q_perp = sum G K m - d sum G K + u sum G K (d.u), d = (dX, dY, 0)
                AKx = dfma(b.ux, AKd, dfma(-dX, AK, AKx));
                AKy = dfma(b.uy, AKd, dfma(-dY, AK, AKy));
                AKz = dfma(b.uz, AKd, AKz);
                AJx = dfma(b.ux, AJd, dfma(-dX, AJ, AJx));
                AJy = dfma(b.uy, AJd, dfma(-dY, AJ, AJy));
                AJz = dfma(b.uz, AJd, AJz);
                const T v0 = wave_sum(Aw), v1 = wave_sum(Aa), v2 = wave_sum(Ab),
                        v3 = wave_sum(AKx), v4 = wave_sum(AKy), v5 = wave_sum(AKz),
                        v6 = wave_sum(AJx), v7 = wave_sum(AJy), v8 = wave_sum(AJz);
                if (lane == kSumLane) {
                    T* sl = slot[b.pos];
                    sl[0] += v0;
                    sl[1] += v1;
                    sl[2] += v2;
                    sl[3] += v3;
                    sl[4] += v4;
                    sl[5] += v5;
                    sl[6] += v6;
                    sl[7] += v7;
                    sl[8] += v8;
                }
                __builtin_amdgcn_wave_barrier();
            }
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
        for (int q = lane; q < nent * kParts; q += kWave)
            part[(size_t)cbase * kParts + (size_t)q] = (&slot[0][0])[q];
        __builtin_amdgcn_wave_barrier();
    }
}

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
    const uint32_t e1 = a.eoff[i] + (uint32_t)(hi - s0 + 1) * nxy;
    double s[kParts];
    for (int q = 0; q < kParts; ++q) s[q] = 0.0;
    const T* part = (const T*)a.partial;
    for (uint32_t e = e0; e < e1; ++e) {
        const uint32_t pos = a.inv[e];
        if (pos >= n_pairs) continue;
        for (int q = 0; q < kParts; ++q) s[q] += (double)part[(size_t)pos * kParts + q];
    }
    const StrutRec<T> r = ((const StrutRec<T>*)a.rec)[p];
    const double w = (double)((const T*)a.w)[p];
    const double R4 = a.R * a.R * a.R * a.R;
    const Line ln = strut_line(r);
    const double u[3] = {ln.ux, ln.uy, ln.uz};
    const double cw = w / R4;
    double* acc = a.acc + (size_t)p * 7;
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
    k_backward<T, SZ><<<n_items, 64, 0, st>>>(a, n_items);
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
    if (dtype == LSL_F32) return launch_bt<float>(a, (uint32_t)n_items, st);
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
