// Strut preparation: validation, slab/tile ranges of each strut's swept box,
// sort keys of the edge list (ascending z of the lower end, Sec. 4; with
// per-strut supports the first slab is a major key) and the histograms the
// slab-group plan is made from.
#include "kernels.hpp"

namespace lsl {
namespace {

struct AxisRange {
    int32_t i0, i1;
    bool ok;
};

// Outward-rounded index range of the points o + (i + 1/2) s inside [lo, hi],
// clamped to [0, n-1].  Evaluated in float64 in this exact order (the file is
// built without floating-point contraction).
__device__ __forceinline__ AxisRange axis_range(double lo, double hi, double o, double inv,
                                                int32_t n) {
    const double f0 = floor((lo - o) * inv - 0.5);
    const double f1 = ceil((hi - o) * inv - 0.5);
    AxisRange r;
    r.ok = (f1 >= 0.0) && (f0 <= (double)(n - 1)) && (f0 <= f1);
    const double c0 = fmin(fmax(f0, 0.0), (double)(n - 1));
    const double c1 = fmin(fmax(f1, 0.0), (double)(n - 1));
    r.i0 = r.ok ? (int32_t)c0 : 0;
    r.i1 = r.ok ? (int32_t)c1 : -1;
    return r;
}

__device__ __forceinline__ uint32_t float_key(float z) {
    z = z + 0.0f;                                 // -0 sorts with +0
    const uint32_t b = __float_as_uint(z);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t double_key(double z) {
    z = z + 0.0;
    const uint64_t b = (uint64_t)__double_as_longlong(z);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// Plan histograms live in LDS per block when the slab count allows it.
constexpr int kLdsSlabs = 2048;

template <typename T>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
    __shared__ uint32_t h_lo[kLdsSlabs], h_hi[kLdsSlabs];
    __shared__ unsigned long long h_pairs[kLdsSlabs + 1];
    __shared__ uint32_t h_rows[kLdsSlabs + 1];   // modulo 2^32: a slab's rows are < 2^32
    __shared__ uint32_t h_n;
    const bool lds = a.n_slabs <= kLdsSlabs;
    if (lds) {
        for (int i = threadIdx.x; i < a.n_slabs; i += blockDim.x) {
            h_lo[i] = 0u;
            h_hi[i] = 0u;
            h_pairs[i] = 0ull;
            h_rows[i] = 0u;
        }
        if (threadIdx.x == 0) {
            h_pairs[a.n_slabs] = 0ull;
            h_rows[a.n_slabs] = 0u;
            h_n = 0u;
        }
        __syncthreads();
    }
    // each block takes a contiguous range of edges (few slabs per block's
    // histograms, flushed once at the end)
    const int64_t per_block = (a.n_edges + gridDim.x - 1) / gridDim.x;
    const int64_t e_beg = (int64_t)blockIdx.x * per_block;
    const int64_t e_end = e_beg + per_block < a.n_edges ? e_beg + per_block : a.n_edges;
    uint32_t inv_acc = 0u, wr_acc = 0u;     // smallest support, largest r R (as bits)
    for (int64_t e = e_beg + threadIdx.x; e < e_end; e += blockDim.x) {
        bool binned = false;
        SRange rg{0, 0, 0, 0, 0, -1};
        PRange pr{0, 0, 0, 0, 0, -1};
        uint32_t klo = 0xffffffffu, khi = 0xffffffffu;
        unsigned long long ntile = 0;
        uint32_t nrow = 0;
        float rs_binned = 0.0f;             // the support of a binned strut
        float wr_binned = 0.0f;             // and its weight times its support
        {
            const int32_t ia = a.edges[2 * e], ib = a.edges[2 * e + 1];
            const T* nd = (const T*)a.nodes;
            const T w = ((const T*)a.weight)[e];
            bool bad = false;
            if (ia < 0 || ib < 0 || (int64_t)ia >= a.n_nodes || (int64_t)ib >= a.n_nodes) {
                atomicOr(a.err, 1u);
                bad = true;
            }
            if (!(w >= T(0)) || !isfinite((double)w)) {
                atomicOr(a.err, 2u);
                bad = true;
            }
            double Rs = a.R;                 // this strut's support
            if (a.support) {
                Rs = (double)((const T*)a.support)[e];
                if (!(Rs > 0.0) || !isfinite(Rs)) {
                    atomicOr(a.err, 8u);
                    bad = true;
                }
            }
            if (!bad && a.max_r_over_sigma > 0.0 && !(Rs <= a.max_r_over_sigma * a.sigma)) {
                atomicOr(a.err, 16u);
                bad = true;
            }
            if (!bad) {
                const double ax = (double)nd[3 * ia], ay = (double)nd[3 * ia + 1],
                             az = (double)nd[3 * ia + 2];
                const double bx = (double)nd[3 * ib], by = (double)nd[3 * ib + 1],
                             bz = (double)nd[3 * ib + 2];
                if (!isfinite(ax) || !isfinite(ay) || !isfinite(az) || !isfinite(bx) ||
                    !isfinite(by) || !isfinite(bz)) {
                    atomicOr(a.err, 4u);
                } else if ((w != T(0) || a.keep_zero) && !(ax == bx && ay == by && az == bz)) {
                    const AxisRange rz = axis_range(fmin(az, bz) - Rs, fmax(az, bz) + Rs, a.z0,
                                                    a.inv_dz, a.S);
                    const AxisRange rx = axis_range(fmin(ax, bx) - Rs, fmax(ax, bx) + Rs, a.x0,
                                                    a.inv_dx, a.W);
                    const AxisRange ry = axis_range(fmin(ay, by) - Rs, fmax(ay, by) + Rs, a.y0,
                                                    a.inv_dy, a.H);
                    if (rz.ok && rx.ok && ry.ok) {
                        binned = true;
                        rs_binned = (float)Rs;
                        wr_binned = (float)((double)w * Rs);
                        pr.i0 = (uint16_t)rx.i0;
                        pr.i1 = (uint16_t)rx.i1;
                        pr.j0 = (uint16_t)ry.i0;
                        pr.j1 = (uint16_t)ry.i1;
                        pr.k0 = rz.i0;
                        pr.k1 = rz.i1;
                        rg.s0 = rz.i0 / a.slab;
                        rg.s1 = rz.i1 / a.slab;
                        rg.tx0 = (uint16_t)(rx.i0 / a.tile);
                        rg.tx1 = (uint16_t)(rx.i1 / a.tile);
                        rg.ty0 = (uint16_t)(ry.i0 / a.tile);
                        rg.ty1 = (uint16_t)(ry.i1 / a.tile);
                        ntile = (unsigned long long)(rg.tx1 - rg.tx0 + 1) *
                                (unsigned long long)(rg.ty1 - rg.ty0 + 1);
                        nrow = row_segments(rg);
                        const T zlo = nd[3 * ia + 2] < nd[3 * ib + 2] ? nd[3 * ia + 2]
                                                                      : nd[3 * ib + 2];
                        if (sizeof(T) == 4) {
                            klo = float_key((float)zlo);
                        } else {
                            const uint64_t k = double_key((double)zlo);
                            klo = (uint32_t)k;
                            khi = (uint32_t)(k >> 32);
                        }
                    }
                }
            }
            a.key_lo[e] = klo;
            if (sizeof(T) == 8) a.key_hi[e] = khi;
            if (a.key_s0) a.key_s0[e] = binned ? (uint32_t)rg.s0 : (uint32_t)a.n_slabs;
            a.vals[e] = (uint32_t)e;
            a.ranges[e] = rg;
            a.pranges[e] = pr;
        }
        if (binned) {
            // (positive floats order as their bits; the complement turns the
            // minimum into a maximum from zero)
            const uint32_t iv = ~__float_as_uint(rs_binned), wv = __float_as_uint(wr_binned);
            inv_acc = iv > inv_acc ? iv : inv_acc;
            wr_acc = wv > wr_acc ? wv : wr_acc;
            // plan histograms: struts starting / ending in each slab, and
            // difference arrays of (slab, tile) pairs and of (slab, tile row,
            // column segment) cells
            if (lds) {
                atomicAdd(&h_lo[rg.s0], 1u);
                atomicAdd(&h_hi[rg.s1], 1u);
                atomicAdd(&h_pairs[rg.s0], ntile);
                atomicAdd(&h_pairs[rg.s1 + 1], 0ull - ntile);
                atomicAdd(&h_rows[rg.s0], nrow);
                atomicAdd(&h_rows[rg.s1 + 1], 0u - nrow);
                atomicAdd(&h_n, 1u);
            } else {
                atomicAdd(&a.cnt_lo[rg.s0], 1u);
                atomicAdd(&a.cnt_hi[rg.s1], 1u);
                atomicAdd(&a.pair_diff[rg.s0], ntile);
                atomicAdd(&a.pair_diff[rg.s1 + 1], 0ull - ntile);
                atomicAdd(&a.row_diff[rg.s0], nrow);
                atomicAdd(&a.row_diff[rg.s1 + 1], 0u - nrow);
                atomicAdd(a.n_binned, 1u);
            }
        }
    }
    // the smallest support of a binned strut
    if (a.support && a.min_support) {
        uint32_t inv = inv_acc;
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)inv, d, kWave);
            inv = inv > o ? inv : o;
        }
        if ((threadIdx.x & (kWave - 1)) == 0 && inv != 0u) atomicMax(a.min_support, inv);
    }
    // the largest r R of a binned strut (the float32 field kernel's scale)
    if (a.max_wr) {
        uint32_t v = wr_acc;
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)v, d, kWave);
            v = v > o ? v : o;
        }
        if ((threadIdx.x & (kWave - 1)) == 0 && v != 0u) atomicMax(a.max_wr, v);
    }
    if (lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < a.n_slabs; i += blockDim.x) {
            if (h_lo[i]) atomicAdd(&a.cnt_lo[i], h_lo[i]);
            if (h_hi[i]) atomicAdd(&a.cnt_hi[i], h_hi[i]);
            if (h_pairs[i]) atomicAdd(&a.pair_diff[i], h_pairs[i]);
            if (h_rows[i]) atomicAdd(&a.row_diff[i], h_rows[i]);
        }
        if (threadIdx.x == 0) {
            if (h_pairs[a.n_slabs]) atomicAdd(&a.pair_diff[a.n_slabs], h_pairs[a.n_slabs]);
            if (h_rows[a.n_slabs]) atomicAdd(&a.row_diff[a.n_slabs], h_rows[a.n_slabs]);
            if (h_n) atomicAdd(a.n_binned, h_n);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_binned) return;
    const uint32_t e = a.perm[p];
    const int32_t ia = a.edges[2 * (size_t)e], ib = a.edges[2 * (size_t)e + 1];
    const T* nd = (const T*)a.nodes;
    const double w = (double)((const T*)a.weight)[e];
    const double Rs = a.support ? (double)((const T*)a.support)[e] : a.R;
    const double R2 = Rs * Rs;
    StrutRec<T> r;
    r.ax = nd[3 * ia];
    r.ay = nd[3 * ia + 1];
    r.az = nd[3 * ia + 2];
    // the weight folded with the kernel's constant: r / R^4 (Eq. 5), or
    // r exp(-R^2 / 2 sigma^2) (Gaussian)
    r.wq = a.kernel == LSL_KERNEL_GAUSS ? (T)(w * exp(-R2 / (2.0 * a.sigma * a.sigma)))
                                        : (T)(w / (R2 * R2));
    r.bx = nd[3 * ib];
    r.by = nd[3 * ib + 1];
    r.bz = nd[3 * ib + 2];
    r.pad = a.support ? ((const T*)a.support)[e] : T(0);
    ((StrutRec<T>*)a.rec)[p] = r;
    a.ranges[p] = a.ranges_by_id[e];
    a.pranges[p] = a.pranges_by_id[e];
    ((T*)a.w)[p] = (T)w;
    a.ends[p] = make_int2(ia, ib);
    const Line ln = strut_line(r);
    a.line[p] = make_double4(ln.ux, ln.uy, ln.uz, ln.L);
    // lengths of the float32 field kernel are in units of R / rho, which
    // folds the weight into the closed form's degree-5 scaling
    a.rho[p] = (float)(pow(w * Rs, 0.2) * ldexp(1.0, -a.wexp));
}

__global__ void k_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

}  // namespace

lsl_status launch_prep(int dtype, const PrepArgs& a, hipStream_t st) {
    if (a.n_edges == 0) return LSL_OK;
    int dev = 0, cus = 0;
    LSL_HIP(hipGetDevice(&dev));
    LSL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // four blocks per compute unit (the histograms' LDS allows that many),
    // each over a contiguous range of at least 256 edges
    const int64_t by_edges = (a.n_edges + 255) / 256;
    const int64_t cap = 4 * (int64_t)(cus > 0 ? cus : 1);
    const unsigned g = (unsigned)(by_edges < cap ? by_edges : cap);
    if (dtype == LSL_F32)
        k_prep<float><<<g, 256, 0, st>>>(a);
    else
        k_prep<double><<<g, 256, 0, st>>>(a);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_gather(int dtype, const GatherArgs& a, hipStream_t st) {
    if (a.n_binned == 0) return LSL_OK;
    const unsigned g = (unsigned)((a.n_binned + 255) / 256);
    if (dtype == LSL_F32)
        k_gather<float><<<g, 256, 0, st>>>(a);
    else
        k_gather<double><<<g, 256, 0, st>>>(a);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status launch_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, size_t n,
                             hipStream_t st) {
    if (n == 0) return LSL_OK;
    k_gather_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, idx, dst, n);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace lsl
