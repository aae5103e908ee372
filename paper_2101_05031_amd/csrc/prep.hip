// Strut preparation: validation, slab/tile ranges of each strut's swept box,
// sort keys of the edge list (ascending z of the lower end, Sec. 4) and the
// histograms the slab-group plan is made from.
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

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Adds `cnt` of each distinct bin value held by the lanes in `mask` with one
// atomic per value (lanes of a wave are usually in the same slab).
__device__ __forceinline__ void wave_hist_add(bool take, int32_t bin, unsigned long long amount,
                                              uint32_t* cnt, unsigned long long* acc,
                                              int acc_off, bool negate) {
    const int lane = lane_id();
    uint64_t todo = ballot64(take);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int32_t v = __shfl(bin, leader, kWave);
        const bool mine = take && bin == v && ((todo >> lane) & 1ull);
        const uint64_t peers = ballot64(mine);
        const unsigned long long s = wave_sum_u64(mine ? amount : 0ull);
        if (lane == leader) {
            atomicAdd(&cnt[v], (uint32_t)__popcll(peers));
            atomicAdd(&acc[v + acc_off], negate ? (0ull - s) : s);
        }
        todo &= ~peers;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = e < a.n_edges;
    bool binned = false;
    SRange rg{0, 0, 0, 0, 0, -1};
    uint32_t klo = 0xffffffffu, khi = 0xffffffffu;
    unsigned long long ntile = 0;
    if (live) {
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
        if (!bad) {
            const double ax = (double)nd[3 * ia], ay = (double)nd[3 * ia + 1],
                         az = (double)nd[3 * ia + 2];
            const double bx = (double)nd[3 * ib], by = (double)nd[3 * ib + 1],
                         bz = (double)nd[3 * ib + 2];
            if (!isfinite(ax) || !isfinite(ay) || !isfinite(az) || !isfinite(bx) ||
                !isfinite(by) || !isfinite(bz)) {
                atomicOr(a.err, 4u);
            } else if (w != T(0) && !(ax == bx && ay == by && az == bz)) {
                const AxisRange rz = axis_range(fmin(az, bz) - a.R, fmax(az, bz) + a.R, a.z0,
                                                a.inv_dz, a.S);
                const AxisRange rx = axis_range(fmin(ax, bx) - a.R, fmax(ax, bx) + a.R, a.x0,
                                                a.inv_dx, a.W);
                const AxisRange ry = axis_range(fmin(ay, by) - a.R, fmax(ay, by) + a.R, a.y0,
                                                a.inv_dy, a.H);
                if (rz.ok && rx.ok && ry.ok) {
                    binned = true;
                    rg.s0 = rz.i0 / a.slab;
                    rg.s1 = rz.i1 / a.slab;
                    rg.tx0 = (uint16_t)(rx.i0 / a.tile);
                    rg.tx1 = (uint16_t)(rx.i1 / a.tile);
                    rg.ty0 = (uint16_t)(ry.i0 / a.tile);
                    rg.ty1 = (uint16_t)(ry.i1 / a.tile);
                    ntile = (unsigned long long)(rg.tx1 - rg.tx0 + 1) *
                            (unsigned long long)(rg.ty1 - rg.ty0 + 1);
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
        a.vals[e] = (uint32_t)e;
        a.ranges[e] = rg;
    }
    // plan histograms: one atomic per distinct slab per wave
    wave_hist_add(binned, rg.s0, ntile, a.cnt_lo, a.pair_diff, 0, false);
    wave_hist_add(binned, rg.s1, ntile, a.cnt_hi, a.pair_diff, 1, true);
    const uint64_t nb = ballot64(binned);
    if (lane_id() == 0 && nb) atomicAdd(a.n_binned, (uint32_t)__popcll(nb));
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_binned) return;
    const uint32_t e = a.perm[p];
    const int32_t ia = a.edges[2 * (size_t)e], ib = a.edges[2 * (size_t)e + 1];
    const T* nd = (const T*)a.nodes;
    const double w = (double)((const T*)a.weight)[e];
    const double R2 = a.R * a.R;
    StrutRec<T> r;
    r.ax = nd[3 * ia];
    r.ay = nd[3 * ia + 1];
    r.az = nd[3 * ia + 2];
    r.wq = (T)(w / (R2 * R2));
    r.bx = nd[3 * ib];
    r.by = nd[3 * ib + 1];
    r.bz = nd[3 * ib + 2];
    r.pad = T(0);
    ((StrutRec<T>*)a.rec)[p] = r;
    a.ranges[p] = a.ranges_by_id[e];
    ((T*)a.w)[p] = (T)w;
    a.ends[p] = make_int2(ia, ib);
}

__global__ void k_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

}  // namespace

lsl_status launch_prep(int dtype, const PrepArgs& a, hipStream_t st) {
    if (a.n_edges == 0) return LSL_OK;
    const unsigned g = (unsigned)((a.n_edges + 255) / 256);
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
