// Per-voxel density of the sliced solid (Sec. 5, Eq. 9), a smooth
// voxel-density loss for the radius adjustment of Sec. 5.3, and the per-pixel
// soft-occupancy loss of a sliced field (the same loss with one-sample voxels,
// without the per-voxel pass).
//
// The density of a voxel is the fraction of its samples inside the solid,
// g >= C, the samples being the pixel centres of the slice planes (a
// stratified Monte-Carlo sample on the slicing grid).  Voxel (l, j, i) holds
// planes [l vz, (l+1) vz), rows [j vy, (j+1) vy) and columns [i vx, (i+1) vx)
// of the given field, clipped at its last plane, row and column.
//
// The loss variant replaces the inside test by s = sigmoid((g - C) / tau),
// averages s per voxel, and returns L = sum_v (s_v - target_v)^2 together with
// dL/dg(p) = 2 (s_v - target_v) / n_v * s (1 - s) / tau per pixel (n_v the
// voxel's sample count), the input of the field adjoint.
//
// Work layout.  A 256-thread block owns whole voxels: vpb = 256 / vx
// consecutive voxel columns of one voxel row and layer (one voxel when
// vx > 256).  Thread t owns pixel column xa + t (and xa + t + 256 q when the
// voxel is wider than 256) and walks the voxel's planes and rows, so each
// load of a wave reads 64 consecutive values of one row, the field is read
// once, and no atomics are needed.  Column totals are summed per voxel through
// LDS in a fixed pairwise tree, so every result is bitwise repeatable.
#include "kernels.hpp"

namespace lsl {
namespace {

constexpr int kDThreads = 256;
constexpr int kRowBatch = 8;     // loads in flight per thread

// sigmoid(z) and sigmoid'(z) = s (1 - s) from e = exp(-|z|), which neither
// overflows nor loses 1 - s to cancellation.  float: the hardware exp2 and
// reciprocal (relative errors ~|z| 6e-8 and 1 ulp), since the float32 argument
// z already carries an error of that size; double: correctly rounded
// operations.
__device__ __forceinline__ float sigm(float z) {
    const float e = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    return z >= 0.0f ? r : e * r;
}
__device__ __forceinline__ float sigm_prime(float z) {
    const float e = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    return e * r * r;
}
__device__ __forceinline__ double sigm(double z) {
    const double e = exp(-fabs(z));
    const double d = 1.0 + e;
    return z >= 0.0 ? 1.0 / d : e / d;
}
__device__ __forceinline__ double sigm_prime(double z) {
    const double e = exp(-fabs(z));
    const double d = 1.0 + e;
    return e / (d * d);
}

// sigmoid(z) and its derivative from one exponential
__device__ __forceinline__ void sigm_both(float z, float& s, float& sp) {
    const float e = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    s = z >= 0.0f ? r : e * r;
    sp = e * r * r;
}
__device__ __forceinline__ void sigm_both(double z, double& s, double& sp) {
    const double e = exp(-fabs(z));
    const double d = 1.0 + e;
    s = z >= 0.0 ? 1.0 / d : e / d;
    sp = e / (d * d);
}

struct Box {
    int32_t l, j, ia, ib;          // voxel layer, row, columns [ia, ib)
    int32_t ka, kb, ya, yb;        // planes and rows
    int64_t xa, xb;                // pixel columns
};

__device__ __forceinline__ Box block_box(const DensityArgs& a, uint32_t b) {
    Box x;
    const uint32_t bx = b % (uint32_t)a.nbx, r = b / (uint32_t)a.nbx;
    x.j = (int32_t)(r % (uint32_t)a.ny);
    x.l = (int32_t)(r / (uint32_t)a.ny);
    x.ia = (int32_t)bx * a.vpb;
    x.ib = min(a.nx, x.ia + a.vpb);
    x.ka = x.l * a.vz;
    x.kb = min(a.nk, x.ka + a.vz);
    x.ya = x.j * a.vy;
    x.yb = min(a.H, x.ya + a.vy);
    x.xa = (int64_t)x.ia * a.vx;
    x.xb = min((int64_t)a.W, (int64_t)x.ib * a.vx);
    return x;
}

// samples in voxel column i of the box
__device__ __forceinline__ double box_samples(const DensityArgs& a, const Box& x, int32_t i) {
    const int64_t c0 = (int64_t)i * a.vx, c1 = min((int64_t)a.W, c0 + a.vx);
    return (double)(x.kb - x.ka) * (double)(x.yb - x.ya) * (double)(c1 - c0);
}

// The thread's column total of f(g) over the box's planes and rows, in a fixed
// order: columns, then planes, then rows; each batch of rows is summed in Part
// before it is added to the total in Acc.
template <typename T, typename Acc, typename Part, typename F>
__device__ __forceinline__ Acc column_total(const T* field, const DensityArgs& a, const Box& x,
                                            F f) {
    Acc acc = Acc(0);
    const size_t W = (size_t)a.W;
    for (int64_t c = x.xa + threadIdx.x; c < x.xb; c += kDThreads) {
        for (int32_t k = x.ka; k < x.kb; ++k) {
            const T* p = field + ((size_t)k * (size_t)a.H + (size_t)x.ya) * W + (size_t)c;
            int32_t y = x.ya;
            for (; y + kRowBatch <= x.yb; y += kRowBatch) {
                T v[kRowBatch];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) v[q] = p[(size_t)q * W];
                Part part = f(v[0]);
#pragma unroll
                for (int q = 1; q < kRowBatch; ++q) part += f(v[q]);
                acc += (Acc)part;
                p += kRowBatch * W;
            }
            for (; y < x.yb; ++y, p += W) acc += (Acc)f(*p);
        }
    }
    return acc;
}

// After each thread has put its column total in col[t]: col[v * vxs] holds the
// total of voxel v of the block (vxs = min(vx, 256)), by a pairwise tree.
__device__ __forceinline__ void voxel_tree(double* col, int32_t vxs) {
    const int t = threadIdx.x;
    const int o = t % vxs;
    __syncthreads();
    for (int s = 1; s < vxs; s <<= 1) {
        if ((o & (2 * s - 1)) == 0 && o + s < vxs && t + s < kDThreads) col[t] += col[t + s];
        __syncthreads();
    }
}

// fixed-order total of v over the block (every thread gets it)
__device__ __forceinline__ double block_total(double v, double* sm) {
    const int t = threadIdx.x;
    __syncthreads();
    sm[t] = v;
    __syncthreads();
    for (int s = kDThreads / 2; s >= 1; s >>= 1) {
        if (t < s) sm[t] += sm[t + s];
        __syncthreads();
    }
    return sm[0];
}

template <typename T>
__global__ __launch_bounds__(kDThreads) void k_density(const T* field, DensityArgs a, T C,
                                                       float* out) {
    __shared__ double col[kDThreads];
    const Box x = block_box(a, blockIdx.x);
    const uint64_t n = column_total<T, uint64_t, uint32_t>(field, a, x, [C](T g) -> uint32_t {
        return g >= C ? 1u : 0u;
    });
    col[threadIdx.x] = (double)n;          // exact: sample counts stay below 2^53
    const int32_t vxs = min(a.vx, kDThreads);
    voxel_tree(col, vxs);
    const int v = threadIdx.x;
    if (v < x.ib - x.ia) {
        const int32_t i = x.ia + v;
        const double frac = col[v * vxs] / box_samples(a, x, i);
        out[((size_t)x.l * (size_t)a.ny + (size_t)x.j) * (size_t)a.nx + (size_t)i] = (float)frac;
    }
}

// soft voxel densities, residuals s_v - target_v and the block's sum of
// squared residuals
template <typename T>
__global__ __launch_bounds__(kDThreads) void k_soft_density(const T* field, DensityArgs a, T C,
                                                            T inv_tau, const float* target,
                                                            float* soft, double* resid,
                                                            double* part) {
    __shared__ double col[kDThreads];
    const Box x = block_box(a, blockIdx.x);
    const double s = column_total<T, double, T>(field, a, x, [C, inv_tau](T g) -> T {
        return sigm((g - C) * inv_tau);
    });
    col[threadIdx.x] = s;
    const int32_t vxs = min(a.vx, kDThreads);
    voxel_tree(col, vxs);
    const int v = threadIdx.x;
    double r2 = 0.0;
    if (v < x.ib - x.ia) {
        const int32_t i = x.ia + v;
        const size_t idx = ((size_t)x.l * (size_t)a.ny + (size_t)x.j) * (size_t)a.nx + (size_t)i;
        const double d = col[v * vxs] / box_samples(a, x, i);
        const double r = d - (double)target[idx];
        if (soft) soft[idx] = (float)d;
        resid[idx] = r;
        r2 = r * r;
    }
    const double tot = block_total(r2, col);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// one block: thread t sums partials t, t + 256, ... in four interleaved
// chains (fixed order), then the block total
__global__ __launch_bounds__(kDThreads) void k_loss_final(const double* part, uint32_t nb,
                                                          double* loss) {
    __shared__ double sm[kDThreads];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t b = threadIdx.x;
    for (; b + 3 * kDThreads < nb; b += 4 * kDThreads) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += part[b + q * kDThreads];
    }
    for (int q = 0; b < nb; b += kDThreads, ++q) v[q] += part[b];
    const double tot = block_total((v[0] + v[1]) + (v[2] + v[3]), sm);
    if (threadIdx.x == 0) *loss = tot;
}

// dL/dg per pixel; every pixel of the field lies in exactly one block's box.
// The gradient is written once and not read back here: streaming stores.
template <typename T>
__global__ __launch_bounds__(kDThreads) void k_density_grad(const T* field, DensityArgs a, T C,
                                                            T inv_tau, double tau,
                                                            const double* resid, T* grad) {
    const Box x = block_box(a, blockIdx.x);
    const size_t W = (size_t)a.W;
    for (int64_t c = x.xa + threadIdx.x; c < x.xb; c += kDThreads) {
        const int32_t i = (int32_t)(c / a.vx);
        const size_t idx = ((size_t)x.l * (size_t)a.ny + (size_t)x.j) * (size_t)a.nx + (size_t)i;
        const T coef = (T)(2.0 * resid[idx] / (box_samples(a, x, i) * tau));
        for (int32_t k = x.ka; k < x.kb; ++k) {
            const size_t base = ((size_t)k * (size_t)a.H + (size_t)x.ya) * W + (size_t)c;
            const T* p = field + base;
            T* o = grad + base;
            int32_t y = x.ya;
            for (; y + kRowBatch <= x.yb; y += kRowBatch) {
                T v[kRowBatch];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) v[q] = p[(size_t)q * W];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q)
                    __builtin_nontemporal_store(coef * sigm_prime((v[q] - C) * inv_tau),
                                                o + (size_t)q * W);
                p += kRowBatch * W;
                o += kRowBatch * W;
            }
            for (; y < x.yb; ++y, p += W, o += W)
                __builtin_nontemporal_store(coef * sigm_prime((*p - C) * inv_tau), o);
        }
    }
}

// Per-pixel soft-occupancy loss: L = sum_p (s_p - t_p)^2, s = sigmoid((g - C)
// / tau), and dL/dg = 2 (s - t) s' / tau, in one pass over field and target.
// A fixed grid walks the pixels with a fixed stride, four loads in flight per
// thread; each block writes its sum of squares, so the total has a fixed order.
constexpr int kOccUnroll = 4;

template <typename T>
__global__ __launch_bounds__(kDThreads) void k_occupancy_loss(const T* field, const T* target,
                                                              size_t n, T C, T inv_tau,
                                                              T two_over_tau, T* grad,
                                                              double* part) {
    __shared__ double sm[kDThreads];
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * kDThreads;
    for (size_t i0 = (size_t)blockIdx.x * kDThreads + threadIdx.x; i0 < n;
         i0 += kOccUnroll * stride) {
        T g[kOccUnroll], t[kOccUnroll];
#pragma unroll
        for (int q = 0; q < kOccUnroll; ++q) {
            const size_t i = i0 + (size_t)q * stride;
            g[q] = i < n ? field[i] : C;
            t[q] = i < n ? target[i] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kOccUnroll; ++q) {
            const size_t i = i0 + (size_t)q * stride;
            if (i < n) {
                T sv, sp;
                sigm_both((g[q] - C) * inv_tau, sv, sp);
                const T r = sv - t[q];
                if (grad) __builtin_nontemporal_store(two_over_tau * r * sp, grad + i);
                acc += (double)r * (double)r;
            }
        }
    }
    const double tot = block_total(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
lsl_status occupancy_t(const void* field, const void* target, size_t n, double C, double tau,
                       void* grad, double* loss, double* part, uint32_t nb, hipStream_t st) {
    k_occupancy_loss<T><<<nb, kDThreads, 0, st>>>((const T*)field, (const T*)target, n, (T)C,
                                                  (T)(1.0 / tau), (T)(2.0 / tau), (T*)grad, part);
    if (loss) k_loss_final<<<1, kDThreads, 0, st>>>(part, nb, loss);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

template <typename T>
lsl_status density_t(const DensityArgs& a, const void* field, double C, float* out,
                     hipStream_t st) {
    k_density<T><<<a.n_blocks, kDThreads, 0, st>>>((const T*)field, a, (T)C, out);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

template <typename T>
lsl_status loss_t(const DensityArgs& a, const void* field, double C, double tau,
                  const float* target, float* soft, void* grad, double* loss, double* scratch,
                  hipStream_t st) {
    double* resid = scratch;
    double* part = scratch + density_voxels(a);
    const T inv_tau = (T)(1.0 / tau);
    k_soft_density<T><<<a.n_blocks, kDThreads, 0, st>>>((const T*)field, a, (T)C, inv_tau, target,
                                                        soft, resid, part);
    if (loss) k_loss_final<<<1, kDThreads, 0, st>>>(part, a.n_blocks, loss);
    if (grad)
        k_density_grad<T><<<a.n_blocks, kDThreads, 0, st>>>((const T*)field, a, (T)C, inv_tau,
                                                            tau, resid, (T*)grad);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace

lsl_status density_plan(int32_t nk, int32_t W, int32_t H, int32_t vx, int32_t vy, int32_t vz,
                        DensityArgs* a) {
    if (nk < 1 || W < 1 || H < 1 || vx < 1 || vy < 1 || vz < 1) {
        set_error("density: sizes and voxel extents must be >= 1");
        return LSL_EINVAL;
    }
    // a voxel wider than the field is the same voxel clipped to it
    a->nk = nk;
    a->W = W;
    a->H = H;
    a->vx = std::min(vx, W);
    a->vy = std::min(vy, H);
    a->vz = std::min(vz, nk);
    a->nx = (W + a->vx - 1) / a->vx;
    a->ny = (H + a->vy - 1) / a->vy;
    a->nz = (nk + a->vz - 1) / a->vz;
    a->vpb = std::max(1, kDThreads / a->vx);
    a->nbx = (a->nx + a->vpb - 1) / a->vpb;
    const uint64_t nb = (uint64_t)a->nbx * (uint64_t)a->ny * (uint64_t)a->nz;
    if (nb > 0x7fffffffull) {
        set_error("density: too many voxel blocks in one call");
        return LSL_EINVAL;
    }
    a->n_blocks = (uint32_t)nb;
    return LSL_OK;
}

size_t density_voxels(const DensityArgs& a) {
    return (size_t)a.nx * (size_t)a.ny * (size_t)a.nz;
}

size_t density_scratch_elems(const DensityArgs& a) { return density_voxels(a) + a.n_blocks; }

lsl_status launch_density(int dtype, const DensityArgs& a, const void* field, double C,
                          float* out, hipStream_t st) {
    return dtype == LSL_F32 ? density_t<float>(a, field, C, out, st)
                            : density_t<double>(a, field, C, out, st);
}

uint32_t occupancy_blocks(size_t n) {
    const size_t b = (n + (size_t)kDThreads * kOccUnroll - 1) / ((size_t)kDThreads * kOccUnroll);
    return (uint32_t)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

lsl_status launch_occupancy_loss(int dtype, const void* field, const void* target, size_t n,
                                 double C, double tau, void* grad, double* loss, double* part,
                                 hipStream_t st) {
    const uint32_t nb = occupancy_blocks(n);
    return dtype == LSL_F32 ? occupancy_t<float>(field, target, n, C, tau, grad, loss, part, nb, st)
                            : occupancy_t<double>(field, target, n, C, tau, grad, loss, part, nb,
                                                  st);
}

lsl_status launch_density_loss(int dtype, const DensityArgs& a, const void* field, double C,
                               double tau, const float* target, float* soft, void* grad,
                               double* loss, double* scratch, hipStream_t st) {
    return dtype == LSL_F32
               ? loss_t<float>(a, field, C, tau, target, soft, grad, loss, scratch, st)
               : loss_t<double>(a, field, C, tau, target, soft, grad, loss, scratch, st);
}

}  // namespace lsl
