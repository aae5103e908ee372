// Self-support metrics of a lattice (Sec. 5.2, Eqs. 11-14) and the gradient
// of Gamma with respect to node positions, for the vertex position
// optimisation of Sec. 5.2.
//
// Per edge j with unit direction u, length L and weight r (the radius the
// paper stores on the edge), c = u . t_P and theta = arccos |c| (Eq. 11); the
// edge is self-supported when theta <= alpha = pi/4.  Otherwise the risky part
// of its projected area 2 r L is the fraction g(theta), the paper's degree-5
// polynomial for alpha = pi/4 (Eq. 12).  Gamma = N / D with N the sum of
// r L g over unsupported edges and D the sum of r L (Eq. 13); Psi = 100 x
// supported length / total length (Eq. 14).  Zero-length edges add nothing.
//
// Gradient: dGamma/dv_e gets r [g u + g'(theta) dtheta/dc (t - c u) - Gamma u] / D
// from each unsupported edge (r [-Gamma u] / D from a supported one, whose g
// and g' are 0), dtheta/dc = -sign(c) / sqrt(1 - c^2), and v_s the opposite;
// the step of g at alpha has no derivative and is left out.
//
// Everything is float64.  The sums run in a fixed order (per block, then
// over blocks), and each node gathers its edges' contributions in edge order
// through a node -> (edge, end) incidence list, so results are bitwise
// repeatable.
#include "kernels.hpp"

namespace lsl {
namespace {

constexpr double kAlpha = 0.78539816339744830962;   // pi / 4
constexpr int kSThreads = 256;
constexpr int kSums = 5;          // N, D, supported length, length, supported count

__device__ __constant__ double kPoly[6] = {-0.02, -0.31, 1.44, -1.11, 0.58, -0.16};

__device__ __forceinline__ double g_of(double th) {
    double p = kPoly[5];
    for (int i = 4; i >= 0; --i) p = fma(p, th, kPoly[i]);
    return p;
}

__device__ __forceinline__ double g_prime(double th) {
    double p = 5.0 * kPoly[5];
    for (int i = 4; i >= 1; --i) p = fma(p, th, (double)i * kPoly[i]);
    return p;
}

template <typename T>
struct EdgeGeom {
    bool ok;
    double L, ux, uy, uz, c, th, r;
};

template <typename T>
__device__ __forceinline__ EdgeGeom<T> edge_geom(const T* nodes, const int32_t* edges,
                                                 const T* weight, int64_t n_nodes, int64_t j,
                                                 double tx, double ty, double tz, int* err) {
    EdgeGeom<T> e{};
    const int32_t a = edges[2 * j], b = edges[2 * j + 1];
    if (a < 0 || b < 0 || a >= n_nodes || b >= n_nodes) {
        atomicOr(err, 1);
        return e;
    }
    const double dx = (double)nodes[3 * (int64_t)b] - (double)nodes[3 * (int64_t)a];
    const double dy = (double)nodes[3 * (int64_t)b + 1] - (double)nodes[3 * (int64_t)a + 1];
    const double dz = (double)nodes[3 * (int64_t)b + 2] - (double)nodes[3 * (int64_t)a + 2];
    e.L = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
    e.r = (double)weight[j];
    if (!(e.L > 0.0)) return e;
    e.ok = true;
    e.ux = dx / e.L;
    e.uy = dy / e.L;
    e.uz = dz / e.L;
    e.c = fma(e.ux, tx, fma(e.uy, ty, e.uz * tz));
    e.th = acos(fmin(fabs(e.c), 1.0));
    return e;
}

__device__ __forceinline__ double block_sum(double v, double* sm) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) sm[w] = v;
    __syncthreads();
    return sm[0] + sm[1] + sm[2] + sm[3];
}

template <typename T>
__global__ __launch_bounds__(kSThreads) void k_support_sums(const T* nodes, const int32_t* edges,
                                                            const T* weight, int64_t n_nodes,
                                                            int64_t n_edges, double tx, double ty,
                                                            double tz, double* part, int* err) {
    __shared__ double sm[4];
    const int64_t j = (int64_t)blockIdx.x * kSThreads + threadIdx.x;
    double v[kSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < n_edges) {
        const EdgeGeom<T> e = edge_geom<T>(nodes, edges, weight, n_nodes, j, tx, ty, tz, err);
        if (e.ok) {
            const bool sup = e.th <= kAlpha;
            v[0] = sup ? 0.0 : e.r * e.L * g_of(e.th);
            v[1] = e.r * e.L;
            v[2] = sup ? e.L : 0.0;
            v[3] = e.L;
            v[4] = sup ? 1.0 : 0.0;
        }
    }
    for (int q = 0; q < kSums; ++q) {
        const double s = block_sum(v[q], sm);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * kSums + q] = s;
    }
}

// one block: thread t sums blocks t, t + 256, ... in order, then the block
__global__ __launch_bounds__(kSThreads) void k_support_final(const double* part, uint32_t nb,
                                                             double* out) {
    __shared__ double sm[4];
    for (int q = 0; q < kSums; ++q) {
        double v = 0.0;
        for (uint32_t b = threadIdx.x; b < nb; b += kSThreads) v += part[(size_t)b * kSums + q];
        const double s = block_sum(v, sm);
        if (threadIdx.x == 0) out[q] = s;
    }
}

// per edge: its contribution to dGamma/dv_e (v_s gets the opposite)
template <typename T>
__global__ void k_support_edge_grad(const T* nodes, const int32_t* edges, const T* weight,
                                    int64_t n_nodes, int64_t n_edges, double tx, double ty,
                                    double tz, const double* sums, double* te, int* err) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_edges) return;
    const EdgeGeom<T> e = edge_geom<T>(nodes, edges, weight, n_nodes, j, tx, ty, tz, err);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    const double D = sums[1];
    if (e.ok && D > 0.0) {
        const double gamma = sums[0] / D;
        double g = 0.0, s = 0.0;
        if (e.th > kAlpha) {
            g = g_of(e.th);
            const double sgn = e.c > 0.0 ? 1.0 : (e.c < 0.0 ? -1.0 : 0.0);
            s = g_prime(e.th) * (-sgn / sqrt(1.0 - e.c * e.c));
        }
        const double f = e.r / D;
        gx = f * ((g - gamma) * e.ux + s * (tx - e.c * e.ux));
        gy = f * ((g - gamma) * e.uy + s * (ty - e.c * e.uy));
        gz = f * ((g - gamma) * e.uz + s * (tz - e.c * e.uz));
    }
    te[3 * j] = gx;
    te[3 * j + 1] = gy;
    te[3 * j + 2] = gz;
}

__global__ void k_inc_keys(const int32_t* edges, int64_t n_edges, uint32_t* keys, uint32_t* vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_edges) return;
    keys[2 * j] = (uint32_t)edges[2 * j];            // v_s
    vals[2 * j] = (uint32_t)(2 * j);
    keys[2 * j + 1] = (uint32_t)edges[2 * j + 1];    // v_e
    vals[2 * j + 1] = (uint32_t)(2 * j + 1);
}

// off[n] = first sorted position whose node is >= n
__global__ void k_inc_offsets(const uint32_t* keys, uint32_t n, uint32_t n_nodes, uint32_t* off) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const uint32_t kprev = i == 0 ? 0u : keys[i - 1] + 1u;
    const uint32_t k = i == n ? n_nodes : keys[i];
    for (uint32_t b = kprev; b <= k && b <= n_nodes; ++b) off[b] = i;
}

template <typename T>
__global__ void k_support_gather(const uint32_t* off, const uint32_t* inc, const double* te,
                                 int64_t n_nodes, T* grad) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    double g[3] = {0.0, 0.0, 0.0};
    for (uint32_t i = off[v]; i < off[v + 1]; ++i) {
        const uint32_t x = inc[i];
        const double sgn = (x & 1u) ? 1.0 : -1.0;    // end v_e: +, v_s: -
        const double* t = te + 3 * (size_t)(x >> 1);
        g[0] += sgn * t[0];
        g[1] += sgn * t[1];
        g[2] += sgn * t[2];
    }
    grad[3 * v] = (T)g[0];
    grad[3 * v + 1] = (T)g[1];
    grad[3 * v + 2] = (T)g[2];
}

template <typename T>
lsl_status support_t(const SupportArgs& a, hipStream_t st) {
    const T* nodes = (const T*)a.nodes;
    const T* weight = (const T*)a.weight;
    const uint32_t nb = (uint32_t)((a.n_edges + kSThreads - 1) / kSThreads);
    if (a.n_edges > 0)
        k_support_sums<T><<<nb, kSThreads, 0, st>>>(nodes, a.edges, weight, a.n_nodes, a.n_edges,
                                                     a.t[0], a.t[1], a.t[2], a.part, a.err);
    k_support_final<<<1, kSThreads, 0, st>>>(a.part, a.n_edges > 0 ? nb : 0u, a.sums);
    LSL_HIP(hipGetLastError());
    if (!a.grad) return LSL_OK;
    const unsigned g = (unsigned)((a.n_edges + 255) / 256);
    if (a.n_edges > 0) {
        k_support_edge_grad<T><<<g, 256, 0, st>>>(nodes, a.edges, weight, a.n_nodes, a.n_edges,
                                                  a.t[0], a.t[1], a.t[2], a.sums, a.te, a.err);
        k_inc_keys<<<g, 256, 0, st>>>(a.edges, a.n_edges, a.k0, a.v0);
    }
    const size_t n2 = 2 * (size_t)a.n_edges;
    int which = 0;
    int bits = 0;
    while (bits < 32 && (1ull << bits) < (uint64_t)a.n_nodes) ++bits;
    LSL_TRY(radix_sort_pairs(a.k0, a.v0, a.k1, a.v1, n2, bits, a.tmp, &which, st));
    const uint32_t* ks = which ? a.k1 : a.k0;
    const uint32_t* vs = which ? a.v1 : a.v0;
    k_inc_offsets<<<(unsigned)((n2 + 1 + 255) / 256), 256, 0, st>>>(ks, (uint32_t)n2,
                                                                     (uint32_t)a.n_nodes, a.off);
    k_support_gather<T><<<(unsigned)((a.n_nodes + 255) / 256), 256, 0, st>>>(
        a.off, vs, a.te, a.n_nodes, (T*)a.grad);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

}  // namespace

size_t support_part_elems(int64_t n_edges) {
    return (size_t)((n_edges + kSThreads - 1) / kSThreads + 1) * kSums;
}

lsl_status launch_support(int dtype, const SupportArgs& a, hipStream_t st) {
    return dtype == LSL_F32 ? support_t<float>(a, st) : support_t<double>(a, st);
}

}  // namespace lsl
