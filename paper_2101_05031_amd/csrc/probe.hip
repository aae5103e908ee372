// Throughput probes of the GPU's vector ALU, for the roofline of the field
// and adjoint kernels (diagnostics; not part of the slicing path).  Each
// mode runs 16 independent chains per lane over a grid of 16 blocks of 256
// per compute unit and reports the lane operations issued.
#include "field_q32.hpp"

namespace lsl {
namespace {

constexpr int kChains = 16;

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(float* out, const float* bv, int iters, float sb,
                                               float sc) {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const float b = bv[threadIdx.x], c = bv[threadIdx.x + 256];
    float a[kChains];
#pragma unroll
    for (int q = 0; q < kChains; ++q) a[q] = 1e-3f * (float)(threadIdx.x + q);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < kChains; ++q) {
            if (MODE == 0) a[q] = __builtin_fmaf(b, c, a[q]);             // v_fmac_f32, VGPR operands
            if (MODE == 1) a[q] = __builtin_fmaf(a[q], sb, sc);           // v_fma_f32, SGPR operands
            if (MODE == 2) a[q] = __builtin_amdgcn_sqrtf(a[q]);           // v_sqrt_f32
            if (MODE == 5) a[q] = __builtin_fmaf(a[q], b, c);             // v_fma_f32, VGPR operands
            if (MODE == 6) a[q] = __builtin_amdgcn_fmed3f(a[q], -b, b);   // v_med3_f32 (a clamp)
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < kChains; ++q) s += a[q];
    out[gid] = s;
}

__global__ __launch_bounds__(256) void k_probe_f64(double* out, int iters, double sb, double sc) {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    double a[kChains];
#pragma unroll
    for (int q = 0; q < kChains; ++q) a[q] = 1e-3 * (double)(threadIdx.x + q);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int q = 0; q < kChains; ++q) a[q] = __builtin_fma(a[q], sb, sc);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kChains; ++q) s += a[q];
    out[gid] = s;
}

// The float32 field kernel's evaluation alone: every wave one 8x8 block, 64
// struts staged in LDS as the kernel stages them (a slab of 8 planes sharing
// one reference plane), each a candidate at every plane, the terms formed and
// summed by the kernel's own code (q32::add_candidate).  The staged values
// put every pixel inside every strut's support.
__global__ __launch_bounds__(256) void k_probe_term(float* out, int iters) {
    constexpr int SZ = 8;
    __shared__ q32::Lds<SZ> lds[4];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    q32::Lds<SZ>& L = lds[wv];
    for (int k = 0; k < SZ; ++k) L.pg[k][lane] = 0.6f - 0.01f * (float)k - 0.002f * (float)lane;
    L.gr[0][lane] = make_float4(-0.3f - 0.004f * (float)lane, 0.8f + 0.004f * (float)lane, 0.02f,
                                -0.03f);
    L.e[lane] = make_float4(0.35f, 0.28f, 0.01f, 0.44f);
    L.dl[lane] = -0.01f;
    L.cand[lane] = (uint32_t)lane | (0xffu << 8);
    __builtin_amdgcn_wave_barrier();
    const float dX = 0.05f * ((float)(lane & 7) - 3.5f), dY = 0.05f * ((float)(lane >> 3) - 3.5f);
    const float nd2 = -(dX * dX + dY * dY);
    float acc_s[SZ], acc_c[SZ], run[SZ];
    int open[SZ];
    q32::for_planes<0, SZ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        acc_s[k] = acc_c[k] = run[k] = 0.0f;
        open[k] = 0;
    });
    unsigned long long n_cand = 0, n_useful = 0;
    for (int i = 0; i < iters; ++i) {
        uint32_t c = L.cand[0];
        float4 E = L.e[c & 63u];
        float nD = L.dl[c & 63u];
#pragma unroll 1
        for (int j = 0; j < kWave; ++j) {
            const uint32_t e = c & 63u;
            const uint32_t mask = __builtin_amdgcn_readfirstlane(c >> 8);
            float Gk[SZ];
            q32::for_planes<0, SZ>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                Gk[k] = L.pg[k][e];
            });
            const uint32_t cn = L.cand[j + 1 < kWave ? j + 1 : j];
            const float4 En = L.e[cn & 63u];
            const float nDn = L.dl[cn & 63u];
            q32::add_candidate<SZ, false>(L, e, mask, E, nD, 0, 0, Gk, dX, dY, nd2, true,
                                                 acc_s, acc_c, run, open, n_cand, n_useful);
            c = cn;
            E = En;
            nD = nDn;
        }
    }
    float t = 0.0f;
    q32::for_planes<0, SZ>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        t += acc_s[k] + acc_c[k] + run[k];
    });
    out[blockIdx.x * 256 + threadIdx.x] = t;
}

}  // namespace
}  // namespace lsl

extern "C" lsl_status lsl_probe_valu(int32_t mode, int32_t iters, float* ms, double* lane_ops,
                                     void* stream) {
    using namespace lsl;
    set_error("");
    if (mode < 0 || mode > 6 || iters < 1 || !ms || !lane_ops) {
        set_error("lsl_probe_valu: mode in [0, 6], iters >= 1, ms and lane_ops required");
        return LSL_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 0;
    LSL_HIP(hipGetDevice(&dev));
    LSL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = 16 * cus;
    const size_t n = (size_t)blocks * 256;
    void* buf = nullptr;
    float* bv = nullptr;
    LSL_HIP(hipMalloc(&buf, n * sizeof(double)));
    if (hipMalloc(&bv, 512 * sizeof(float)) != hipSuccess) {
        hipFree(buf);
        set_error("lsl_probe_valu: out of device memory");
        return LSL_ENOMEM;
    }
    float h[512];
    for (int i = 0; i < 512; ++i) h[i] = i < 256 ? 0.9999f : 1e-4f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipMemcpyAsync(bv, h, sizeof(h), hipMemcpyHostToDevice, st);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    if (err == hipSuccess) {
        if (mode == 0) k_probe<0><<<blocks, 256, 0, st>>>((float*)buf, bv, iters, 0.9999f, 1e-4f);
        if (mode == 1) k_probe<1><<<blocks, 256, 0, st>>>((float*)buf, bv, iters, 0.9999f, 1e-4f);
        if (mode == 2) k_probe<2><<<blocks, 256, 0, st>>>((float*)buf, bv, iters, 0.9999f, 1e-4f);
        if (mode == 3) k_probe_f64<<<blocks, 256, 0, st>>>((double*)buf, iters, 0.9999, 1e-4);
        if (mode == 4) k_probe_term<<<blocks, 256, 0, st>>>((float*)buf, iters);
        if (mode == 5) k_probe<5><<<blocks, 256, 0, st>>>((float*)buf, bv, iters, 0.9999f, 1e-4f);
        if (mode == 6) k_probe<6><<<blocks, 256, 0, st>>>((float*)buf, bv, iters, 0.9999f, 1e-4f);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(bv);
    hipFree(buf);
    if (err != hipSuccess) {
        set_error(std::string("lsl_probe_valu: ") + hipGetErrorString(err));
        return LSL_EDEVICE;
    }
    *ms = t;
    // mode 4: one pair = one term (64 struts x 8 planes per lane and
    // iteration); the others: one lane operation per chain step
    *lane_ops = (double)n * (double)iters * (mode == 4 ? (double)kWave * 8.0 : (double)kChains);
    return LSL_OK;
}
