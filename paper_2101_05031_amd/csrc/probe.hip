// Throughput probes of the GPU's vector ALU, for the roofline of the field
// and adjoint kernels (diagnostics; not part of the slicing path).  Each
// mode runs 16 independent chains per lane over a grid of 16 blocks of 256
// per compute unit and reports the lane operations issued.
#include "field_block.hpp"

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

// The field kernel's per-pair sequence alone: 64 staged struts in LDS (as
// the field kernel stages them), every lane one pixel of an 8x8 block, the
// terms summed as the field kernel sums them (runs of Group<float>::n).
__global__ __launch_bounds__(256) void k_probe_term(float* out, int iters) {
    __shared__ Stage<float> st[4][kWave];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    Stage<float> e;
    e.mx2 = 0.02f * (float)(lane & 7);
    e.my2 = -0.03f * (float)(lane >> 3);
    e.ux = 0.6f;
    e.uy = 0.48f;
    e.ntc = -0.5f - 0.01f * (float)lane;
    e.nbtc = 1.5f + 0.01f * (float)lane;
    e.H0 = 1.9f - 0.005f * (float)lane;
    e.wq = 0.2f;
    st[wv][lane] = e;
    __syncthreads();
    const float dX = 0.05f * ((float)(lane & 7) - 3.5f), dY = 0.05f * ((float)(lane >> 3) - 3.5f);
    const float d2 = dX * dX + dY * dY;
    float s = 0.0f, c = 0.0f;
    constexpr int G = fieldk::Group<float>::n;
    static_assert(kWave % G == 0, "runs must tile the staged list");
    for (int i = 0; i < iters; ++i)
        for (int j = 0; j < kWave; j += G) {
            float g = fieldk::eval_term<float>(st[wv][j], dX, dY, d2);
#pragma unroll
            for (int q = 1; q < G; ++q) g += fieldk::eval_term<float>(st[wv][j + q], dX, dY, d2);
            fieldk::comp_add(g, s, c);
        }
    out[blockIdx.x * 256 + threadIdx.x] = s + c;
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
    // mode 4: one pair = one term; the others: one lane operation per chain step
    *lane_ops = (double)n * (double)iters * (mode == 4 ? (double)kWave : (double)kChains);
    return LSL_OK;
}
