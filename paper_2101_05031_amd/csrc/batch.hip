// Persistent field kernel for batched slicing.  The paper notes that slicing
// time follows the number of struts meeting a plane (Sec. 6.4), so planes
// and tiles carry very uneven work.  Work items are (slab, tile) buckets; a
// queue orders them by descending cost (bucket length x planes, in 256
// logarithmic classes; a stable sort keeps tiles of one class in spatial
// order), and a grid sized to the GPU's occupancy pulls items from it with
// one atomic counter until the queue is drained.  Every block leaves the loop
// once the counter passes the item count, so the grid always drains.
#include <type_traits>

#include "field_block.hpp"
#include "field_q32.hpp"

namespace lsl {
namespace {

__global__ void k_queue_keys(FieldArgs a, uint32_t n_items, uint32_t* keys, uint32_t* vals) {
    const uint32_t it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= n_items) return;
    uint32_t t = it;
    const uint32_t tx = t % (uint32_t)a.ntx;
    t /= (uint32_t)a.ntx;
    const uint32_t ty = t % (uint32_t)a.nty;
    t /= (uint32_t)a.nty;
    const int slab = a.s_lo + (int)t;
    int kb = slab * a.slab, ke = kb + a.slab;
    if (kb < a.k0) kb = a.k0;
    if (ke > a.k0 + a.nk) ke = a.k0 + a.nk;
    const uint32_t bucket = ((uint32_t)(slab - a.group_s0) * (uint32_t)a.nty + ty) *
                                (uint32_t)a.ntx + tx;
    const uint32_t len = a.offsets[bucket + 1] - a.offsets[bucket];
    const float cost = (float)len * (float)(ke - kb);
    int cls = (int)(8.0f * __log2f(1.0f + cost));
    cls = cls < 0 ? 0 : (cls > 255 ? 255 : cls);
    keys[it] = 255u - (uint32_t)cls;          // descending cost
    vals[it] = it;
}

template <typename T, int SZ, int K, bool SR, bool PR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_persistent(FieldArgs a, const uint32_t* queue,
                                                    uint32_t n_items, uint32_t* counter) {
    __shared__ uint32_t s_item;
    const int wv = threadIdx.x >> 6;
    const int nsub = a.tile / kBlockPix;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t q = s_item;
        __syncthreads();
        if (q >= n_items) break;
        uint32_t t = queue[q];
        const int tx = (int)(t % (uint32_t)a.ntx);
        t /= (uint32_t)a.ntx;
        const int ty = (int)(t % (uint32_t)a.nty);
        t /= (uint32_t)a.nty;
        if constexpr (std::is_same<T, float>::value && K == LSL_KERNEL_QUARTIC && !PR) {
            __shared__ q32::Lds<SZ> lds[4];
            for (int sub = wv; sub < nsub * nsub; sub += 4)
                q32::field_block<SZ, false, SR>(a, a.s_lo + (int)t, tx, ty, sub, lds[wv]);
        } else {
            __shared__ Stage<T> stage[4][kWave];
            __shared__ T pend[4][fieldk::pend_elems<T, SZ>()];
            __shared__ double line[4][fieldk::kLineVals * kWave];
            for (int sub = wv; sub < nsub * nsub; sub += 4)
                fieldk::field_block<T, SZ, false, K, SR>(a, a.s_lo + (int)t, tx, ty, sub,
                                                         stage[wv], pend[wv], line[wv]);
        }
    }
}

template <typename T, int SZ>
int blocks_t() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, k_persistent<T, SZ, LSL_KERNEL_QUARTIC, false, false>, 256, 0) !=
        hipSuccess)
        return 0;
    return cus * (per > 0 ? per : 1);
}

template <typename T>
int blocks_dt(int slab) {
    if (slab <= 1) return blocks_t<T, 1>();
    if (slab <= 2) return blocks_t<T, 2>();
    if (slab <= 4) return blocks_t<T, 4>();
    if (slab <= 8) return blocks_t<T, 8>();
    return blocks_t<T, 16>();
}

template <typename T, int K, bool SR, bool PR>
lsl_status persistent_dtkp(const BatchArgs& b, int n_blocks, hipStream_t st) {
    const int s = b.f.slab;
    if (s <= 1)
        k_persistent<T, 1, K, SR, PR><<<n_blocks, 256, 0, st>>>(b.f, b.queue, b.n_items, b.counter);
    else if (s <= 2)
        k_persistent<T, 2, K, SR, PR><<<n_blocks, 256, 0, st>>>(b.f, b.queue, b.n_items, b.counter);
    else if (s <= 4)
        k_persistent<T, 4, K, SR, PR><<<n_blocks, 256, 0, st>>>(b.f, b.queue, b.n_items, b.counter);
    else if (s <= 8)
        k_persistent<T, 8, K, SR, PR><<<n_blocks, 256, 0, st>>>(b.f, b.queue, b.n_items, b.counter);
    else
        k_persistent<T, 16, K, SR, PR><<<n_blocks, 256, 0, st>>>(b.f, b.queue, b.n_items,
                                                                 b.counter);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

template <typename T, int K, bool SR>
lsl_status persistent_dtk(const BatchArgs& b, int n_blocks, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value && K == LSL_KERNEL_QUARTIC) {
        if (b.f.plane_ref) return persistent_dtkp<T, K, SR, true>(b, n_blocks, st);
    }
    return persistent_dtkp<T, K, SR, false>(b, n_blocks, st);
}

template <typename T>
lsl_status persistent_dt(const BatchArgs& b, int n_blocks, hipStream_t st) {
    if (b.f.kernel == LSL_KERNEL_GAUSS)
        return b.f.strut_R ? persistent_dtk<T, LSL_KERNEL_GAUSS, true>(b, n_blocks, st)
                           : persistent_dtk<T, LSL_KERNEL_GAUSS, false>(b, n_blocks, st);
    return b.f.strut_R ? persistent_dtk<T, LSL_KERNEL_QUARTIC, true>(b, n_blocks, st)
                       : persistent_dtk<T, LSL_KERNEL_QUARTIC, false>(b, n_blocks, st);
}

}  // namespace

int persistent_blocks(int dtype, int slab) {
    return dtype == LSL_F32 ? blocks_dt<float>(slab) : blocks_dt<double>(slab);
}

lsl_status launch_queue_build(const FieldArgs& f, uint32_t* keys, uint32_t* vals,
                              uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n_items,
                              uint32_t* tmp, const uint32_t** queue_out, hipStream_t st) {
    k_queue_keys<<<(n_items + 255) / 256, 256, 0, st>>>(f, n_items, keys, vals);
    LSL_HIP(hipGetLastError());
    int which = 0;
    LSL_TRY(radix_sort_pairs(keys, vals, keys_alt, vals_alt, n_items, 8, tmp, &which, st));
    *queue_out = which ? vals_alt : vals;
    return LSL_OK;
}

lsl_status launch_persistent(int dtype, const BatchArgs& b, int n_blocks, hipStream_t st) {
    if (b.n_items == 0) return LSL_OK;
    if (n_blocks <= 0) n_blocks = 1024;
    return dtype == LSL_F32 ? persistent_dt<float>(b, n_blocks, st)
                            : persistent_dt<double>(b, n_blocks, st);
}

}  // namespace lsl
