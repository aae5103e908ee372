// Shared definitions of the native slicer: device records, wave primitives
// and the internal launcher API between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "lsl.h"

namespace lsl {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlockPix = 8;       // a wave evaluates one 8x8 pixel block

// ---------------------------------------------------------------------------
// Per-strut records, in edge-list order (ascending z of the lower end; with
// per-strut supports, ascending first slab, then z).
// ---------------------------------------------------------------------------
// One strut: its ends a = v_s and b = v_e as given (the kernels form the
// direction and length in float64), the folded weight wq = r / R^4 (the
// Gaussian kernel: r exp(-R^2 / 2 sigma^2)) and, with per-strut supports,
// its support R in pad.
template <typename T>
struct alignas(16) StrutRec {
    T ax, ay, az, wq;
    T bx, by, bz, pad;
};

// Slab and tile ranges of a strut's swept box (inclusive).
struct SRange {
    uint16_t tx0, tx1, ty0, ty1;
    int32_t s0, s1;
};

// The binning groups a tile row's columns in segments of this many tiles.
constexpr int kSegTiles = 8;

// (slab, tile row, column segment) cells of a box, per slab
__host__ __device__ inline uint32_t row_segments(const SRange& r) {
    return (uint32_t)(r.ty1 - r.ty0 + 1) * (uint32_t)(r.tx1 / kSegTiles - r.tx0 / kSegTiles + 1);
}

// The pixel columns, rows and planes of the same box (inclusive; the
// binning's integers, from which the tile and slab ranges follow).
struct PRange {
    uint16_t i0, i1, j0, j1;
    int32_t k0, k1;
};

// One staged (strut, plane) pair as a wave reads it from LDS: everything a
// pixel needs, expressed around the 8x8 block centre c of that plane.
//   m = F - c with F the foot of c on the strut's line; tc = (c - a).u
//   H0 = R^2 - |m|^2; the ends sit at -tc and L - tc from F along u.
template <typename T>
struct alignas(16) Stage {
    T mx2, my2, ux, uy;   // 2 m_x, 2 m_y, u_x, u_y
    T ntc, nbtc, H0, wq;  // -tc, L - tc, H0, r / R^4
};

// Direction and length of a strut in float64.
struct Line {
    double ux, uy, uz, L;
};
template <typename T>
__device__ __forceinline__ Line strut_line(const StrutRec<T>& r) {
    const double dx = (double)r.bx - (double)r.ax, dy = (double)r.by - (double)r.ay,
                 dz = (double)r.bz - (double)r.az;
    const double L = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
    const double inv = 1.0 / L;
    return Line{dx * inv, dy * inv, dz * inv, L};
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Blocks are handed to the 8 XCDs round-robin; remap so that each XCD works
// on one contiguous range of logical blocks (neighbouring tiles share L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
    const uint32_t per = n / 8u, rem = n % 8u;
    const uint32_t x = b % 8u, i = b / 8u;
    return x < rem ? x * (per + 1u) + i : rem * (per + 1u) + (x - rem) * per + i;
}

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* last_error();

#define LSL_HIP(call)                                                         \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            ::lsl::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return LSL_EDEVICE;                                               \
        }                                                                     \
    } while (0)

#define LSL_TRY(call)                                                         \
    do {                                                                      \
        lsl_status s_ = (call);                                               \
        if (s_ != LSL_OK) return s_;                                          \
    } while (0)

// ---------------------------------------------------------------------------
// Primitives (primitives.hip)
// ---------------------------------------------------------------------------
// Exclusive prefix sum of n values; out may alias in.  tmp must hold
// scan_tmp_elems(n) elements of the same type.  Writes the total to
// *total_dev when non-null.
size_t scan_tmp_elems(size_t n);
lsl_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t n,
                              uint32_t* tmp, uint32_t* total_dev, hipStream_t st);
lsl_status exclusive_scan_u64(const uint64_t* in, uint64_t* out, size_t n,
                              uint64_t* tmp, uint64_t* total_dev, hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on key bits [0, key_bits).
// Input in (k0, v0); (k1, v1) are equal-sized alternates.  Returns in *which
// 0 if the result is in (k0, v0), 1 if in (k1, v1).  tmp must hold
// radix_tmp_elems(n) uint32 elements.
size_t radix_tmp_elems(size_t n);
lsl_status radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                            size_t n, int key_bits, uint32_t* tmp, int* which,
                            hipStream_t st);

lsl_status fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
lsl_status fill_bytes0(void* p, size_t bytes, hipStream_t st);
lsl_status iota_u32(uint32_t* p, uint32_t base, size_t n, hipStream_t st);

}  // namespace lsl
