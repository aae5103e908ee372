// lsl_slice: slices a lattice file through the C ABI alone (no Python).
//
//   lsl_slice <lattice file> <output file> <k0> <nk>
//
// Lattice file (little endian): "LSL1", int64 n_nodes, int64 n_edges,
// int32 dtype (0 float32, 1 float64), float64 R, C, x0, y0, dx, dy, z0, dz,
// int32 W, H, n_slices, then nodes [n_nodes][3], edges [n_edges][2] int32 and
// weights [n_edges] of the dtype.
//
// Output file: int64 nk, W, H, total segments; the field of planes
// k0 .. k0+nk-1 [nk][H][W] (dtype); the contour offsets [nk + 1] int64; the
// segments [total][4] float32; and dL/dr [n_edges] (dtype) for the loss
// L = sum of the field over those planes (slice_field_backward with a gradient
// of ones).  Exit status 0 on success; 1 bad arguments or unreadable files, 2
// bad or truncated lattice file, 3 device allocation or copy failed, 4 a
// library call failed (stderr has the library's message), 5 the output file
// could not be written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lsl.h"

namespace {

bool fail(const char* what, lsl_status s) {
    std::fprintf(stderr, "lsl_slice: %s: %s (%d): %s\n", what, lsl_status_string(s), (int)s,
                 lsl_last_error());
    return false;
}

template <typename T>
bool read_vec(std::FILE* f, std::vector<T>& v, size_t n) {
    v.resize(n);
    return std::fread(v.data(), sizeof(T), n, f) == n;
}

// A device buffer freed when it goes out of scope (every return path).
struct DevBuf {
    void* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1) == hipSuccess; }
};

// The bins handle, freed likewise.
struct BinsGuard {
    lattice_bins* b = nullptr;
    ~BinsGuard() { lattice_bins_free(b); }
};

// device copy of a host vector
template <typename T>
bool to_dev(DevBuf& d, const std::vector<T>& v) {
    if (!d.alloc(v.size() * sizeof(T))) return false;
    return v.empty() ||
           hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

template <typename T>
bool write_all(std::FILE* f, const T* p, size_t n) {
    return n == 0 || std::fwrite(p, sizeof(T), n, f) == n;
}

template <typename T>
int run(std::FILE* in, std::FILE* out, int64_t n_nodes, int64_t n_edges, int32_t dtype,
        const double* hdr, const int32_t* dims, int32_t k0, int32_t nk) {
    std::vector<T> nodes, weight;
    std::vector<int32_t> edges;
    if (!read_vec(in, nodes, 3 * (size_t)n_nodes) || !read_vec(in, edges, 2 * (size_t)n_edges) ||
        !read_vec(in, weight, (size_t)n_edges)) {
        std::fprintf(stderr, "lsl_slice: truncated lattice file\n");
        return 2;
    }
    DevBuf d_nodes, d_edges, d_weight;
    if (!to_dev(d_nodes, nodes) || !to_dev(d_edges, edges) || !to_dev(d_weight, weight)) {
        std::fprintf(stderr, "lsl_slice: device allocation or copy failed\n");
        return 3;
    }
    lsl_lattice L{};
    L.n_nodes = n_nodes;
    L.n_edges = n_edges;
    L.dtype = dtype;
    L.nodes = d_nodes.p;
    L.edges = (const int32_t*)d_edges.p;
    L.weight = d_weight.p;
    L.R = hdr[0];
    L.C = hdr[1];
    lsl_grid G{hdr[2], hdr[3], hdr[4], hdr[5], dims[0], dims[1], hdr[6], hdr[7], dims[2]};
    lsl_bin_params P{};
    BinsGuard bins;
    lsl_status s = lattice_bin(&L, &G, &P, &bins.b, nullptr);
    if (s != LSL_OK) return fail("lattice_bin", s), 4;

    const size_t plane = (size_t)G.W * (size_t)G.H;
    DevBuf field, offsets, ones, gw, segs;
    if (!field.alloc((size_t)nk * plane * sizeof(T)) ||
        !offsets.alloc(((size_t)nk + 1) * sizeof(int64_t)) ||
        !ones.alloc((size_t)nk * plane * sizeof(T)) ||
        !gw.alloc((size_t)std::max<int64_t>(n_edges, 1) * sizeof(T))) {
        std::fprintf(stderr, "lsl_slice: device allocation failed\n");
        return 3;
    }
    if ((s = slice_field(bins.b, k0, nk, field.p, nullptr, nullptr)) != LSL_OK)
        return fail("slice_field", s), 4;
    // contours: size the output first, then emit
    int64_t total = 0;
    s = slice_contours(bins.b, nk, field.p, nullptr, 0, (int64_t*)offsets.p, nullptr, &total,
                       nullptr);
    if (s != LSL_OK && s != LSL_ECAPACITY) return fail("slice_contours", s), 4;
    if (!segs.alloc((size_t)std::max<int64_t>(total, 1) * 4 * sizeof(float))) {
        std::fprintf(stderr, "lsl_slice: device allocation failed\n");
        return 3;
    }
    if ((s = slice_contours(bins.b, nk, field.p, (float*)segs.p, total, (int64_t*)offsets.p,
                            nullptr, &total, nullptr)) != LSL_OK)
        return fail("slice_contours", s), 4;
    // dL/dr for L = sum of the field: a gradient of ones
    std::vector<T> h_ones((size_t)nk * plane, T(1));
    if (hipMemcpy(ones.p, h_ones.data(), h_ones.size() * sizeof(T), hipMemcpyHostToDevice) !=
        hipSuccess) {
        std::fprintf(stderr, "lsl_slice: copy to device failed\n");
        return 3;
    }
    if ((s = slice_field_backward(bins.b, k0, nk, ones.p, gw.p, nullptr, 0, nullptr)) != LSL_OK)
        return fail("slice_field_backward", s), 4;

    std::vector<T> h_field((size_t)nk * plane), h_gw((size_t)n_edges);
    std::vector<int64_t> h_off((size_t)nk + 1);
    std::vector<float> h_segs((size_t)total * 4);
    if (hipMemcpy(h_field.data(), field.p, h_field.size() * sizeof(T), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(h_off.data(), offsets.p, h_off.size() * sizeof(int64_t),
                  hipMemcpyDeviceToHost) != hipSuccess ||
        (total && hipMemcpy(h_segs.data(), segs.p, h_segs.size() * sizeof(float),
                            hipMemcpyDeviceToHost) != hipSuccess) ||
        (n_edges && hipMemcpy(h_gw.data(), gw.p, h_gw.size() * sizeof(T),
                              hipMemcpyDeviceToHost) != hipSuccess)) {
        std::fprintf(stderr, "lsl_slice: copy to host failed\n");
        return 3;
    }
    const int64_t hdr_out[4] = {nk, G.W, G.H, total};
    if (!write_all(out, hdr_out, 4) || !write_all(out, h_field.data(), h_field.size()) ||
        !write_all(out, h_off.data(), h_off.size()) ||
        !write_all(out, h_segs.data(), h_segs.size()) ||
        !write_all(out, h_gw.data(), h_gw.size())) {
        std::fprintf(stderr, "lsl_slice: writing the output file failed\n");
        return 5;
    }
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 5) {
        std::fprintf(stderr, "usage: lsl_slice <lattice file> <output file> <k0> <nk>\n");
        return 1;
    }
    std::FILE* in = std::fopen(argv[1], "rb");
    if (!in) {
        std::fprintf(stderr, "lsl_slice: cannot open %s\n", argv[1]);
        return 1;
    }
    char magic[4];
    int64_t n_nodes = 0, n_edges = 0;
    int32_t dtype = 0;
    double hdr[8];
    int32_t dims[3];
    if (std::fread(magic, 1, 4, in) != 4 || std::memcmp(magic, "LSL1", 4) != 0 ||
        std::fread(&n_nodes, 8, 1, in) != 1 || std::fread(&n_edges, 8, 1, in) != 1 ||
        std::fread(&dtype, 4, 1, in) != 1 || std::fread(hdr, 8, 8, in) != 8 ||
        std::fread(dims, 4, 3, in) != 3 || n_nodes < 1 || n_edges < 0 ||
        (dtype != LSL_F32 && dtype != LSL_F64)) {
        std::fprintf(stderr, "lsl_slice: bad lattice file header\n");
        return 2;
    }
    const int32_t k0 = std::atoi(argv[3]), nk = std::atoi(argv[4]);
    if (k0 < 0 || nk < 1 || (int64_t)k0 + nk > (int64_t)dims[2]) {
        std::fprintf(stderr, "lsl_slice: planes [k0, k0+nk) must lie in [0, %d)\n", dims[2]);
        return 1;
    }
    std::FILE* out = std::fopen(argv[2], "wb");
    if (!out) {
        std::fprintf(stderr, "lsl_slice: cannot open %s\n", argv[2]);
        return 1;
    }
    int rc = dtype == LSL_F32 ? run<float>(in, out, n_nodes, n_edges, dtype, hdr, dims, k0, nk)
                              : run<double>(in, out, n_nodes, n_edges, dtype, hdr, dims, k0, nk);
    std::fclose(in);
    if (std::fclose(out) != 0 && rc == 0) {
        std::fprintf(stderr, "lsl_slice: closing the output file failed\n");
        rc = 5;
    }
    return rc;
}
