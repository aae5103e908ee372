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
// of ones).  Exit status 0 on success; errors go to stderr with the library's
// message.
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

// device copy of a host vector
template <typename T>
void* to_dev(const std::vector<T>& v) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(v.size(), 1) * sizeof(T)) != hipSuccess) return nullptr;
    if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) !=
                          hipSuccess)
        return nullptr;
    return p;
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
    lsl_lattice L{};
    L.n_nodes = n_nodes;
    L.n_edges = n_edges;
    L.dtype = dtype;
    L.nodes = to_dev(nodes);
    L.edges = (const int32_t*)to_dev(edges);
    L.weight = to_dev(weight);
    L.R = hdr[0];
    L.C = hdr[1];
    if (!L.nodes || !L.edges || !L.weight) {
        std::fprintf(stderr, "lsl_slice: device allocation failed\n");
        return 3;
    }
    lsl_grid G{hdr[2], hdr[3], hdr[4], hdr[5], dims[0], dims[1], hdr[6], hdr[7], dims[2]};
    lsl_bin_params P{};
    lattice_bins* bins = nullptr;
    lsl_status s = lattice_bin(&L, &G, &P, &bins, nullptr);
    if (s != LSL_OK) return fail("lattice_bin", s), 4;

    const size_t plane = (size_t)G.W * (size_t)G.H;
    void* field = nullptr;
    int64_t* offsets = nullptr;
    void* ones = nullptr;
    void* gw = nullptr;
    if (hipMalloc(&field, (size_t)nk * plane * sizeof(T)) != hipSuccess ||
        hipMalloc((void**)&offsets, ((size_t)nk + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&ones, (size_t)nk * plane * sizeof(T)) != hipSuccess ||
        hipMalloc(&gw, std::max<int64_t>(n_edges, 1) * sizeof(T)) != hipSuccess) {
        std::fprintf(stderr, "lsl_slice: device allocation failed\n");
        return 3;
    }
    if ((s = slice_field(bins, k0, nk, field, nullptr, nullptr)) != LSL_OK)
        return fail("slice_field", s), 4;
    // contours: size the output first, then emit
    int64_t total = 0;
    s = slice_contours(bins, nk, field, nullptr, 0, offsets, nullptr, &total, nullptr);
    if (s != LSL_OK && s != LSL_ECAPACITY) return fail("slice_contours", s), 4;
    float* segs = nullptr;
    if (hipMalloc((void**)&segs, std::max<int64_t>(total, 1) * 4 * sizeof(float)) != hipSuccess)
        return 3;
    if ((s = slice_contours(bins, nk, field, segs, total, offsets, nullptr, &total, nullptr)) !=
        LSL_OK)
        return fail("slice_contours", s), 4;
    // dL/dr for L = sum of the field: a gradient of ones
    std::vector<T> h_ones((size_t)nk * plane, T(1));
    if (hipMemcpy(ones, h_ones.data(), h_ones.size() * sizeof(T), hipMemcpyHostToDevice) !=
        hipSuccess)
        return 3;
    if ((s = slice_field_backward(bins, k0, nk, ones, gw, nullptr, 0, nullptr)) != LSL_OK)
        return fail("slice_field_backward", s), 4;

    std::vector<T> h_field((size_t)nk * plane), h_gw((size_t)n_edges);
    std::vector<int64_t> h_off((size_t)nk + 1);
    std::vector<float> h_segs((size_t)total * 4);
    if (hipMemcpy(h_field.data(), field, h_field.size() * sizeof(T), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(h_off.data(), offsets, h_off.size() * sizeof(int64_t), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        (total && hipMemcpy(h_segs.data(), segs, h_segs.size() * sizeof(float),
                            hipMemcpyDeviceToHost) != hipSuccess) ||
        (n_edges && hipMemcpy(h_gw.data(), gw, h_gw.size() * sizeof(T), hipMemcpyDeviceToHost) !=
                        hipSuccess)) {
        std::fprintf(stderr, "lsl_slice: copy to host failed\n");
        return 3;
    }
    const int64_t hdr_out[4] = {nk, G.W, G.H, total};
    std::fwrite(hdr_out, sizeof(int64_t), 4, out);
    std::fwrite(h_field.data(), sizeof(T), h_field.size(), out);
    std::fwrite(h_off.data(), sizeof(int64_t), h_off.size(), out);
    std::fwrite(h_segs.data(), sizeof(float), h_segs.size(), out);
    std::fwrite(h_gw.data(), sizeof(T), h_gw.size(), out);

    lattice_bins_free(bins);
    for (void* p : {(void*)L.nodes, (void*)L.edges, (void*)L.weight, field, (void*)offsets, ones,
                    gw, (void*)segs})
        (void)hipFree(p);
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
    std::FILE* out = std::fopen(argv[2], "wb");
    if (!out) {
        std::fprintf(stderr, "lsl_slice: cannot open %s\n", argv[2]);
        return 1;
    }
    const int rc = dtype == LSL_F32 ? run<float>(in, out, n_nodes, n_edges, dtype, hdr, dims, k0, nk)
                                    : run<double>(in, out, n_nodes, n_edges, dtype, hdr, dims, k0,
                                                  nk);
    std::fclose(in);
    std::fclose(out);
    return rc;
}
