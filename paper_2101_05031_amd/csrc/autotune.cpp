// slice_autotune: picks the tile edge and slab depth for a lattice and grid
// by binning with each candidate (all slab groups, as one pass over the planes
// bins them) and timing the persistent field launch of slice_batch on a few
// sampled plane windows.  The field does not depend on the choice (every pixel sees the
// same struts in the same order), so only speed is compared.  Results are
// cached in a small JSON file keyed by the problem's shape.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace lsl;

namespace {

std::string shape_key(const lsl_lattice* L, const lsl_grid* G) {
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "E%lld_N%lld_d%d_W%d_H%d_S%d_R%.6g_dx%.6g_dy%.6g_dz%.6g_k%d_s%.6g_ps%d",
                  (long long)L->n_edges, (long long)L->n_nodes, L->dtype, G->W, G->H, G->n_slices,
                  L->R, G->dx, G->dy, G->dz, L->kernel, L->sigma, L->support ? 1 : 0);
    return buf;
}

// Reads {"key": {"tile": t, "slab": s}, ...}; returns false if key is absent.
bool cache_lookup(const char* path, const std::string& key, int* tile, int* slab) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const std::string q = "\"" + key + "\"";
    size_t p = s.find(q);
    if (p == std::string::npos) return false;
    size_t e = s.find('}', p);
    if (e == std::string::npos) return false;
    const std::string obj = s.substr(p, e - p);
    size_t pt = obj.find("\"tile\""), ps = obj.find("\"slab\"");
    if (pt == std::string::npos || ps == std::string::npos) return false;
    int t = 0, sl = 0;
    if (std::sscanf(obj.c_str() + obj.find(':', pt) + 1, "%d", &t) != 1) return false;
    if (std::sscanf(obj.c_str() + obj.find(':', ps) + 1, "%d", &sl) != 1) return false;
    *tile = t;
    *slab = sl;
    return true;
}

void cache_store(const char* path, const std::string& key, int tile, int slab) {
    std::string s;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            s = ss.str();
        }
    }
    const std::string entry = "\"" + key + "\": {\"tile\": " + std::to_string(tile) +
                              ", \"slab\": " + std::to_string(slab) + "}";
    size_t close = s.rfind('}');
    if (s.empty() || close == std::string::npos || s.find('{') == std::string::npos) {
        s = "{\n  " + entry + "\n}\n";
    } else {
        const bool empty = s.find('"') == std::string::npos;
        s = s.substr(0, close);
        while (!s.empty() && (s.back() == '\n' || s.back() == ' ')) s.pop_back();
        s += (empty ? "\n  " : ",\n  ") + entry + "\n}\n";
    }
    std::ofstream o(path);
    o << s;
}

}  // namespace

extern "C" lsl_status slice_autotune(const lsl_lattice* L, const lsl_grid* G,
                                     lsl_bin_params* P, const char* cache_path, void* stream) {
    set_error("");
    if (!L || !G || !P) {
        set_error("slice_autotune: NULL argument");
        return LSL_EINVAL;
    }
    const std::string key = shape_key(L, G);
    if (cache_path) {
        int t = 0, s = 0;
        if (cache_lookup(cache_path, key, &t, &s)) {
            if (!P->tile) P->tile = t;
            if (!P->slab) P->slab = s;
            return LSL_OK;
        }
    }
    std::vector<int> tiles = P->tile ? std::vector<int>{P->tile} : std::vector<int>{16, 32};
    std::vector<int> slabs = P->slab ? std::vector<int>{P->slab} : std::vector<int>{4, 8, 16};
    // windows of 64 planes: long enough that the persistent launch's tail
    // (its last, unevenly sized work items) weighs on every tile as it does
    // on a full pass, which a short window overstates for large tiles
    const int win = std::min(64, G->n_slices);
    const int nwin = G->n_slices >= 3 * win ? 3 : 1;
    std::vector<int> starts;
    for (int w = 0; w < nwin; ++w)
        starts.push_back(nwin == 1 ? 0 : (int)((int64_t)(G->n_slices - win) * (2 * w + 1) / (2 * nwin)) / 16 * 16);
    hipStream_t st = (hipStream_t)stream;
    const size_t es = L->dtype == LSL_F64 ? 8 : 4;
    void* field = nullptr;
    int64_t* offs = nullptr;
    hipError_t he = hipMalloc(&field, (size_t)win * G->W * G->H * es);
    if (he == hipSuccess) he = hipMalloc((void**)&offs, ((size_t)win + 1) * sizeof(int64_t));
    if (he != hipSuccess) {
        hipGetLastError();
        hipFree(field);
        set_error("slice_autotune: cannot allocate the sample field");
        return LSL_ENOMEM;
    }
    double best = 1e300;
    int bt = tiles[0], bs = slabs[0];
    lsl_status result = LSL_OK;
    {
        // warm-up: the first binning fills the device-memory cache, which
        // would otherwise be charged to the first candidate
        lsl_bin_params bp{tiles[0], slabs[0], P->max_pairs};
        lattice_bins* b = nullptr;
        if (lattice_bin(L, G, &bp, &b, stream) == LSL_OK) lattice_bins_free(b);
        set_error("");
    }
    for (int t : tiles) {
        for (int s : slabs) {
            lsl_bin_params bp{t, s, P->max_pairs};
            lattice_bins* b = nullptr;
            // the binning's cost: the faster of two runs (lattice_bin leaves
            // the first group's lists in flight: wait for them, so the score
            // carries the whole binning)
            double bin_s = 1e300;
            lsl_status rs = LSL_OK;
            for (int rep = 0; rep < 2 && rs == LSL_OK; ++rep) {
                if (b) {
                    lattice_bins_free(b);
                    b = nullptr;
                }
                const auto c0 = std::chrono::steady_clock::now();
                rs = lattice_bin(L, G, &bp, &b, stream);
                if (rs == LSL_OK && hipStreamSynchronize(st) != hipSuccess) rs = LSL_EDEVICE;
                bin_s = std::min(bin_s, std::chrono::duration<double>(
                                            std::chrono::steady_clock::now() - c0).count());
            }
            if (rs != LSL_OK) {
                if (b) lattice_bins_free(b);
                if (rs == LSL_ENOMEM) continue;    // candidate does not fit
                result = rs;
                break;
            }
            double field_s = 0;
            for (int k0 : starts) {
                float best_ms = 1e30f;
                // the persistent path a full pass takes (its field launch,
                // HIP events inside slice_batch); no segments are stored
                for (int rep = 0; rep < 2; ++rep) {
                    int64_t total = 0;
                    rs = slice_batch(b, k0, win, field, nullptr, nullptr, 0, offs, &total, stream);
                    if (rs == LSL_ECAPACITY) rs = LSL_OK;
                    lsl_bins_info bi{};
                    if (rs == LSL_OK) rs = lattice_bins_info(b, &bi);
                    if (rs == LSL_OK && bi.last_field_ms >= 0.0)
                        best_ms = std::min(best_ms, (float)bi.last_field_ms);
                }
                field_s += best_ms * 1e-3;
            }
            // a pass over all planes bins every group after the first once,
            // each from its predecessor's active struts: time that sequence
            double groups_s = 0;
            lsl_bins_info inf{};
            if (rs == LSL_OK) rs = lattice_bins_info(b, &inf);
            if (rs == LSL_OK && inf.n_groups > 1) {
                rs = lattice_bins_export(b, 0, nullptr, nullptr, stream);
                if (rs == LSL_OK && hipStreamSynchronize(st) != hipSuccess) rs = LSL_EDEVICE;
                const auto g0 = std::chrono::steady_clock::now();
                for (int g = 1; g < inf.n_groups && rs == LSL_OK; ++g)
                    rs = lattice_bins_export(b, g, nullptr, nullptr, stream);
                if (rs == LSL_OK && hipStreamSynchronize(st) != hipSuccess) rs = LSL_EDEVICE;
                groups_s =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - g0).count();
            }
            lattice_bins_free(b);
            if (rs != LSL_OK) {
                result = rs;
                break;
            }
            const double score = field_s / (nwin * win) * G->n_slices + bin_s + groups_s;
            if (score < best) {
                best = score;
                bt = t;
                bs = s;
            }
        }
        if (result != LSL_OK) break;
    }
    hipFree(field);
    hipFree(offs);
    if (result != LSL_OK) return result;
    P->tile = bt;
    P->slab = bs;
    if (cache_path) cache_store(cache_path, key, bt, bs);
    return LSL_OK;
}
