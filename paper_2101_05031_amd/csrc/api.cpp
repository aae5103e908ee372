// C ABI of liblsl: handle management, argument validation, slab-group
// planning and the entry points declared in include/lsl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace lsl {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Device memory cache.  Binning a lattice of a million struts takes ~7 GB in
// a few dozen buffers; hipMalloc / hipFree of that much costs milliseconds
// per handle, so freed buffers are kept per device in size classes (eight
// per power of two, at most 1/8 over the request) and handed to the next
// request of the same class.  Buffers only return to the cache once the
// device is idle (handles synchronize before releasing), so reuse never
// races with work still in flight.  lsl_cache_trim gives the memory back;
// LSL_NO_CACHE=1 in the environment turns the cache off.
// ---------------------------------------------------------------------------
class DeviceCache {
  public:
    static DeviceCache& get() {
        static DeviceCache* c = new DeviceCache();   // never destroyed: no teardown at exit
        return *c;
    }
    static size_t size_class(size_t bytes) {
        bytes = std::max<size_t>(bytes, 256);
        size_t p = 1;
        while (p <= bytes / 2) p <<= 1;              // largest power of two <= bytes
        const size_t step = std::max<size_t>(256, p / 8);
        return (bytes + step - 1) / step * step;
    }
    hipError_t alloc(void** p, size_t bytes) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (enabled_) {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.find(Key{dev, bytes});
            if (it != free_.end() && !it->second.empty()) {
                *p = it->second.back();
                it->second.pop_back();
                cached_ -= bytes;
                return hipSuccess;
            }
        }
        e = hipMalloc(p, bytes);
        if (e == hipErrorOutOfMemory && enabled_) {
            // give back what the cache holds and try once more
            trim();
            hipGetLastError();
            e = hipMalloc(p, bytes);
        }
        return e;
    }
    void release(void* p, size_t bytes) {
        if (!p) return;
        int dev = 0;
        if (!enabled_ || hipGetDevice(&dev) != hipSuccess) {
            hipFree(p);
            return;
        }
        std::lock_guard<std::mutex> lk(mu_);
        free_[Key{dev, bytes}].push_back(p);
        cached_ += bytes;
    }
    void trim() {
        std::lock_guard<std::mutex> lk(mu_);
        if (free_.empty()) return;
        int cur = 0;
        hipGetDevice(&cur);
        for (auto& kv : free_) {
            hipSetDevice(kv.first.dev);
            hipDeviceSynchronize();
            for (void* p : kv.second) hipFree(p);
        }
        free_.clear();
        cached_ = 0;
        hipSetDevice(cur);
    }
    size_t cached() const { return cached_; }

  private:
    DeviceCache() {
        const char* v = std::getenv("LSL_NO_CACHE");
        enabled_ = !(v && *v && std::strcmp(v, "0") != 0);
    }
    struct Key {
        int dev;
        size_t bytes;
        bool operator<(const Key& o) const {
            return dev != o.dev ? dev < o.dev : bytes < o.bytes;
        }
    };
    std::mutex mu_;
    std::map<Key, std::vector<void*>> free_;
    size_t cached_ = 0;
    bool enabled_ = true;
};

// ---------------------------------------------------------------------------
// Static device scratch for slice_occupancy_loss_static, the entry point
// that allocates nothing: the per-block partial sums of the loss (at most
// occupancy_blocks(n) <= 8192 doubles, 64 KB) live in this file-scope array,
// one copy per GPU for the life of the process.  In host code `scratch`
// names a host-side stand-in, so kernels get the device address that
// hipGetSymbolAddress returns, taken once per device on its first use.
// Calls that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchElems = 8192;
static __device__ __align__(256) double scratch[kStaticScratchElems];

lsl_status static_scratch(double** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = 0;
    LSL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("static scratch: device index out of range");
        return LSL_EINTERNAL;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        LSL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        addr[dev] = (double*)p;
    }
    *out = addr[dev];
    return LSL_OK;
}

}  // namespace lsl

using namespace lsl;

namespace {

struct Group {
    int32_t sa, sb;
    uint64_t pairs;
    uint64_t cells;                   // (slab, tile row, column segment, strut) cells, <= pairs
    uint32_t n_active;
    uint32_t n_buckets;
};

}  // namespace

// ---------------------------------------------------------------------------
// Executable graphs of slice_batch, shared by every handle of the process.
// A call captures its launches afresh (a cheap recording) and brings a cached
// executable graph of the same launch shape up to date with
// hipGraphExecUpdate; a new one is instantiated only when no entry of that
// shape exists or the update is refused (the recorded launches differ in
// kind or number).  Consecutive slab groups of a call use two entries of a
// shape in turn, and an entry's previous launch is waited for before it is
// updated, so an executable graph is never changed while the device may run
// it.  At most kCap entries are kept (the least recently used goes first);
// lsl_cache_trim releases them all.
// ---------------------------------------------------------------------------
class GraphCache {
  public:
    static GraphCache& get() {
        static GraphCache* c = new GraphCache();     // never destroyed: no teardown at exit
        return *c;
    }
    // Launches `graph` (captured, not instantiated; the caller keeps
    // ownership) on `st` through the entry for `key` on the current device.
    lsl_status launch(const std::vector<unsigned char>& key, hipGraph_t graph, hipStream_t st) {
        int dev = 0;
        LSL_HIP(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lk(mu_);
        Entry* ent = nullptr;
        for (auto& e : e_)
            if (e.dev == dev && e.key == key) ent = &e;
        if (ent) {
            LSL_HIP(hipEventSynchronize(ent->done));
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            if (hipGraphExecUpdate(ent->exec, graph, &bad, &res) == hipSuccess &&
                res == hipGraphExecUpdateSuccess) {
                ++n_update_;
            } else {
                hipGetLastError();
                hipGraphExecDestroy(ent->exec);
                ent->exec = nullptr;
            }
        } else {
            if (e_.size() >= kCap) {
                size_t old = 0;
                for (size_t i = 1; i < e_.size(); ++i)
                    if (e_[i].use < e_[old].use) old = i;
                LSL_TRY(release(e_[old]));
                e_.erase(e_.begin() + (std::ptrdiff_t)old);
            }
            Entry ne{};
            ne.key = key;
            ne.dev = dev;
            LSL_HIP(hipEventCreateWithFlags(&ne.done, hipEventDisableTiming));
            e_.push_back(ne);
            ent = &e_.back();
        }
        if (!ent->exec) {
            const hipError_t ie = hipGraphInstantiate(&ent->exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                ent->exec = nullptr;
                hipGetLastError();
                set_error(std::string("slice_batch: graph instantiation failed: ") +
                          hipGetErrorString(ie));
                return LSL_EDEVICE;
            }
            ++n_instantiate_;
        }
        ent->use = ++tick_;
        LSL_HIP(hipGraphLaunch(ent->exec, st));
        LSL_HIP(hipEventRecord(ent->done, st));
        return LSL_OK;
    }
    // Waits for and releases every entry (each on its own device).
    lsl_status trim() {
        std::lock_guard<std::mutex> lk(mu_);
        int cur = 0;
        LSL_HIP(hipGetDevice(&cur));
        lsl_status st = LSL_OK;
        for (auto& e : e_) {
            const lsl_status s = release(e);
            if (st == LSL_OK) st = s;
        }
        e_.clear();
        hipSetDevice(cur);
        return st;
    }
    void stats(int64_t* inst, int64_t* upd, int64_t* n) {
        std::lock_guard<std::mutex> lk(mu_);
        if (inst) *inst = n_instantiate_;
        if (upd) *upd = n_update_;
        if (n) *n = (int64_t)e_.size();
    }

  private:
    struct Entry {
        std::vector<unsigned char> key;
        int dev;
        hipGraphExec_t exec;
        hipEvent_t done;            // recorded after the entry's last launch
        uint64_t use;
    };
    static lsl_status release(Entry& e) {
        LSL_HIP(hipSetDevice(e.dev));
        if (e.done) LSL_HIP(hipEventSynchronize(e.done));
        if (e.exec) hipGraphExecDestroy(e.exec);
        if (e.done) hipEventDestroy(e.done);
        e.exec = nullptr;
        e.done = nullptr;
        return LSL_OK;
    }
    static constexpr size_t kCap = 64;
    std::mutex mu_;
    std::vector<Entry> e_;
    uint64_t tick_ = 0;
    int64_t n_instantiate_ = 0, n_update_ = 0;
};

struct lattice_bins {
    int dtype = LSL_F32;
    int64_t n_nodes = 0, n_edges = 0;
    uint32_t n_binned = 0;
    double R = 0, C = 0;
    bool strut_R = false;              // per-strut supports (in rec[].pad)
    bool plane_ref = false;            // float32 field: every plane its own reference
    bool wide = false;                 // float32 adjoint: 16x16-pixel regions
    int32_t wexp = 0;                  // float32 field: sums times 2^(5 wexp)
    float* rho = nullptr;              // float32 field: per-strut length scale
    int32_t kernel = LSL_KERNEL_QUARTIC;
    double sigma = 0;
    lsl_grid grid{};
    double inv_dx = 0, inv_dy = 0, inv_dz = 0;
    int32_t tile = 16, slab = 8, ntx = 0, nty = 0, n_slabs = 0;
    int64_t max_pairs = 0;

    std::vector<uint64_t> pairs_slab;   // pairs of each slab
    std::vector<uint32_t> win_end;      // # struts whose first slab <= s
    std::vector<uint32_t> gone;         // # struts whose last slab < s
    std::vector<Group> groups;
    int cur_group = -1;
    int cur_buf = 0;
    uint64_t total_pairs = 0, max_group_pairs = 0;

    // per-strut arrays in edge-list order
    void* rec = nullptr;
    uint32_t* perm = nullptr;
    SRange* ranges = nullptr;
    PRange* pranges = nullptr;
    void* w = nullptr;
    int2* ends = nullptr;
    double4* line = nullptr;          // direction and length per strut, float64

    // resident group
    uint32_t* active[2] = {nullptr, nullptr};
    uint32_t* eoff = nullptr;
    uint32_t* toff = nullptr;          // [cap_active + 1] row-segment cells per active strut
    uint32_t* roffs = nullptr;         // CSR of the row segments of the largest group
    uint32_t* offsets = nullptr;
    const uint32_t* ids = nullptr;     // bucket entries (points into v0 or v1)
    uint32_t* skeys = nullptr;         // their bucket keys, written for the adjoint (k0 or k1)
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr;
    uint32_t* tmp = nullptr;
    uint32_t* blk = nullptr;
    size_t cap_active = 0, cap_pairs = 0, cap_buckets = 0;

    // backward
    uint32_t* emi = nullptr;           // [cap_pairs] entry -> emission index
    uint32_t* inv = nullptr;           // [n_binned] inverse of the active list
    int emi_group = -1;                // group whose emi is current
    void* partial = nullptr;
    double* acc = nullptr;
    uint32_t* node_off = nullptr;
    uint32_t* node_inc = nullptr;

    // misc
    unsigned long long* stats = nullptr;
    unsigned long long* ctmp = nullptr;
    size_t ctmp_elems = 0;
    uint32_t* cbits = nullptr;        // binary images: slice_contours, slice_batch
    size_t cbits_elems = 0;
    uint32_t* pscratch = nullptr;     // slice_polylines: edges, cells, links, jumps
    size_t pscratch_elems = 0;
    double* dscratch = nullptr;       // slice_density_loss: residuals, block partials
    size_t dscratch_elems = 0;
    uint32_t* queue_buf = nullptr;     // persistent path: keys/vals/alternates + counter
    size_t queue_cap = 0;
    std::vector<std::pair<void*, size_t>> allocs;
    int64_t dev_bytes = 0, peak_bytes = 0;

    // per slab group of a slice_batch call, on the caller's stream: before and
    // after binning the group, after each of the three graphs
    struct StageEvents {
        hipEvent_t ev[5];
    };
    std::vector<StageEvents> stage_events;
    // around each slab group's adjoint kernel of the last slice_field_backward
    struct EvPair {
        hipEvent_t ev[2];
    };
    std::vector<EvPair> back_events;
    size_t n_back = 0;
    double last_field_ms = -1.0, last_group_bin_ms = -1.0, last_queue_ms = -1.0,
           last_contour_ms = -1.0;
    bool queue_in_alt = false;      // the sorted work queue is in the alternate buffer

    ~lattice_bins() {
        hipDeviceSynchronize();
        for (auto& se : stage_events)
            for (auto& e : se.ev)
                if (e) hipEventDestroy(e);
        for (auto& bp : back_events)
            for (auto& e : bp.ev)
                if (e) hipEventDestroy(e);
        for (auto& a : allocs) DeviceCache::get().release(a.first, a.second);
    }

    lsl_status alloc(void** p, size_t bytes) {
        *p = nullptr;
        bytes = DeviceCache::size_class(bytes);
        hipError_t e = DeviceCache::get().alloc(p, bytes);
        if (e != hipSuccess) {
            hipGetLastError();
            *p = nullptr;
            set_error("device allocation of " + std::to_string(bytes) + " bytes failed: " +
                      hipGetErrorString(e));
            return LSL_ENOMEM;
        }
        allocs.emplace_back(*p, bytes);
        dev_bytes += (int64_t)bytes;
        peak_bytes = std::max(peak_bytes, dev_bytes);
        return LSL_OK;
    }
    template <typename T>
    lsl_status alloc_t(T** p, size_t n) {
        return alloc((void**)p, n * sizeof(T));
    }
    // callers release only buffers no queued work still uses
    void release(void* p) {
        if (!p) return;
        for (size_t i = 0; i < allocs.size(); ++i)
            if (allocs[i].first == p) {
                DeviceCache::get().release(p, allocs[i].second);
                dev_bytes -= (int64_t)allocs[i].second;
                allocs.erase(allocs.begin() + (long)i);
                return;
            }
    }
    size_t esize() const { return dtype == LSL_F64 ? 8 : 4; }
    // Grows library scratch *p (capacity *cap elements) to `need` elements:
    // waits for the work queued on `st` (it may still use the old buffer),
    // releases it and allocates the new one.
    template <typename T>
    lsl_status grow(T** p, size_t* cap, size_t need, hipStream_t st) {
        if (need <= *cap) return LSL_OK;
        LSL_HIP(hipStreamSynchronize(st));
        release(*p);
        *p = nullptr;
        *cap = 0;
        LSL_TRY(alloc_t(p, need));
        *cap = need;
        return LSL_OK;
    }
};

namespace {

#define LSL_CHECK(cond, msg)        \
    do {                            \
        if (!(cond)) {              \
            set_error(msg);         \
            return LSL_EINVAL;      \
        }                           \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

// Gaussian kernel: exp(R^2 / 2 sigma^2) must stay finite in float32
constexpr double kMaxROverSigma = 12.0;

lsl_status check_lattice(const lsl_lattice* L) {
    LSL_CHECK(L != nullptr, "lattice is NULL");
    LSL_CHECK(L->dtype == LSL_F32 || L->dtype == LSL_F64, "lattice dtype must be LSL_F32 or LSL_F64");
    LSL_CHECK(L->n_nodes >= 1, "n_nodes must be >= 1");
    LSL_CHECK(L->n_edges >= 0, "n_edges must be >= 0");
    LSL_CHECK(L->n_edges < (int64_t)0x7fffffff, "n_edges must be < 2^31");
    LSL_CHECK(L->n_nodes < (int64_t)0x7fffffff, "n_nodes must be < 2^31");
    LSL_CHECK(L->nodes != nullptr, "nodes is NULL");
    LSL_CHECK(L->n_edges == 0 || L->edges != nullptr, "edges is NULL");
    LSL_CHECK(L->n_edges == 0 || L->weight != nullptr, "weight is NULL");
    LSL_CHECK(finite_pos(L->R), "R must be finite and > 0");
    LSL_CHECK(finite_pos(L->C), "C must be finite and > 0");
    LSL_CHECK(L->kernel == LSL_KERNEL_QUARTIC || L->kernel == LSL_KERNEL_GAUSS,
              "kernel must be LSL_KERNEL_QUARTIC or LSL_KERNEL_GAUSS");
    if (L->kernel == LSL_KERNEL_GAUSS) {
        LSL_CHECK(finite_pos(L->sigma), "sigma must be finite and > 0");
        LSL_CHECK(L->support != nullptr || L->R <= kMaxROverSigma * L->sigma,
                  "the support may be at most 12 sigma");
    }
    return LSL_OK;
}

lsl_status check_grid(const lsl_grid* g) {
    LSL_CHECK(g != nullptr, "grid is NULL");
    LSL_CHECK(std::isfinite(g->x0) && std::isfinite(g->y0) && std::isfinite(g->z0),
              "grid origin must be finite");
    LSL_CHECK(finite_pos(g->dx) && finite_pos(g->dy) && finite_pos(g->dz),
              "grid steps must be finite and > 0");
    LSL_CHECK(g->W >= 2 && g->H >= 2, "grid W and H must be >= 2");
    LSL_CHECK(g->W <= 65536 && g->H <= 65536, "grid W and H must be <= 65536");
    LSL_CHECK(g->n_slices >= 1, "grid n_slices must be >= 1");
    return LSL_OK;
}

lsl_status check_params(const lsl_bin_params* p, int32_t* tile, int32_t* slab, int64_t* mp) {
    *tile = 16;
    *slab = 8;
    *mp = (int64_t)1 << 30;
    if (!p) return LSL_OK;
    if (p->tile) *tile = p->tile;
    if (p->slab) *slab = p->slab;
    if (p->max_pairs) *mp = p->max_pairs;
    LSL_CHECK(*tile == 8 || *tile == 16 || *tile == 32 || *tile == 64,
              "tile must be 8, 16, 32 or 64");
    LSL_CHECK(*slab >= 1 && *slab <= 16, "slab must be in 1..16");
    LSL_CHECK(*mp >= 1 && *mp <= (int64_t)0x7fffffff, "max_pairs must be in [1, 2^31)");
    return LSL_OK;
}

hipStream_t S(void* s) { return (hipStream_t)s; }

lsl_status plan_groups(lattice_bins* b, const std::vector<uint32_t>& cnt_lo,
                       const std::vector<uint32_t>& cnt_hi,
                       const std::vector<unsigned long long>& diff,
                       const std::vector<uint32_t>& rdiff) {
    const int ns = b->n_slabs;
    b->pairs_slab.assign(ns, 0);
    // (strut, tile row, column segment) cells per slab: a slab's cells are no
    // more than its pairs (< 2^32), so the modular running sum is exact
    std::vector<uint32_t> rows_slab(ns, 0u);
    uint32_t rrun = 0;
    for (int s = 0; s < ns; ++s) {
        rrun += rdiff[s];
        rows_slab[s] = rrun;
    }
    b->win_end.assign(ns, 0);
    b->gone.assign(ns, 0);
    uint64_t run = 0;
    uint64_t lo = 0, hi = 0;
    for (int s = 0; s < ns; ++s) {
        run += diff[s];
        b->pairs_slab[s] = run;
        lo += cnt_lo[s];
        b->win_end[s] = (uint32_t)lo;
        b->gone[s] = (uint32_t)hi;
        hi += cnt_hi[s];
    }
    b->groups.clear();
    b->total_pairs = 0;
    b->max_group_pairs = 0;
    const uint64_t per_slab_buckets = (uint64_t)b->ntx * (uint64_t)b->nty;
    int s = 0;
    while (s < ns) {
        Group g;
        g.sa = s;
        uint64_t p = b->pairs_slab[s];
        int e = s;
        while (e + 1 < ns && p + b->pairs_slab[e + 1] <= (uint64_t)b->max_pairs &&
               (uint64_t)(e + 2 - s) * per_slab_buckets < 0x7fffffffull)
            p += b->pairs_slab[++e];
        g.sb = e;
        g.pairs = p;
        g.cells = 0;
        for (int q = s; q <= e; ++q) g.cells += rows_slab[q];
        if (p >= 0xfffffff0ull) {
            set_error("one slab holds more than 2^32 (slab, tile, strut) pairs; use larger tiles "
                      "or thinner slabs");
            return LSL_ENOMEM;
        }
        const uint64_t nbk = (uint64_t)(e - s + 1) * per_slab_buckets;
        if (nbk >= 0x7fffffffull) {
            set_error("too many tiles per slab");
            return LSL_EINVAL;
        }
        g.n_buckets = (uint32_t)nbk;
        g.n_active = b->win_end[e] - b->gone[s];
        b->groups.push_back(g);
        b->total_pairs += p;
        b->max_group_pairs = std::max<uint64_t>(b->max_group_pairs, p);
        s = e + 1;
    }
    return LSL_OK;
}

lsl_status ensure_group(lattice_bins* b, int g, hipStream_t st) {
    if (g == b->cur_group) return LSL_OK;
    const Group& G = b->groups[g];
    GroupBuffers gb{};
    gb.ranges = b->ranges;
    const bool incremental = b->cur_group >= 0 && b->cur_group == g - 1;
    if (incremental) {
        const Group& P = b->groups[g - 1];
        gb.prev_active = b->active[b->cur_buf];
        gb.n_prev = P.n_active;
        gb.range_lo = b->win_end[P.sb];
    } else {
        gb.prev_active = nullptr;
        gb.n_prev = 0;
        gb.range_lo = 0;
    }
    gb.range_hi = b->win_end[G.sb];
    const int out = incremental ? 1 - b->cur_buf : 0;
    gb.active = b->active[out];
    gb.n_active = G.n_active;
    gb.sa = G.sa;
    gb.sb = G.sb;
    gb.ntx = b->ntx;
    gb.nty = b->nty;
    gb.n_pairs = (uint32_t)G.pairs;
    gb.n_cells = (uint32_t)G.cells;
    gb.n_buckets = G.n_buckets;
    gb.eoff = b->eoff;
    gb.toff = b->toff;
    gb.roffs = b->roffs;
    gb.offsets = b->offsets;
    gb.keys_out = &b->skeys;
    gb.ids_out = &b->ids;
    gb.k0 = b->k0;
    gb.v0 = b->v0;
    gb.k1 = b->k1;
    gb.v1 = b->v1;
    gb.tmp = b->tmp;
    gb.blk = b->blk;
    b->cur_group = -1;   // invalid until the launches below are enqueued
    b->emi_group = -1;
    LSL_TRY(bin_group(gb, st));
    b->cur_group = g;
    b->cur_buf = out;
    return LSL_OK;
}

FieldArgs field_args(const lattice_bins* b, int32_t k0, int32_t nk, void* field) {
    FieldArgs a{};
    a.rec = b->rec;
    a.line = b->line;
    a.rho = b->rho;
    a.wexp = b->wexp;
    a.offsets = b->offsets;
    a.ids = b->ids;
    a.n_binned = b->n_binned;
    a.ntx = b->ntx;
    a.nty = b->nty;
    a.tile = b->tile;
    a.slab = b->slab;
    a.k0 = k0;
    a.nk = nk;
    a.W = b->grid.W;
    a.H = b->grid.H;
    a.x0 = b->grid.x0;
    a.y0 = b->grid.y0;
    a.dx = b->grid.dx;
    a.dy = b->grid.dy;
    a.z0 = b->grid.z0;
    a.dz = b->grid.dz;
    a.R = b->R;
    a.pranges = b->pranges;
    a.strut_R = b->strut_R ? 1 : 0;
    a.kernel = b->kernel;
    a.plane_ref = b->plane_ref ? 1 : 0;
    if (b->kernel == LSL_KERNEL_GAUSS) {
        a.gk1 = 1.0 / (b->sigma * std::sqrt(2.0));
        a.gk2 = 1.0 / (2.0 * b->sigma * b->sigma);
        a.gc0 = b->sigma * std::sqrt(std::acos(-1.0) / 2.0);
    }
    a.C = b->C;
    a.field = field;
    a.bits_blk = nullptr;
    return a;
}

// Calls fn(group index, first slab, last slab) for every group meeting the
// slabs of planes [k0, k0+nk).
template <typename Fn>
lsl_status for_groups(lattice_bins* b, int32_t k0, int32_t nk, Fn fn) {
    const int s_first = k0 / b->slab, s_last = (k0 + nk - 1) / b->slab;
    for (size_t g = 0; g < b->groups.size(); ++g) {
        const Group& G = b->groups[g];
        if (G.sb < s_first || G.sa > s_last) continue;
        LSL_TRY(fn((int)g, std::max(G.sa, s_first), std::min(G.sb, s_last)));
    }
    return LSL_OK;
}

lsl_status check_range(const lattice_bins* b, int32_t k0, int32_t nk) {
    LSL_CHECK(b != nullptr, "bins handle is NULL");
    LSL_CHECK(k0 >= 0 && nk >= 1 && (int64_t)k0 + nk <= b->grid.n_slices,
              "plane range must lie in [0, n_slices)");
    return LSL_OK;
}

__global__ void k_u32_to_i64(const uint32_t* in, int64_t* out, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i];
}

__global__ void k_ids_to_edges(const uint32_t* ids, const uint32_t* perm, int32_t* out, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)perm[ids[i]];
}

__global__ void k_copy_i32(const uint32_t* in, int32_t* out, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

unsigned nblk(size_t n) { return (unsigned)((n + 255) / 256); }

// 32-bit words of a block-major binary image of nk planes
size_t blk_words(const lattice_bins* b, int32_t nk) {
    return 2 * (size_t)nk * (size_t)((b->grid.H + 7) / 8) * (size_t)((b->grid.W + 7) / 8);
}

// library scratch for the block-major binary images of nk planes
lsl_status ensure_cbits(lattice_bins* b, int32_t nk, hipStream_t st) {
    return b->grow(&b->cbits, &b->cbits_elems, blk_words(b, nk), st);
}

}  // namespace

// ===========================================================================
extern "C" {

const char* lsl_status_string(lsl_status s) {
    switch (s) {
        case LSL_OK: return "ok";
        case LSL_EINVAL: return "invalid argument";
        case LSL_ENOMEM: return "out of device memory";
        case LSL_ECAPACITY: return "output capacity exceeded";
        case LSL_EDEVICE: return "device error";
        case LSL_EINTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* lsl_last_error(void) { return lsl::last_error(); }

const char* lsl_version(void) { return "liblsl 0.1 (gfx950)"; }

lsl_status lattice_bin(const lsl_lattice* L, const lsl_grid* G, const lsl_bin_params* P,
                       lattice_bins** out, void* stream) {
    set_error("");
    LSL_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    LSL_TRY(check_lattice(L));
    LSL_TRY(check_grid(G));
    int32_t tile, slab;
    int64_t mp;
    LSL_TRY(check_params(P, &tile, &slab, &mp));
    hipStream_t st = S(stream);

    lattice_bins* b = new lattice_bins();
    b->dtype = L->dtype;
    b->n_nodes = L->n_nodes;
    b->n_edges = L->n_edges;
    b->R = L->R;
    b->C = L->C;
    b->strut_R = L->support != nullptr;
    b->kernel = L->kernel;
    b->sigma = L->sigma;
    b->grid = *G;
    b->inv_dx = 1.0 / G->dx;
    b->inv_dy = 1.0 / G->dy;
    b->inv_dz = 1.0 / G->dz;
    b->tile = tile;
    b->slab = slab;
    b->max_pairs = mp;
    b->ntx = (G->W + tile - 1) / tile;
    b->nty = (G->H + tile - 1) / tile;
    b->n_slabs = (G->n_slices + slab - 1) / slab;
    const size_t E = (size_t)L->n_edges;
    const int ns = b->n_slabs;

    auto fail = [&](lsl_status s) {
        delete b;
        return s;
    };
    lsl_status s;

    // ---- prep: ranges, sort keys, plan histograms
    uint32_t *klo = nullptr, *khi = nullptr, *vals = nullptr, *ka = nullptr, *va = nullptr;
    uint32_t* ks0 = nullptr;
    uint32_t *cnt = nullptr, *stmp = nullptr;
    SRange* rid = nullptr;
    PRange* prid = nullptr;
    unsigned long long* diff = nullptr;
    const size_t En = std::max<size_t>(E, 1);
    if ((s = b->alloc_t(&klo, En)) || (s = b->alloc_t(&vals, En)) || (s = b->alloc_t(&ka, En)) ||
        (s = b->alloc_t(&va, En)) || (s = b->alloc_t(&rid, En)) || (s = b->alloc_t(&prid, En)) ||
        (s = b->alloc_t(&cnt, 2 * (size_t)ns + 4)) || (s = b->alloc_t(&diff, 2 * ((size_t)ns + 1))) ||
        (s = b->alloc_t(&stmp, radix_tmp_elems(En))))
        return fail(s);
    if (L->dtype == LSL_F64 && (s = b->alloc_t(&khi, En))) return fail(s);
    // per-strut supports: first-slab keys by edge id, then the gathered keys
    // and one alternate key/value pair for their sort
    if (L->support && (s = b->alloc_t(&ks0, 3 * En))) return fail(s);
    uint32_t* cnt_lo = cnt;
    uint32_t* cnt_hi = cnt + ns;
    uint32_t* counters = cnt + 2 * ns;   // [0] n_binned, [1] err, [2] ~smallest support,
                                         // [3] largest r R
    if ((s = fill_u32(cnt, 0u, 2 * (size_t)ns + 4, st)) ||
        (s = fill_bytes0(diff, 2 * ((size_t)ns + 1) * 8, st)))
        return fail(s);
    PrepArgs pa{};
    pa.nodes = L->nodes;
    pa.edges = L->edges;
    pa.weight = L->weight;
    pa.n_nodes = L->n_nodes;
    pa.n_edges = L->n_edges;
    pa.R = L->R;
    pa.x0 = G->x0;
    pa.y0 = G->y0;
    pa.z0 = G->z0;
    pa.inv_dx = b->inv_dx;
    pa.inv_dy = b->inv_dy;
    pa.inv_dz = b->inv_dz;
    pa.W = G->W;
    pa.H = G->H;
    pa.S = G->n_slices;
    pa.tile = tile;
    pa.slab = slab;
    pa.n_slabs = ns;
    pa.key_lo = klo;
    pa.key_hi = khi;
    pa.vals = vals;
    pa.ranges = rid;
    pa.pranges = prid;
    pa.cnt_lo = cnt_lo;
    pa.cnt_hi = cnt_hi;
    pa.pair_diff = diff;
    pa.row_diff = (uint32_t*)(diff + ns + 1);
    pa.n_binned = counters;
    pa.err = counters + 1;
    pa.min_support = counters + 2;
    pa.max_wr = counters + 3;
    pa.support = L->support;
    pa.key_s0 = ks0;
    pa.max_r_over_sigma = L->kernel == LSL_KERNEL_GAUSS ? kMaxROverSigma : 0.0;
    pa.sigma = L->sigma;
    pa.keep_zero = L->keep_zero_weight ? 1 : 0;
    if ((s = launch_prep(L->dtype, pa, st))) return fail(s);

    // edge list: stable sort by the lower end's z (64-bit keys in two passes)
    int which = 0;
    uint32_t* perm_src = vals;
    if (E > 0) {
        if ((s = radix_sort_pairs(klo, vals, ka, va, E, 32, stmp, &which, st))) return fail(s);
        uint32_t* sv = which ? va : vals;
        if (L->dtype == LSL_F64) {
            uint32_t* sk = which ? ka : klo;        // low words, sorted (unused now)
            uint32_t* hk = which ? klo : ka;        // free buffer for gathered high words
            uint32_t* hv = which ? vals : va;       // free buffer for the carried values
            if ((s = launch_gather_u32(khi, sv, hk, E, st))) return fail(s);
            (void)sk;
            int w2 = 0;
            if ((s = radix_sort_pairs(hk, sv, khi, hv, E, 32, stmp, &w2, st))) return fail(s);
            sv = w2 ? hv : sv;
        }
        if (ks0) {
            // per-strut supports: the first slab is the major key (a stable
            // sort over the z order), so each slab's window is a prefix
            uint32_t* gk = ks0 + En;                  // keys in z order
            uint32_t* ak = ks0;                       // alternates: the by-id keys
            uint32_t* av = ks0 + 2 * En;              //   are no longer needed
            if ((s = launch_gather_u32(ks0, sv, gk, E, st))) return fail(s);
            int bits = 1;
            while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)ns) ++bits;
            int w3 = 0;
            if ((s = radix_sort_pairs(gk, sv, ak, av, E, bits, stmp, &w3, st))) return fail(s);
            sv = w3 ? av : sv;
        }
        perm_src = sv;
    }

    // read the plan back
    std::vector<uint32_t> h_cnt(2 * (size_t)ns + 4);
    std::vector<unsigned long long> h_diff((size_t)ns + 1);
    std::vector<uint32_t> h_rdiff((size_t)ns + 1);
    hipError_t he = hipMemcpyAsync(h_cnt.data(), cnt, h_cnt.size() * 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess)
        he = hipMemcpyAsync(h_diff.data(), diff, h_diff.size() * 8, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess)
        he = hipMemcpyAsync(h_rdiff.data(), diff + ns + 1, h_rdiff.size() * 4,
                            hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
        set_error(std::string("lattice_bin: ") + hipGetErrorString(he));
        return fail(LSL_EDEVICE);
    }
    const uint32_t err = h_cnt[2 * ns + 1];
    if (err) {
        std::string m = "lattice_bin:";
        if (err & 1u) m += " edge index out of range;";
        if (err & 2u) m += " negative or non-finite weight;";
        if (err & 4u) m += " non-finite node position;";
        if (err & 8u) m += " support radius not finite and > 0;";
        if (err & 16u) m += " support radius above 12 sigma;";
        set_error(m);
        return fail(LSL_EINVAL);
    }
    b->n_binned = h_cnt[2 * ns];
    {
        // The float32 field kernel shares one reference plane among 8 planes
        // when the shift it applies stays small against the support:
        // 7 dz |d| <= R^2 / 10 for the farthest pixel d of an 8x8 block and
        // the smallest support; otherwise every plane is its own reference.
        double rmin = L->R;
        const uint32_t inv = h_cnt[2 * ns + 2];
        if (L->support && inv != 0u) {
            const uint32_t bits = ~inv;
            float f;
            std::memcpy(&f, &bits, 4);
            rmin = (double)f;
        }
        const double dmax = 3.5 * std::sqrt(G->dx * G->dx + G->dy * G->dy);
        b->plane_ref = !(7.0 * G->dz * dmax <= 0.1 * rmin * rmin);
        // the float32 adjoint measures pixel offsets from the centre of a
        // 16x16 region when the farthest one, 7.5 |(dx, dy)|, stays within
        // the smallest support (the rounding of H grows with |d| / R), else
        // from the centre of each 8x8 block
        b->wide = 7.5 * std::sqrt(G->dx * G->dx + G->dy * G->dy) <= rmin;
        // the float32 kernel works in units of R / rho_j, rho_j = (r_j R_j)^(1/5)
        // / 2^wexp <= 1 for every strut, and scales its sums by 2^(5 wexp)
        const uint32_t wbits = h_cnt[2 * ns + 3];
        float wmax = 0.0f;
        std::memcpy(&wmax, &wbits, 4);
        b->wexp = wmax > 0.0f ? (int32_t)std::ceil(0.2 * std::log2((double)wmax)) : 0;
        while (b->wexp < 64 && std::pow((double)wmax, 0.2) > std::ldexp(1.0, b->wexp)) ++b->wexp;
    }
    std::vector<uint32_t> vlo(h_cnt.begin(), h_cnt.begin() + ns);
    std::vector<uint32_t> vhi(h_cnt.begin() + ns, h_cnt.begin() + 2 * ns);
    if ((s = plan_groups(b, vlo, vhi, h_diff, h_rdiff))) return fail(s);

    // ---- per-strut arrays in edge-list order
    const size_t nb = std::max<size_t>(b->n_binned, 1);
    if ((s = b->alloc(&b->rec, nb * (L->dtype == LSL_F64 ? sizeof(StrutRec<double>)
                                                         : sizeof(StrutRec<float>)))) ||
        (s = b->alloc_t(&b->perm, nb)) || (s = b->alloc_t(&b->ranges, nb)) ||
        (s = b->alloc_t(&b->pranges, nb)) ||
        (s = b->alloc(&b->w, nb * b->esize())) || (s = b->alloc_t(&b->ends, nb)) ||
        (s = b->alloc_t(&b->line, nb)) || (s = b->alloc_t(&b->rho, nb)))
        return fail(s);
    if (b->n_binned) {
        he = hipMemcpyAsync(b->perm, perm_src, (size_t)b->n_binned * 4, hipMemcpyDeviceToDevice, st);
        if (he != hipSuccess) {
            set_error(std::string("lattice_bin: ") + hipGetErrorString(he));
            return fail(LSL_EDEVICE);
        }
        GatherArgs ga{};
        ga.nodes = L->nodes;
        ga.edges = L->edges;
        ga.weight = L->weight;
        ga.perm = b->perm;
        ga.ranges_by_id = rid;
        ga.pranges_by_id = prid;
        ga.n_binned = b->n_binned;
        ga.R = L->R;
        ga.support = L->support;
        ga.kernel = L->kernel;
        ga.sigma = L->sigma;
        ga.rec = b->rec;
        ga.ranges = b->ranges;
        ga.pranges = b->pranges;
        ga.w = b->w;
        ga.ends = b->ends;
        ga.line = b->line;
        ga.rho = b->rho;
        ga.wexp = b->wexp;
        if ((s = launch_gather(L->dtype, ga, st))) return fail(s);
    }
    he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
        set_error(std::string("lattice_bin: ") + hipGetErrorString(he));
        return fail(LSL_EDEVICE);
    }
    for (void* p : {(void*)klo, (void*)khi, (void*)vals, (void*)ka, (void*)va, (void*)rid,
                    (void*)prid, (void*)cnt, (void*)diff, (void*)stmp, (void*)ks0})
        b->release(p);

    // ---- resident-group buffers sized for the largest group
    size_t max_act = 1, max_pairs = 1, max_bk = 1, max_cand = 1, max_rows = 1;
    for (size_t g = 0; g < b->groups.size(); ++g) {
        const Group& Gr = b->groups[g];
        max_act = std::max<size_t>(max_act, Gr.n_active);
        max_pairs = std::max<size_t>(max_pairs, Gr.pairs);
        max_bk = std::max<size_t>(max_bk, Gr.n_buckets);
        max_rows = std::max<size_t>(max_rows, (size_t)(Gr.sb - Gr.sa + 1) * (size_t)b->nty *
                                                  (size_t)((b->ntx + kSegTiles - 1) / kSegTiles));
        max_cand = std::max<size_t>(max_cand, b->win_end[Gr.sb]);
    }
    b->cap_active = max_act;
    b->cap_pairs = max_pairs;
    b->cap_buckets = max_bk;
    if ((s = b->alloc_t(&b->active[0], max_act)) || (s = b->alloc_t(&b->active[1], max_act)) ||
        (s = b->alloc_t(&b->eoff, max_act + 1)) || (s = b->alloc_t(&b->toff, max_act + 1)) ||
        (s = b->alloc_t(&b->roffs, max_rows + 1)) || (s = b->alloc_t(&b->offsets, max_bk + 1)) ||
        (s = b->alloc_t(&b->k0, max_pairs)) ||
        (s = b->alloc_t(&b->v0, max_pairs)) || (s = b->alloc_t(&b->k1, max_pairs)) ||
        (s = b->alloc_t(&b->v1, max_pairs)) ||
        (s = b->alloc_t(&b->tmp, group_tmp_elems(max_pairs, max_act, max_cand, max_bk))) ||
        (s = b->alloc_t(&b->blk, max_cand / 2048 + 2)) || (s = b->alloc_t(&b->stats, 4)))
        return fail(s);
    if (!b->groups.empty() && (s = ensure_group(b, 0, st))) return fail(s);
    *out = b;
    return LSL_OK;
}

lsl_status lattice_bins_free(lattice_bins* b) {
    delete b;
    return LSL_OK;
}

namespace {
// device scratch from the cache, returned when it goes out of scope (callers
// synchronise the stream first)
struct CachedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    lsl_status get(size_t n) {
        bytes = DeviceCache::size_class(n);
        if (DeviceCache::get().alloc(&p, bytes) != hipSuccess) {
            hipGetLastError();
            p = nullptr;
            set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
            return LSL_ENOMEM;
        }
        return LSL_OK;
    }
    ~CachedBuf() {
        if (p) DeviceCache::get().release(p, bytes);
    }
};
}  // namespace

lsl_status lattice_support(const lsl_lattice* L, const double* print_dir, lsl_support* out,
                           void* grad_nodes, void* stream) {
    set_error("");
    LSL_CHECK(L != nullptr && print_dir != nullptr && out != nullptr, "NULL argument");
    LSL_CHECK(L->dtype == LSL_F32 || L->dtype == LSL_F64, "dtype must be LSL_F32 or LSL_F64");
    LSL_CHECK(L->n_nodes >= 1 && L->n_edges >= 0, "n_nodes >= 1 and n_edges >= 0 required");
    LSL_CHECK(L->n_nodes < ((int64_t)1 << 31) && L->n_edges < ((int64_t)1 << 30),
              "lattice too large");
    LSL_CHECK(L->nodes != nullptr && (L->n_edges == 0 || (L->edges && L->weight)),
              "lattice arrays are NULL");
    const double tn = std::sqrt(print_dir[0] * print_dir[0] + print_dir[1] * print_dir[1] +
                                print_dir[2] * print_dir[2]);
    LSL_CHECK(std::isfinite(tn) && tn > 0.0, "print_dir must be finite and non-zero");
    hipStream_t st = S(stream);
    SupportArgs a{};
    a.nodes = L->nodes;
    a.edges = L->edges;
    a.weight = L->weight;
    a.n_nodes = L->n_nodes;
    a.n_edges = L->n_edges;
    for (int i = 0; i < 3; ++i) a.t[i] = print_dir[i] / tn;
    const size_t np = support_part_elems(L->n_edges);
    CachedBuf small, te, sortb, offb;
    LSL_TRY(small.get((np + 8) * sizeof(double)));
    a.part = (double*)small.p;
    a.sums = a.part + np;
    a.err = (int*)(a.sums + 6);
    const size_t n2 = std::max<size_t>(2 * (size_t)L->n_edges, 1);
    if (grad_nodes) {
        LSL_TRY(te.get(std::max<size_t>(3 * (size_t)L->n_edges, 1) * sizeof(double)));
        LSL_TRY(sortb.get((4 * n2 + radix_tmp_elems(n2)) * sizeof(uint32_t)));
        LSL_TRY(offb.get(((size_t)L->n_nodes + 1) * sizeof(uint32_t)));
        a.grad = grad_nodes;
        a.te = (double*)te.p;
        a.k0 = (uint32_t*)sortb.p;
        a.v0 = a.k0 + n2;
        a.k1 = a.v0 + n2;
        a.v1 = a.k1 + n2;
        a.tmp = a.v1 + n2;
        a.off = (uint32_t*)offb.p;
    }
    LSL_TRY(fill_u32((uint32_t*)a.err, 0u, 1, st));
    LSL_TRY(launch_support(L->dtype, a, st));
    double h[6] = {0, 0, 0, 0, 0, 0};
    int herr = 0;
    LSL_HIP(hipMemcpyAsync(h, a.sums, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
    LSL_HIP(hipMemcpyAsync(&herr, a.err, sizeof(int), hipMemcpyDeviceToHost, st));
    LSL_HIP(hipStreamSynchronize(st));
    LSL_CHECK(herr == 0, "edge index out of range");
    out->risky_area = h[0];
    out->area = h[1];
    out->supported_length = h[2];
    out->length = h[3];
    out->n_supported = (int64_t)std::llround(h[4]);
    out->gamma = h[1] > 0.0 ? h[0] / h[1] : 0.0;
    out->psi = h[3] > 0.0 ? 100.0 * h[2] / h[3] : 0.0;
    return LSL_OK;
}

lsl_status lsl_cache_trim(int64_t* cached_bytes) {
    set_error("");
    if (cached_bytes) *cached_bytes = (int64_t)DeviceCache::get().cached();
    const lsl_status gs = GraphCache::get().trim();
    DeviceCache::get().trim();
    return gs;
}

lsl_status lsl_graph_cache_stats(int64_t* instantiated, int64_t* updated, int64_t* entries) {
    GraphCache::get().stats(instantiated, updated, entries);
    return LSL_OK;
}

lsl_status lattice_bins_info(const lattice_bins* b, lsl_bins_info* o) {
    LSL_CHECK(b != nullptr && o != nullptr, "NULL argument");
    o->n_edges = b->n_edges;
    o->n_nodes = b->n_nodes;
    o->n_binned = b->n_binned;
    o->total_pairs = (int64_t)b->total_pairs;
    o->max_group_pairs = (int64_t)b->max_group_pairs;
    o->device_bytes = b->dev_bytes;
    o->peak_device_bytes = b->peak_bytes;
    o->dtype = b->dtype;
    o->tile = b->tile;
    o->slab = b->slab;
    o->tiles_x = b->ntx;
    o->tiles_y = b->nty;
    o->n_slabs = b->n_slabs;
    o->n_groups = (int32_t)b->groups.size();
    o->current_group = b->cur_group;
    o->last_field_ms = b->last_field_ms;
    o->last_group_bin_ms = b->last_group_bin_ms;
    o->last_queue_ms = b->last_queue_ms;
    o->last_contour_ms = b->last_contour_ms;
    o->plane_group =
        (b->dtype == LSL_F32 && b->kernel == LSL_KERNEL_QUARTIC && !b->plane_ref) ? 8 : 1;
    o->last_backward_ms = -1.0;
    if (b->n_back > 0 && hipEventSynchronize(b->back_events[b->n_back - 1].ev[1]) == hipSuccess) {
        double acc = 0.0;
        bool ok = true;
        for (size_t i = 0; i < b->n_back && ok; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, b->back_events[i].ev[0], b->back_events[i].ev[1]) ==
                hipSuccess)
                acc += ms;
            else
                ok = false;
        }
        if (ok) o->last_backward_ms = acc;
    }
    hipGetLastError();
    return LSL_OK;
}

lsl_status lattice_bins_group(const lattice_bins* b, int32_t g, int32_t* s0, int32_t* s1,
                              int64_t* pairs) {
    LSL_CHECK(b != nullptr, "bins handle is NULL");
    LSL_CHECK(g >= 0 && g < (int32_t)b->groups.size(), "group index out of range");
    if (s0) *s0 = b->groups[g].sa;
    if (s1) *s1 = b->groups[g].sb;
    if (pairs) *pairs = (int64_t)b->groups[g].pairs;
    return LSL_OK;
}

lsl_status lattice_bins_export(lattice_bins* b, int32_t g, int64_t* offsets, int32_t* ids,
                               void* stream) {
    LSL_CHECK(b != nullptr, "bins handle is NULL");
    LSL_CHECK(g >= 0 && g < (int32_t)b->groups.size(), "group index out of range");
    hipStream_t st = S(stream);
    LSL_TRY(ensure_group(b, g, st));
    const Group& G = b->groups[g];
    if (offsets) k_u32_to_i64<<<nblk(G.n_buckets + 1), 256, 0, st>>>(b->offsets, offsets, G.n_buckets + 1);
    if (ids && G.pairs) k_ids_to_edges<<<nblk(G.pairs), 256, 0, st>>>(b->ids, b->perm, ids, G.pairs);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status lattice_bins_order(const lattice_bins* b, int32_t* order, void* stream) {
    LSL_CHECK(b != nullptr && order != nullptr, "NULL argument");
    if (b->n_binned)
        k_copy_i32<<<nblk(b->n_binned), 256, 0, S(stream)>>>(b->perm, order, b->n_binned);
    LSL_HIP(hipGetLastError());
    return LSL_OK;
}

lsl_status slice_field(lattice_bins* b, int32_t k0, int32_t nk, void* field, uint32_t* bits,
                       void* stream) {
    set_error("");
    LSL_TRY(check_range(b, k0, nk));
    LSL_CHECK(field != nullptr, "field is NULL");
    hipStream_t st = S(stream);
    const size_t plane = (size_t)b->grid.W * (size_t)b->grid.H;
    if (b->n_binned == 0 || b->groups.empty()) {
        LSL_TRY(fill_bytes0(field, (size_t)nk * plane * b->esize(), st));
        if (bits)
            LSL_TRY(fill_bytes0(bits, (size_t)nk * b->grid.H * ((b->grid.W + 31) / 32) * 4, st));
        return LSL_OK;
    }
    // binary images: block-major in library scratch, then the caller's
    // row-major copy
    if (bits) LSL_TRY(ensure_cbits(b, nk, st));
    // the plan covers every slab, so every block of every plane is written
    LSL_TRY(for_groups(b, k0, nk, [&](int g, int s_lo, int s_hi) -> lsl_status {
        LSL_TRY(ensure_group(b, g, st));
        FieldArgs a = field_args(b, k0, nk, field);
        a.bits_blk = bits ? (uint64_t*)b->cbits : nullptr;
        a.n_pairs = (uint32_t)b->groups[g].pairs;
        a.group_s0 = b->groups[g].sa;
        a.s_lo = s_lo;
        a.s_hi = s_hi;
        return launch_field(b->dtype, a, false, st);
    }));
    if (bits) LSL_TRY(launch_bits_rows((const uint64_t*)b->cbits, nk, b->grid.W, b->grid.H, bits, st));
    return LSL_OK;
}

lsl_status slice_field_stats(lattice_bins* b, int32_t k0, int32_t nk, int64_t* counts,
                             void* stream) {
    set_error("");
    LSL_TRY(check_range(b, k0, nk));
    LSL_CHECK(counts != nullptr, "counts is NULL");
    hipStream_t st = S(stream);
    LSL_TRY(fill_bytes0(b->stats, 4 * 8, st));
    if (b->n_binned && !b->groups.empty()) {
        LSL_TRY(for_groups(b, k0, nk, [&](int g, int s_lo, int s_hi) -> lsl_status {
            LSL_TRY(ensure_group(b, g, st));
            FieldArgs a = field_args(b, k0, nk, nullptr);
            a.n_pairs = (uint32_t)b->groups[g].pairs;
            a.group_s0 = b->groups[g].sa;
            a.s_lo = s_lo;
            a.s_hi = s_hi;
            a.stats = b->stats;
            return launch_field(b->dtype, a, true, st);
        }));
    }
    unsigned long long h[4] = {0, 0, 0, 0};
    LSL_HIP(hipMemcpyAsync(h, b->stats, sizeof(h), hipMemcpyDeviceToHost, st));
    LSL_HIP(hipStreamSynchronize(st));
    counts[0] = (int64_t)h[0];
    counts[1] = (int64_t)h[1];
    counts[2] = (int64_t)h[2];
    if (b->n_binned == 0) counts[2] = (int64_t)nk * b->grid.W * b->grid.H;
    return LSL_OK;
}

lsl_status slice_contours(const lattice_bins* cb, int32_t nk, const void* field, float* segs,
                          int64_t capacity, int64_t* offsets, uint8_t* case_codes, int64_t* total,
                          void* stream) {
    set_error("");
    LSL_CHECK(cb != nullptr, "bins handle is NULL");
    LSL_CHECK(nk >= 1, "nk must be >= 1");
    LSL_CHECK(field != nullptr && offsets != nullptr, "field and offsets are required");
    LSL_CHECK(capacity >= 0, "capacity must be >= 0");
    LSL_CHECK(capacity == 0 || segs != nullptr, "segs is NULL");
    lattice_bins* b = const_cast<lattice_bins*>(cb);   // scratch only
    hipStream_t st = S(stream);
    LSL_TRY(b->grow(&b->ctmp, &b->ctmp_elems, contour_tmp_elems(nk, b->grid.W, b->grid.H), st));
    LSL_TRY(ensure_cbits(b, nk, st));
    // the binary images (block-major), then marching squares on them
    const uint64_t* img = (const uint64_t*)b->cbits;
    LSL_TRY(launch_bits_blk(b->dtype, field, nk, b->grid.W, b->grid.H, b->C,
                            (uint64_t*)b->cbits, st));
    LSL_TRY(launch_contours_count(img, nk, b->grid.W, b->grid.H, offsets, case_codes, b->ctmp,
                                  nullptr, st));
    int64_t tot = 0;
    LSL_HIP(hipMemcpyAsync(&tot, offsets + nk, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LSL_HIP(hipStreamSynchronize(st));
    if (total) *total = tot;
    if (tot > capacity) {
        set_error("slice_contours: " + std::to_string(tot) + " segments exceed capacity " +
                  std::to_string(capacity));
        return LSL_ECAPACITY;
    }
    if (tot > 0)
        LSL_TRY(launch_contours_emit(img, nk, b->grid.W, b->grid.H, b->ctmp, nullptr, segs,
                                     capacity, st));
    return LSL_OK;
}


lsl_status slice_polylines(const lattice_bins* cb, int32_t nk, const void* field, float* segs,
                           int64_t capacity, int64_t* offsets, int32_t* chain, int32_t* rank,
                           int64_t* total, void* stream) {
    set_error("");
    LSL_CHECK(cb != nullptr, "bins handle is NULL");
    LSL_CHECK(nk >= 1, "nk must be >= 1");
    LSL_CHECK(field != nullptr && offsets != nullptr, "field and offsets are required");
    LSL_CHECK(capacity >= 0, "capacity must be >= 0");
    LSL_CHECK(capacity == 0 || segs != nullptr, "segs is NULL");
    LSL_CHECK((chain == nullptr) == (rank == nullptr), "chain and rank go together");
    lattice_bins* b = const_cast<lattice_bins*>(cb);   // scratch only
    hipStream_t st = S(stream);
    LSL_TRY(b->grow(&b->ctmp, &b->ctmp_elems, contour_tmp_elems(nk, b->grid.W, b->grid.H), st));
    LSL_TRY(ensure_cbits(b, nk, st));
    const uint64_t* img = (const uint64_t*)b->cbits;
    LSL_TRY(launch_bits_blk(b->dtype, field, nk, b->grid.W, b->grid.H, b->C,
                            (uint64_t*)b->cbits, st));
    LSL_TRY(launch_contours_count(img, nk, b->grid.W, b->grid.H, offsets, nullptr, b->ctmp,
                                  nullptr, st));
    std::vector<int64_t> h_off((size_t)nk + 1);
    LSL_HIP(hipMemcpyAsync(h_off.data(), offsets, h_off.size() * 8, hipMemcpyDeviceToHost, st));
    LSL_HIP(hipStreamSynchronize(st));
    const int64_t tot = h_off[nk];
    if (total) *total = tot;
    if (tot > capacity) {
        set_error("slice_polylines: " + std::to_string(tot) + " segments exceed capacity " +
                  std::to_string(capacity));
        return LSL_ECAPACITY;
    }
    LSL_CHECK(tot < ((int64_t)1 << 31) / 2, "slice_polylines: too many segments in one call");
    if (tot == 0) return LSL_OK;
    int64_t longest = 1;
    for (int32_t k = 0; k < nk; ++k) longest = std::max<int64_t>(longest, h_off[k + 1] - h_off[k]);
    int32_t rounds = 1;
    while (((int64_t)1 << (rounds - 1)) < longest) ++rounds;
    LSL_TRY(b->grow(&b->pscratch, &b->pscratch_elems, polyline_scratch_elems((uint64_t)tot), st));
    return launch_polylines(img, field, b->dtype, b->C, nk, b->grid.W, b->grid.H, b->ctmp, offsets,
                            (uint64_t)tot, rounds, segs, b->pscratch, chain, rank, st);
}

lsl_status slice_density(const lattice_bins* b, int32_t nk, const void* field, int32_t vx,
                         int32_t vy, int32_t vz, float* density, void* stream) {
    set_error("");
    LSL_CHECK(b != nullptr, "bins handle is NULL");
    LSL_CHECK(field != nullptr && density != nullptr, "field and density are required");
    DensityArgs a{};
    LSL_TRY(density_plan(nk, b->grid.W, b->grid.H, vx, vy, vz, &a));
    return launch_density(b->dtype, a, field, b->C, density, S(stream));
}

lsl_status slice_occupancy_loss(const lattice_bins* cb, int32_t nk, const void* field,
                                const void* target, double tau, void* grad_field, double* loss,
                                void* stream) {
    set_error("");
    LSL_CHECK(cb != nullptr, "bins handle is NULL");
    LSL_CHECK(nk >= 1, "nk must be >= 1");
    LSL_CHECK(field != nullptr && target != nullptr, "field and target are required");
    LSL_CHECK(std::isfinite(tau) && tau > 0.0, "tau must be finite and > 0");
    lattice_bins* b = const_cast<lattice_bins*>(cb);   // scratch only
    hipStream_t st = S(stream);
    const size_t n = (size_t)nk * (size_t)b->grid.W * (size_t)b->grid.H;
    const size_t need = occupancy_blocks(n);
    LSL_TRY(b->grow(&b->dscratch, &b->dscratch_elems, need, st));
    return launch_occupancy_loss(b->dtype, field, target, n, b->C, tau, grad_field, loss,
                                 b->dscratch, st);
}

lsl_status slice_occupancy_loss_static(const lattice_bins* cb, int32_t nk, const void* field,
                                       const void* target, double tau, void* grad_field,
                                       double* loss, void* stream) {
    set_error("");
    LSL_CHECK(cb != nullptr, "bins handle is NULL");
    LSL_CHECK(nk >= 1, "nk must be >= 1");
    LSL_CHECK(field != nullptr && target != nullptr, "field and target are required");
    LSL_CHECK(std::isfinite(tau) && tau > 0.0, "tau must be finite and > 0");
    const size_t n = (size_t)nk * (size_t)cb->grid.W * (size_t)cb->grid.H;
    const size_t need = occupancy_blocks(n);
    if (need > kStaticScratchElems) {
        set_error("slice_occupancy_loss_static: " + std::to_string(need) +
                  " partial sums exceed the static scratch of " +
                  std::to_string(kStaticScratchElems));
        return LSL_ECAPACITY;
    }
    double* part = nullptr;
    LSL_TRY(static_scratch(&part));
    return launch_occupancy_loss(cb->dtype, field, target, n, cb->C, tau, grad_field, loss,
                                 part, S(stream));
}

lsl_status slice_density_loss(const lattice_bins* cb, int32_t nk, const void* field, int32_t vx,
                              int32_t vy, int32_t vz, const float* target, double tau,
                              float* soft_density, void* grad_field, double* loss,
                              void* stream) {
    set_error("");
    LSL_CHECK(cb != nullptr, "bins handle is NULL");
    LSL_CHECK(field != nullptr && target != nullptr, "field and target are required");
    LSL_CHECK(std::isfinite(tau) && tau > 0.0, "tau must be finite and > 0");
    lattice_bins* b = const_cast<lattice_bins*>(cb);   // scratch only
    hipStream_t st = S(stream);
    DensityArgs a{};
    LSL_TRY(density_plan(nk, b->grid.W, b->grid.H, vx, vy, vz, &a));
    const size_t need = density_scratch_elems(a);
    LSL_TRY(b->grow(&b->dscratch, &b->dscratch_elems, need, st));
    return launch_density_loss(b->dtype, a, field, b->C, tau, target, soft_density, grad_field,
                               loss, b->dscratch, st);
}

}  // extern "C"

namespace {

// Node -> (strut, end) incidence list in edge-list order, built once.
lsl_status ensure_node_csr(lattice_bins* b, hipStream_t st) {
    if (b->node_off) return LSL_OK;
    const size_t n2 = 2 * (size_t)std::max<uint32_t>(b->n_binned, 1);
    uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr, *v1 = nullptr, *tmp = nullptr;
    lsl_status s;
    if ((s = b->alloc_t(&k0, n2)) || (s = b->alloc_t(&v0, n2)) || (s = b->alloc_t(&k1, n2)) ||
        (s = b->alloc_t(&v1, n2)) || (s = b->alloc_t(&tmp, radix_tmp_elems(n2))) ||
        (s = b->alloc_t(&b->node_off, (size_t)b->n_nodes + 1)) ||
        (s = b->alloc_t(&b->node_inc, n2)))
        return s;
    const size_t n = 2 * (size_t)b->n_binned;
    LSL_TRY(launch_node_keys(b->ends, b->n_binned, k0, v0, st));
    int bits = 0;
    while (bits < 32 && (1ull << bits) < (uint64_t)b->n_nodes) ++bits;
    int which = 0;
    LSL_TRY(radix_sort_pairs(k0, v0, k1, v1, n, bits, tmp, &which, st));
    const uint32_t* ks = which ? k1 : k0;
    const uint32_t* vs = which ? v1 : v0;
    LSL_TRY(launch_node_offsets(ks, n, b->n_nodes, b->node_off, st));
    if (n) LSL_HIP(hipMemcpyAsync(b->node_inc, vs, n * 4, hipMemcpyDeviceToDevice, st));
    LSL_HIP(hipStreamSynchronize(st));
    for (void* p : {(void*)k0, (void*)v0, (void*)k1, (void*)v1, (void*)tmp}) b->release(p);
    return LSL_OK;
}

BackArgs back_args(const lattice_bins* b, int g, int32_t k0, int32_t nk, int s_lo, int s_hi,
                   const void* grad) {
    BackArgs a{};
    a.rec = b->rec;
    a.offsets = b->offsets;
    a.ids = b->ids;
    a.n_binned = b->n_binned;
    a.n_pairs = (uint32_t)b->groups[g].pairs;
    a.ntx = b->ntx;
    a.nty = b->nty;
    a.tile = b->tile;
    a.slab = b->slab;
    a.group_s0 = b->groups[g].sa;
    a.s_lo = s_lo;
    a.s_hi = s_hi;
    a.k0 = k0;
    a.nk = nk;
    a.W = b->grid.W;
    a.H = b->grid.H;
    a.x0 = b->grid.x0;
    a.y0 = b->grid.y0;
    a.dx = b->grid.dx;
    a.dy = b->grid.dy;
    a.z0 = b->grid.z0;
    a.dz = b->grid.dz;
    a.R = b->R;
    a.strut_R = b->strut_R ? 1 : 0;
    a.emi = b->emi;
    a.grad = grad;
    a.partial = b->partial;
    a.line = b->line;
    a.plane_ref = b->plane_ref ? 1 : 0;
    a.wide = b->wide ? 1 : 0;
    return a;
}

// What decides the kernels a slab group's graphs record (the cached graphs
// of one shape differ only in launch arguments).
struct GraphShape {
    int32_t dtype, kernel, strut_R, plane_ref, slab, tile, phase;
    int32_t field, bits, segs, slot;
};

// Enqueues one phase of a group's part of slice_batch on `st`:
//   0: work queue (descending cost) and counter reset
//   1: persistent field kernel
//   2: binary image and contours (positions continue from the device-side
//      running total of earlier groups)
lsl_status batch_group_work(lattice_bins* b, int g, int32_t k0, int32_t nk, int s_lo, int s_hi,
                            void* field, uint32_t* bits, float* segs, int64_t capacity,
                            int64_t* offsets, int phase, hipStream_t st) {
    const int kg0 = std::max(k0, s_lo * b->slab);
    const int kg1 = std::min(k0 + nk, (s_hi + 1) * b->slab);
    const int nkg = kg1 - kg0;
    const size_t plane = (size_t)b->grid.W * (size_t)b->grid.H;
    const size_t words = (size_t)(b->grid.W + 31) / 32;
    // this group's planes: the caller's field (if any) and binary images (the
    // caller's, or library scratch)
    void* fbase = field ? (void*)((char*)field + (size_t)(kg0 - k0) * plane * b->esize()) : nullptr;
    // binary images: block-major in library scratch; the caller's bits, if
    // any, get a row-major copy
    uint32_t* bbase = bits ? bits + (size_t)(kg0 - k0) * (size_t)b->grid.H * words : nullptr;
    FieldArgs a = field_args(b, kg0, nkg, fbase);
    a.bits_blk = (uint64_t*)b->cbits;
    const uint64_t* img = (const uint64_t*)b->cbits;
    a.n_pairs = (uint32_t)b->groups[g].pairs;
    a.group_s0 = b->groups[g].sa;
    a.s_lo = s_lo;
    a.s_hi = s_hi;
    const uint32_t n_items = (uint32_t)((s_hi - s_lo + 1) * b->ntx * b->nty);
    uint32_t* qk = b->queue_buf;
    uint32_t* qv = qk + b->queue_cap;
    uint32_t* qk2 = qv + b->queue_cap;
    uint32_t* qv2 = qk2 + b->queue_cap;
    uint32_t* counter = qv2 + b->queue_cap;
    uint32_t* qtmp = counter + 64;
    unsigned long long* base = (unsigned long long*)(counter + 32);
    if (phase == 0) {
        const uint32_t* queue = nullptr;
        LSL_TRY(launch_queue_build(a, qk, qv, qk2, qv2, n_items, qtmp, &queue, st));
        LSL_TRY(fill_u32(counter, 0u, 1, st));
        b->queue_in_alt = queue != qv;
        return LSL_OK;
    }
    if (phase == 1) {
        BatchArgs ba{};
        ba.f = a;
        ba.queue = b->queue_in_alt ? qv2 : qv;
        ba.n_items = n_items;
        ba.counter = counter;
        return launch_persistent(b->dtype, ba, persistent_blocks(b->dtype, b->slab), st);
    }
    LSL_TRY(launch_contours_count(img, nkg, b->grid.W, b->grid.H, offsets + (kg0 - k0), nullptr,
                                  b->ctmp, base, st));
    LSL_TRY(launch_contours_emit(img, nkg, b->grid.W, b->grid.H, b->ctmp, base, segs, capacity,
                                 st));
    if (bbase) LSL_TRY(launch_bits_rows(img, nkg, b->grid.W, b->grid.H, bbase, st));
    return LSL_OK;
}

// Records fn's launches on the capture stream `cap` into *graph (owned by
// the caller afterwards).
lsl_status capture(hipStream_t cap, hipGraph_t* graph,
                   const std::function<lsl_status(hipStream_t)>& fn) {
    *graph = nullptr;
    LSL_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    lsl_status ws = fn(cap);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(cap, &g);
    if (ws != LSL_OK) {
        if (g) hipGraphDestroy(g);
        hipGetLastError();
        return ws;
    }
    if (ce != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        hipGetLastError();
        set_error(std::string("slice_batch: graph capture failed: ") + hipGetErrorString(ce));
        return LSL_EDEVICE;
    }
    *graph = g;
    return LSL_OK;
}

}  // namespace

extern "C" {

lsl_status slice_field_backward(lattice_bins* b, int32_t k0, int32_t nk, const void* grad_field,
                                void* grad_weight, void* grad_nodes, int32_t accumulate,
                                void* stream) {
    set_error("");
    LSL_TRY(check_range(b, k0, nk));
    LSL_CHECK(grad_field != nullptr, "grad_field is NULL");
    LSL_CHECK(b->kernel == LSL_KERNEL_QUARTIC,
              "slice_field_backward covers the quartic kernel only");
    hipStream_t st = S(stream);
    b->n_back = 0;
    if (!b->acc) LSL_TRY(b->alloc_t(&b->acc, (size_t)std::max<uint32_t>(b->n_binned, 1) * 7));
    if (!b->partial) LSL_TRY(b->alloc(&b->partial, b->cap_pairs * 9 * b->esize()));
    if (!b->emi) LSL_TRY(b->alloc_t(&b->emi, b->cap_pairs));
    if (!b->inv) LSL_TRY(b->alloc_t(&b->inv, std::max<uint32_t>(b->n_binned, 1)));
    LSL_TRY(ensure_node_csr(b, st));
    LSL_TRY(fill_bytes0(b->acc, (size_t)std::max<uint32_t>(b->n_binned, 1) * 7 * 8, st));
    if (b->n_binned && !b->groups.empty()) {
        LSL_TRY(for_groups(b, k0, nk, [&](int g, int s_lo, int s_hi) -> lsl_status {
            LSL_TRY(ensure_group(b, g, st));
            const Group& G = b->groups[g];
            if (G.pairs == 0) return LSL_OK;
            if (b->emi_group != g) {
                EmiArgs ea{};
                ea.keys = b->skeys;
                ea.offsets = b->offsets;
                ea.n_buckets = G.n_buckets;
                ea.ids = b->ids;
                ea.active = b->active[b->cur_buf];
                ea.eoff = b->eoff;
                ea.ranges = b->ranges;
                ea.n_pairs = (uint32_t)G.pairs;
                ea.n_active = G.n_active;
                ea.sa = G.sa;
                ea.ntx = b->ntx;
                ea.nty = b->nty;
                ea.inv = b->inv;
                ea.emi = b->emi;
                LSL_TRY(group_emi(ea, st));
                b->emi_group = g;
            }
            BackArgs a = back_args(b, g, k0, nk, s_lo, s_hi, grad_field);
            if (b->back_events.size() <= b->n_back) {
                lattice_bins::EvPair bp{};
                for (auto& e : bp.ev) LSL_HIP(hipEventCreate(&e));
                b->back_events.push_back(bp);
            }
            hipEvent_t* bev = b->back_events[b->n_back++].ev;
            LSL_HIP(hipEventRecord(bev[0], st));
            LSL_TRY(launch_backward(b->dtype, a, st));
            LSL_HIP(hipEventRecord(bev[1], st));
            ReduceArgs r{};
            r.partial = b->partial;
            r.active = b->active[b->cur_buf];
            r.n_active = G.n_active;
            r.eoff = b->eoff;
            r.rec = b->rec;
            r.w = b->w;
            r.R = b->R;
            r.strut_R = b->strut_R ? 1 : 0;
            r.normalized = b->dtype == LSL_F32 ? 1 : 0;
            r.acc = b->acc;
            return launch_reduce(b->dtype, r, b->ranges, G.sa, s_lo, s_hi, (uint32_t)G.pairs,
                                 b->n_binned, st);
        }));
    }
    ScatterArgs sc{};
    sc.acc = b->acc;
    sc.perm = b->perm;
    sc.n_binned = b->n_binned;
    sc.n_edges = b->n_edges;
    sc.n_nodes = b->n_nodes;
    sc.node_off = b->node_off;
    sc.node_inc = b->node_inc;
    sc.grad_weight = grad_weight;
    sc.grad_nodes = grad_nodes;
    sc.accumulate = accumulate;
    return launch_scatter(b->dtype, sc, st);
}

lsl_status slice_batch(lattice_bins* b, int32_t k0, int32_t nk, void* field, uint32_t* bits,
                       float* segs, int64_t capacity, int64_t* offsets, int64_t* total,
                       void* stream) {
    set_error("");
    LSL_TRY(check_range(b, k0, nk));
    LSL_CHECK(offsets != nullptr, "offsets is NULL");
    LSL_CHECK(capacity >= 0 && (capacity == 0 || segs != nullptr), "bad segment buffer");
    hipStream_t st = S(stream);
    const size_t plane = (size_t)b->grid.W * (size_t)b->grid.H;
    // scratch sized for the largest group
    size_t max_items = 1, max_planes = 1;
    for (auto& G : b->groups) {
        max_items = std::max<size_t>(max_items, (size_t)(G.sb - G.sa + 1) * b->ntx * b->nty);
        max_planes = std::max<size_t>(max_planes, (size_t)(G.sb - G.sa + 1) * b->slab);
    }
    max_planes = std::min<size_t>(max_planes, (size_t)nk);
    if (b->queue_cap < max_items) {
        LSL_HIP(hipStreamSynchronize(st));
        b->release(b->queue_buf);
        b->queue_buf = nullptr;
        b->queue_cap = 0;
        LSL_TRY(b->alloc_t(&b->queue_buf, 4 * max_items + 64 + radix_tmp_elems(max_items)));
        b->queue_cap = max_items;
    }
    LSL_TRY(b->grow(&b->ctmp, &b->ctmp_elems,
                    contour_tmp_elems((int32_t)max_planes, b->grid.W, b->grid.H), st));
    LSL_TRY(ensure_cbits(b, (int32_t)max_planes, st));
    uint32_t* counter = b->queue_buf + 4 * b->queue_cap;
    unsigned long long* base = (unsigned long long*)(counter + 32);
    LSL_TRY(fill_bytes0(base, 8, st));
    if (b->n_binned == 0 || b->groups.empty()) {
        // nothing binned: empty field, empty images, no segments
        if (field) LSL_TRY(fill_bytes0(field, (size_t)nk * plane * b->esize(), st));
        if (bits)
            LSL_TRY(fill_bytes0(bits, (size_t)nk * b->grid.H * ((b->grid.W + 31) / 32) * 4, st));
        LSL_TRY(fill_bytes0(offsets, (size_t)(nk + 1) * 8, st));
        if (total) *total = 0;
        LSL_HIP(hipStreamSynchronize(st));
        b->last_field_ms = b->last_group_bin_ms = b->last_queue_ms = b->last_contour_ms = 0.0;
        return LSL_OK;
    }
    hipStream_t cap = nullptr;
    size_t n_call_groups = 0;
    LSL_TRY(for_groups(b, k0, nk, [&](int g, int s_lo, int s_hi) -> lsl_status {
        if (b->stage_events.size() <= n_call_groups) {
            lattice_bins::StageEvents se{};
            for (auto& e : se.ev) LSL_HIP(hipEventCreate(&e));
            b->stage_events.push_back(se);
        }
        hipEvent_t* ev = b->stage_events[n_call_groups++].ev;
        LSL_HIP(hipEventRecord(ev[0], st));
        LSL_TRY(ensure_group(b, g, st));
        // the group's three phases, recorded on the capture stream, then
        // launched through the process's graph cache: the launch shape (what
        // decides which kernels run) and which of the shape's two entries
        // this group takes
        if (!cap) LSL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t gr[3] = {nullptr, nullptr, nullptr};
        lsl_status cs = LSL_OK;
        for (int ph = 0; ph < 3 && cs == LSL_OK; ++ph)
            cs = capture(cap, &gr[ph], [&](hipStream_t cs_st) {
                return batch_group_work(b, g, k0, nk, s_lo, s_hi, field, bits, segs, capacity,
                                        offsets, ph, cs_st);
            });
        // the captures took host time: the group's binning stage ends here
        if (cs == LSL_OK && hipEventRecord(ev[1], st) != hipSuccess) cs = LSL_EDEVICE;
        for (int ph = 0; ph < 3 && cs == LSL_OK; ++ph) {
            GraphShape shape{b->dtype,   b->kernel,        b->strut_R ? 1 : 0,
                             b->plane_ref ? 1 : 0, b->slab, b->tile, ph,
                             field ? 1 : 0, bits ? 1 : 0, capacity > 0 ? 1 : 0,
                             (int32_t)((n_call_groups - 1) & 1)};
            std::vector<unsigned char> key((unsigned char*)&shape,
                                           (unsigned char*)&shape + sizeof(shape));
            cs = GraphCache::get().launch(key, gr[ph], st);
            if (cs == LSL_OK && hipEventRecord(ev[2 + ph], st) != hipSuccess) cs = LSL_EDEVICE;
        }
        for (auto& x : gr)
            if (x) hipGraphDestroy(x);
        return cs;
    }));
    if (cap) hipStreamDestroy(cap);
    unsigned long long tot = 0;
    LSL_HIP(hipMemcpyAsync(&tot, base, 8, hipMemcpyDeviceToHost, st));
    LSL_HIP(hipStreamSynchronize(st));
    // stage times of this call from its event sets
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    bool ok = true;
    for (size_t i = 0; i < n_call_groups && ok; ++i)
        for (int q = 0; q < 4 && ok; ++q) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, b->stage_events[i].ev[q], b->stage_events[i].ev[q + 1]) ==
                hipSuccess)
                acc[q] += ms;
            else
                ok = false;
        }
    if (!ok) hipGetLastError();
    b->last_group_bin_ms = ok ? acc[0] : -1.0;
    b->last_queue_ms = ok ? acc[1] : -1.0;
    b->last_field_ms = ok ? acc[2] : -1.0;
    b->last_contour_ms = ok ? acc[3] : -1.0;
    if (total) *total = (int64_t)tot;
    if ((int64_t)tot > capacity) {
        set_error("slice_batch: " + std::to_string(tot) + " segments exceed capacity " +
                  std::to_string(capacity));
        return LSL_ECAPACITY;
    }
    return LSL_OK;
}

}  // extern "C"
