// Launcher interfaces between the C-ABI host code and the kernel files.
#pragma once

#include "common.hpp"

namespace lsl {

// ----------------------------------------------------------------- prep.hip
struct PrepArgs {
    const void* nodes;
    const int32_t* edges;
    const void* weight;
    int64_t n_nodes, n_edges;
    double R;
    double x0, y0, z0, inv_dx, inv_dy, inv_dz;
    int32_t W, H, S;
    int32_t tile, slab, n_slabs;
    // outputs, indexed by edge id
    uint32_t* key_lo;
    uint32_t* key_hi;                 // float64 lattices only
    uint32_t* vals;                   // edge ids
    SRange* ranges;
    PRange* pranges;
    // plan histograms
    uint32_t* cnt_lo;                 // [n_slabs] struts whose first slab is s
    uint32_t* cnt_hi;                 // [n_slabs] struts whose last slab is s
    unsigned long long* pair_diff;    // [n_slabs + 1] difference array of pairs
    uint32_t* row_diff;               // [n_slabs + 1] difference array of (strut, tile row,
                                      // column segment) cells, modulo 2^32
    uint32_t* n_binned;
    uint32_t* err;                    // bit 0 index, 1 weight, 2 node, 3 support, 4 sigma
    uint32_t* min_support;            // ~(float bits) of the smallest binned support, max-reduced
    uint32_t* max_wr;                 // float bits of the largest r R of a binned strut, max-reduced
    // variants
    const void* support;              // [n_edges] per-strut supports, or null (R for all)
    uint32_t* key_s0;                 // [n_edges] first slab (n_slabs if not binned), or null
    double max_r_over_sigma;          // > 0: reject supports above this many sigma
    double sigma;
    int32_t keep_zero;                // 1: bin struts of weight 0 too
};
lsl_status launch_prep(int dtype, const PrepArgs& a, hipStream_t st);

struct GatherArgs {
    const void* nodes;
    const int32_t* edges;
    const void* weight;
    const uint32_t* perm;             // [n_binned] sorted position -> edge id
    const SRange* ranges_by_id;
    const PRange* pranges_by_id;
    int64_t n_binned;
    double R;
    const void* support;              // per-strut supports or null
    int32_t kernel;                   // LSL_KERNEL_*
    double sigma;
    void* rec;                        // StrutRec<T> [n_binned]; pad holds R_j with supports
    SRange* ranges;                   // [n_binned]
    PRange* pranges;                  // [n_binned]
    void* w;                          // T [n_binned]
    int2* ends;                       // [n_binned]
    double4* line;                    // [n_binned] (u_x, u_y, u_z, L) of each strut, float64
    float* rho;                       // [n_binned] (r R)^(1/5) / 2^wexp (float32 field kernel)
    int32_t wexp;
};
lsl_status launch_gather(int dtype, const GatherArgs& a, hipStream_t st);
lsl_status launch_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst,
                             size_t n, hipStream_t st);

// ------------------------------------------------------------------ bin.hip
struct GroupBuffers {
    // inputs
    const SRange* ranges;             // [n_binned]
    // active lists (double buffered by the caller)
    const uint32_t* prev_active;      // may be null
    uint32_t n_prev;
    uint32_t range_lo, range_hi;      // sorted positions [lo, hi) to consider
    uint32_t* active;                 // out [n_active]
    uint32_t n_active;
    int32_t sa, sb;                   // slabs of the group
    int32_t ntx, nty;
    uint32_t n_pairs;
    uint32_t n_cells;                 // (slab, tile row, column segment, strut) cells,
                                      // <= n_pairs
    uint32_t n_buckets;
    // outputs
    uint32_t* eoff;                   // [n_active + 1] pairs before each active strut
    uint32_t* toff;                   // [n_active + 1] scratch: cells before each
    uint32_t* roffs;                  // [(sb - sa + 1) nty nseg + 1] scratch: row-segment CSR
    uint32_t* offsets;                // [n_buckets + 1]
    uint32_t* k0; uint32_t* v0; uint32_t* k1; uint32_t* v1;   // [n_pairs] work buffers
    uint32_t** keys_out;              // out: the buffer group_emi fills with the entries'
                                      // bucket keys (k0 or k1)
    const uint32_t** ids_out;         // out: bucket entries, edge-list positions (v0 or v1)
    uint32_t* tmp;                    // scan / sort scratch
    uint32_t* blk;                    // compaction block counts
};
size_t group_tmp_elems(size_t n_pairs, size_t n_active, size_t n_cand, size_t n_buckets);
lsl_status bin_group(const GroupBuffers& g, hipStream_t st);

// Emission index of every bucket entry of the resident group (the position
// of the (strut, bucket) pair in the strut-major emission order), rebuilt
// from the entry's bucket, its strut and the strut's box.  keys receives
// every entry's bucket (from the offsets), inv ([n_binned], scratch) the
// inverse of the active list.
struct EmiArgs {
    uint32_t* keys;                   // [n_pairs] out: bucket of each entry
    const uint32_t* offsets;          // [n_buckets + 1]
    uint32_t n_buckets;
    const uint32_t* ids;              // [n_pairs] edge-list positions
    const uint32_t* active;           // [n_active]
    const uint32_t* eoff;             // [n_active + 1]
    const SRange* ranges;             // [n_binned]
    uint32_t n_pairs, n_active;
    int32_t sa, ntx, nty;
    uint32_t* inv;
    uint32_t* emi;                    // out [n_pairs]
};
lsl_status group_emi(const EmiArgs& a, hipStream_t st);

// ---------------------------------------------------------------- field.hip
struct FieldArgs {
    const void* rec;
    const double4* line;              // [n_binned] direction and length of rec[] (float64)
    const float* rho;                 // [n_binned] length scale of rec[] (float32 kernel)
    int32_t wexp;                     // the float32 kernel's sums times 2^(5 wexp) are the field
    const uint32_t* offsets;
    const uint32_t* ids;
    uint32_t n_binned, n_pairs;       // bounds of rec[] and ids[]
    int32_t ntx, nty, tile, slab;
    int32_t group_s0;                 // first slab of the resident group
    int32_t s_lo, s_hi;               // slabs to evaluate (absolute)
    int32_t k0, nk;                   // planes written: [k0, k0+nk)
    int32_t W, H;
    double x0, y0, dx, dy, z0, dz, R;
    const PRange* pranges;            // [n_binned] pixel and plane ranges of rec[]
    int32_t strut_R;                  // 1: strut j's support is rec[j].pad, else R
    int32_t kernel;                   // LSL_KERNEL_*
    double gk1, gk2, gc0;             // Gaussian: 1/(sigma sqrt 2), 1/(2 sigma^2), sigma sqrt(pi/2)
    int32_t plane_ref;                // float32 quartic: 1 = every plane is its own
                                      // reference plane (field_q32.hpp), 0 = groups of 8
    void* field;                      // [nk][H][W] or null (not written)
    uint64_t* bits_blk;               // [nk][ceil(H/8)][ceil(W/8)] or null: field >= C,
                                      // one word per 8x8 block (bit 8*row+col)
    double C;
    unsigned long long* stats;        // [3] (stats kernels only)
};
lsl_status launch_field(int dtype, const FieldArgs& a, bool stats, hipStream_t st);
// Block-major binary image (see FieldArgs::bits_blk) of a field.
lsl_status launch_bits_blk(int dtype, const void* field, int32_t nk, int32_t W, int32_t H,
                           double C, uint64_t* bits_blk, hipStream_t st);

// ------------------------------------------------------------- contours.hip
size_t contour_tmp_elems(int32_t nk, int32_t W, int32_t H);
// Marching squares on block-major binary images [nk][ceil(H/8)][ceil(W/8)].
// base (optional, device): running segment count added to this call's
// offsets and positions; the emit pass advances it by this call's total.
lsl_status launch_contours_count(const uint64_t* img, int32_t nk, int32_t W, int32_t H,
                                 int64_t* offsets, uint8_t* codes, unsigned long long* tmp,
                                 const unsigned long long* base, hipStream_t st);
lsl_status launch_contours_emit(const uint64_t* img, int32_t nk, int32_t W, int32_t H,
                                const unsigned long long* tmp, unsigned long long* base,
                                float* segs, int64_t capacity, hipStream_t st);
// Sub-pixel segments of nk planes (same cells and order as the emit pass;
// tmp, offsets from launch_contours_count with no base) and, if chain and
// rank are given, each segment's chain head and rank within its plane.
// scratch holds polyline_scratch_elems(total) words; rounds is
// 1 + ceil(log2(longest chain)).
lsl_status launch_polylines(const uint64_t* img, const void* field, int dtype, double C,
                            int32_t nk, int32_t W, int32_t H, const unsigned long long* tmp,
                            const int64_t* offsets, uint64_t total, int32_t rounds, float* segs,
                            uint32_t* scratch, int32_t* chain, int32_t* rank, hipStream_t st);
size_t polyline_scratch_elems(uint64_t total);
// Row-major bits [nk][H][ceil(W/32)] from block-major images.
lsl_status launch_bits_rows(const uint64_t* img, int32_t nk, int32_t W, int32_t H,
                            uint32_t* bits, hipStream_t st);

// ------------------------------------------------------------- backward.hip
struct BackArgs {
    const void* rec;
    const uint32_t* offsets;
    const uint32_t* ids;
    uint32_t n_binned, n_pairs;
    int32_t ntx, nty, tile, slab;
    int32_t group_s0;
    int32_t s_lo, s_hi;
    int32_t k0, nk;
    int32_t W, H;
    double x0, y0, dx, dy, z0, dz, R;
    int32_t strut_R;                  // 1: strut j's support is rec[j].pad, else R
    const uint32_t* emi;              // bucket entry -> emission index
    const void* grad;                 // [nk][H][W]
    void* partial;                    // [n_pairs][9] T, in emission order
    const double4* line;              // [n_binned]: u (x, y, z), L per strut (float64)
    int32_t plane_ref;                // 1: every plane its own reference (coarse plane pitch)
    int32_t wide;                     // float32: 1 = 16x16-pixel regions, 0 = 8x8
};
lsl_status launch_backward(int dtype, const BackArgs& a, hipStream_t st);

struct ReduceArgs {
    const void* partial;              // [n_pairs][9], emission order
    const uint32_t* active;           // [n_active] sorted positions
    uint32_t n_active;
    const uint32_t* eoff;             // [n_active + 1]
    const void* rec;
    const void* w;
    double R;
    int32_t strut_R;                  // 1: strut j's support is rec[j].pad, else R
    int32_t normalized;               // 1: partials in units of the support (float32 path)
    double* acc;                      // [n_binned][7]: dL/dw, dL/da (3), dL/db (3)
};
lsl_status launch_reduce(int dtype, const ReduceArgs& a, const SRange* ranges, int32_t sa,
                         int32_t s_lo, int32_t s_hi, uint32_t n_pairs, uint32_t n_binned,
                         hipStream_t st);

struct ScatterArgs {
    const double* acc;                // [n_binned][7]
    const uint32_t* perm;             // sorted position -> edge id
    int64_t n_binned, n_edges, n_nodes;
    const uint32_t* node_off;         // [n_nodes + 1]
    const uint32_t* node_inc;         // incidences 2p + end
    void* grad_weight;                // [n_edges] or null
    void* grad_nodes;                 // [n_nodes][3] or null
    int32_t accumulate;
};
lsl_status launch_scatter(int dtype, const ScatterArgs& a, hipStream_t st);
lsl_status launch_node_keys(const int2* ends, int64_t n_binned, uint32_t* keys,
                            uint32_t* vals, hipStream_t st);
lsl_status launch_node_offsets(const uint32_t* sorted_keys, size_t n, int64_t n_nodes,
                               uint32_t* node_off, hipStream_t st);

// ---------------------------------------------------------------- batch.hip
struct BatchArgs {
    FieldArgs f;
    const uint32_t* queue;            // items (s_rel, tile) in cost order
    uint32_t n_items;
    uint32_t* counter;                // device work counter (zeroed per launch)
};
lsl_status launch_queue_build(const FieldArgs& f, uint32_t* keys, uint32_t* vals,
                              uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n_items,
                              uint32_t* tmp, const uint32_t** queue_out, hipStream_t st);
// The caller zeroes a.counter before the launch.
lsl_status launch_persistent(int dtype, const BatchArgs& a, int n_blocks, hipStream_t st);
int persistent_blocks(int dtype, int slab);

// ---------------------------------------------------------------- support.hip
// Self-support metrics (Sec. 5.2, Eqs. 11-14) and dGamma/dv.
struct SupportArgs {
    const void* nodes;                // [n_nodes][3], lattice dtype
    const int32_t* edges;             // [n_edges][2]
    const void* weight;               // [n_edges]
    int64_t n_nodes, n_edges;
    double t[3];                      // unit printing direction
    double* part;                     // [support_part_elems(n_edges)]
    double* sums;                     // [5]: N, D, supported length, length, #supported
    int* err;                         // set to 1 on an edge index out of range
    void* grad;                       // [n_nodes][3] lattice dtype, or null
    double* te;                       // [n_edges][3] per-edge gradient terms
    uint32_t *k0, *v0, *k1, *v1;      // [2 n_edges] incidence sort
    uint32_t* tmp;                    // radix_tmp_elems(2 n_edges)
    uint32_t* off;                    // [n_nodes + 1]
};
size_t support_part_elems(int64_t n_edges);
lsl_status launch_support(int dtype, const SupportArgs& a, hipStream_t st);

// ---------------------------------------------------------------- density.hip
// Per-voxel density (Sec. 5, Eq. 9) and the soft voxel-density loss.
struct DensityArgs {
    int32_t nk, W, H;                 // field planes and plane size
    int32_t vx, vy, vz;               // voxel extents, clipped to the field
    int32_t nx, ny, nz;               // voxels per axis
    int32_t vpb, nbx;                 // voxel columns per block, blocks per voxel row
    uint32_t n_blocks;
};
lsl_status density_plan(int32_t nk, int32_t W, int32_t H, int32_t vx, int32_t vy, int32_t vz,
                        DensityArgs* a);
size_t density_voxels(const DensityArgs& a);
// doubles: residuals [voxels] + per-block partial losses [n_blocks]
size_t density_scratch_elems(const DensityArgs& a);
lsl_status launch_density(int dtype, const DensityArgs& a, const void* field, double C,
                          float* out, hipStream_t st);
lsl_status launch_density_loss(int dtype, const DensityArgs& a, const void* field, double C,
                               double tau, const float* target, float* soft, void* grad,
                               double* loss, double* scratch, hipStream_t st);
// Per-pixel soft-occupancy loss over n values; part holds occupancy_blocks(n)
// doubles.
uint32_t occupancy_blocks(size_t n);
lsl_status launch_occupancy_loss(int dtype, const void* field, const void* target, size_t n,
                                 double C, double tau, void* grad, double* loss, double* part,
                                 hipStream_t st);

}  // namespace lsl
