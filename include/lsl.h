/*
 * lsl.h -- C ABI of liblsl, an MI355X (gfx950) slicer for lattice structures
 * whose solid is a convolution surface with a compactly supported kernel
 * (Liu et al., "Memory-Efficient Modeling and Slicing of Large-Scale Adaptive
 * Lattice Structures").
 *
 * What is computed.  A lattice is a strut graph: nodes v_i in R^3 and edges
 * e_j = (v_s, v_e, r_j) (Sec. 3.1).  Its field at a point p is
 *
 *     g(p) = sum_j r_j * integral over e_j of f(p - x) d(arclength)   (Eq. 6)
 *     f(d) = (1 - |d|^2 / R^2)^2  for |d| < R, else 0                  (Eq. 5)
 *
 * and p lies inside the solid where g(p) >= C (the paper writes the implicit
 * function as F = -C + g; inside is where the skeleton's sum reaches the
 * iso-value).  Slices are planes z_k = z0 + (k + 1/2) dz (Sec. 4: the first
 * half a layer up, one layer apart); each plane is sampled at pixel centres
 * (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy), i < W, j < H, giving a field image,
 * a binary image (Sec. 4) and its marching-squares contours (Sec. 4).
 * Two kernel variants (per-strut supports, a compact Gaussian) are selected
 * in lsl_lattice; zero-initialised, it describes the paper's method.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers unless marked [host].  The caller owns every
 *    buffer it passes; the library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it in order.  Calls that must read a size back from
 *    the device synchronise that stream; this is stated per call.
 *  - Errors are returned, never thrown, and leave outputs unspecified.
 *    lsl_last_error() gives a message for the calling thread's last error.
 *  - dtype LSL_F32 computes in float32 (compensated sums of runs of terms),
 *    LSL_F64 in float64.  Field, weight and gradient arrays use the lattice's dtype.
 *  - Image layout: [slice][row j][column i], i fastest.
 *  - A handle may be used by one stream at a time.
 */
#ifndef LSL_H
#define LSL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lsl_status;
#define LSL_OK          0
#define LSL_EINVAL     (-1) /* bad argument or lattice (message says which)   */
#define LSL_ENOMEM     (-2) /* device allocation failed or budget exceeded    */
#define LSL_ECAPACITY  (-3) /* output buffer too small; required size given   */
#define LSL_EDEVICE    (-4) /* HIP runtime error (also from earlier work)     */
#define LSL_EINTERNAL  (-5) /* internal invariant failed                      */

#define LSL_F32 0
#define LSL_F64 1

/* The strut graph (Sec. 3.1).  [host] struct; arrays are device memory and are
 * only read during lattice_bin (they may be freed after it returns). */
typedef struct lsl_lattice {
    int64_t n_nodes;        /* >= 1                                              */
    int64_t n_edges;        /* >= 0                                              */
    int32_t dtype;          /* LSL_F32 or LSL_F64: element type of nodes, weight */
    const void* nodes;      /* [n_nodes][3] positions v_i, finite                */
    const int32_t* edges;   /* [n_edges][2] node indices (v_s, v_e), in range    */
    const void* weight;     /* [n_edges] r_j of Eq. (6), finite, >= 0;
                               0 marks an absent strut (never binned) unless
                               keep_zero_weight is set                          */
    double R;               /* kernel support of Eq. (5), finite, > 0            */
    double C;               /* iso-value, finite, > 0                            */
    /* Variants beyond the paper's single quartic kernel (zero-initialise for
     * the paper's method):                                                   */
    const void* support;    /* NULL: every strut's support is R.  Otherwise
                               [n_edges] per-strut supports R_j (lattice
                               dtype), finite, > 0; strut j then uses R_j in
                               its kernel and its reach (R is not used)        */
    int32_t kernel;         /* LSL_KERNEL_QUARTIC (Eq. (5)) or LSL_KERNEL_GAUSS:
                               exp(-d^2/2 sigma^2) - exp(-R^2/2 sigma^2) for
                               d < R, else 0 (the Gaussian the paper compares
                               with, shifted and cut at the same support)     */
    double sigma;           /* LSL_KERNEL_GAUSS only: width, finite, > 0, with
                               every support <= 12 sigma                       */
    int32_t keep_zero_weight; /* 0: a strut of weight 0 is absent (not binned;
                               slice_field_backward reports dL/dr_j = 0 for
                               it).  1: it is binned like the others -- its
                               terms are exact zeros, so the field is the same
                               -- and slice_field_backward returns the true
                               dL/dr_j = sum_p G(p) I_j(p) (Eq. 6 is linear in
                               r_j), which gradient steps on the weights need */
} lsl_lattice;

enum { LSL_KERNEL_QUARTIC = 0, LSL_KERNEL_GAUSS = 1 };

/* Pixel grid and slice planes.  [host] struct. */
typedef struct lsl_grid {
    double x0, y0;          /* origin: pixel (i,j) centre is                     */
    double dx, dy;          /*   (x0 + (i+1/2) dx, y0 + (j+1/2) dy); dx, dy > 0  */
    int32_t W, H;           /* pixels per row / rows, >= 2                       */
    double z0, dz;          /* plane k at z0 + (k+1/2) dz; dz > 0               */
    int32_t n_slices;       /* >= 1                                              */
} lsl_grid;

/* Binning choices.  [host] struct; a zero field takes the default. */
typedef struct lsl_bin_params {
    int32_t tile;           /* square xy tile edge in pixels: 8, 16, 32 or 64
                               (default 16)                                      */
    int32_t slab;           /* consecutive slices per z-slab, 1..16 (default 8)  */
    int64_t max_pairs;      /* most (slab, tile, strut) pairs binned at once;
                               more slabs than that are binned group by group
                               as slices are requested (default 2^30)            */
} lsl_bin_params;

/* Opaque handle: the prepared struts in edge-list order (ascending z of the
 * lower end, Sec. 4), their slab/tile ranges, the slab-group plan and the
 * bucket lists of the group binned last.  Owned by the library. */
typedef struct lattice_bins lattice_bins;

typedef struct lsl_bins_info {
    int64_t n_edges;        /* as given                                          */
    int64_t n_nodes;
    int64_t n_binned;       /* struts with w > 0, v_s != v_e, meeting the grid   */
    int64_t total_pairs;    /* (slab, tile, strut) pairs over all slabs          */
    int64_t max_group_pairs;
    int64_t device_bytes;   /* device memory the handle holds now                */
    int64_t peak_device_bytes;
    int32_t dtype, tile, slab;
    int32_t tiles_x, tiles_y, n_slabs, n_groups;
    int32_t current_group;  /* group whose bucket lists are resident, or -1      */
    double last_field_ms;   /* device time of the persistent field launches of
                               the last slice_batch call (HIP events around the
                               kernel on its stream); -1 if unavailable          */
    double last_group_bin_ms;   /* the same call's other stages, summed over its */
    double last_queue_ms;       /* slab groups: binning of groups not resident,  */
    double last_contour_ms;     /* work-queue build, binary image + contours     */
    int32_t plane_group;    /* planes that share one reference plane in the
                               float32 field kernel of the paper's kernel: 8
                               when 7 dz |d| <= R^2 / 10 (d the farthest pixel
                               of an 8x8 block from its centre, R the smallest
                               support), else 1; 1 for other kernels          */
    double last_backward_ms;    /* device time of the adjoint kernels of the last
                                   slice_field_backward call (HIP events around
                                   them on its stream, waited for here); -1 if
                                   none                                        */
} lsl_bins_info;

/* ---------------------------------------------------------------------------
 * lattice_bin -- prepare a lattice for slicing (Sec. 4).
 *
 * Builds the paper's edge list sorted by the z of each strut's lower end
 * (Sec. 4, the first of its two lists), the per-strut slab and tile ranges of
 * the swept sphere of radius R around the strut (Sec. 4; only struts within R
 * of p contribute, Sec. 3.2), and a plan that splits the slabs into groups
 * of at most max_pairs bucket entries.  The first group's bucket lists are
 * built at once; later groups are built when their slices are requested,
 * reusing the active struts of the previous group (the active list of
 * Eq. (8), kept up to date as the sweep of Sec. 4 moves up).
 *
 * Bin set (exact; evaluated in float64 in this operation order, no fused
 * multiply-add): for each strut with ends a, b and each axis with origin o,
 * step s, count n:  i0 = floor(((min(a,b) - R) - o) * (1/s) - 0.5),
 * i1 = ceil(((max(a,b) + R) - o) * (1/s) - 0.5), clamped to [0, n-1]
 * (strut dropped if empty).  Slab range [k0/slab, k1/slab], tile range
 * [i0/tile, i1/tile] x [j0/tile, j1/tile].  A bucket (slab, tile_y, tile_x)
 * lists the struts covering it in edge-list order.  With per-strut supports
 * (lattice.support) R is R_j in these formulas and the edge list is ordered
 * by (first slab, z of the lower end, id), which keeps each slab's window a
 * prefix of the list; with one R that is the same order.  (The lists are
 * built by a stable sort of (slab, tile row, 8-column segment) cells and a
 * per-cell count and fill; the bin set and its order are the above.)
 *
 * On success *out holds a new handle.  Synchronises `stream` while it runs
 * (to read back the plan); the first group's bucket lists may still be in
 * flight on `stream` when it returns.  Errors: LSL_EINVAL (bad argument, edge index out of range,
 * negative or non-finite weight, non-finite node used by an edge, support
 * not finite and > 0, unknown kernel, sigma not finite and > 0 or a support
 * above 12 sigma), LSL_ENOMEM, LSL_EDEVICE.
 * ------------------------------------------------------------------------- */
lsl_status lattice_bin(const lsl_lattice* lattice, const lsl_grid* grid,
                       const lsl_bin_params* params, lattice_bins** out,
                       void* stream);

/* Frees the handle (synchronises the device first).  Its device buffers go
 * to the library's device-memory cache, from which later handles of similar
 * sizes take them without hipMalloc; lsl_cache_trim returns them to the
 * device.  NULL is accepted. */
lsl_status lattice_bins_free(lattice_bins* bins);

/* Returns every cached device buffer to the device (hipFree, after
 * synchronising each device that holds some) and releases the cached
 * executable graphs of slice_batch (after their last launches complete).
 * *cached_bytes (host, nullable) receives the bytes the buffer cache held.
 * Setting LSL_NO_CACHE=1 in the environment before the first call disables
 * the buffer cache: buffers are then allocated and freed directly. */
lsl_status lsl_cache_trim(int64_t* cached_bytes);

/* slice_batch runs each slab group as three HIP graphs (work queue, field,
 * image + contours) through one cache of executable graphs per process,
 * shared by every handle: a call records its launches and updates a cached
 * executable graph of the same launch shape (Sec. 6.4: layers differ only
 * in how much work they carry), instantiating one only for a new shape or
 * a refused update.  Two entries per shape serve consecutive groups in
 * turn, at most 64 entries are kept.  Reports (host pointers, each
 * nullable) the graphs instantiated and updated since the process started
 * and the entries held now. */
lsl_status lsl_graph_cache_stats(int64_t* instantiated, int64_t* updated, int64_t* entries);

/* Sizes and memory use of a handle.  `out` is [host]. */
lsl_status lattice_bins_info(const lattice_bins* bins, lsl_bins_info* out);

/* Slab range and pair count of plan group g.  Outputs are [host]. */
lsl_status lattice_bins_group(const lattice_bins* bins, int32_t g,
                              int32_t* slab_first, int32_t* slab_last,
                              int64_t* pairs);

/* Builds group g's bucket lists (if not resident) and copies them out:
 * offsets [n_buckets + 1] int64 (bucket b = (slab - slab_first) * tiles_y *
 * tiles_x + tile_y * tiles_x + tile_x) and ids [pairs] int32 original edge
 * ids.  Either output may be NULL.  Stream-ordered; no synchronisation. */
lsl_status lattice_bins_export(lattice_bins* bins, int32_t g, int64_t* offsets,
                               int32_t* ids, void* stream);

/* The edge list: original ids of the binned struts in ascending (z of the
 * lower end, id) order (with per-strut supports: (first slab, z of the lower
 * end, id)), [n_binned] int32.  Stream-ordered. */
lsl_status lattice_bins_order(const lattice_bins* bins, int32_t* order,
                              void* stream);

/* ---------------------------------------------------------------------------
 * slice_field -- evaluate g (Eq. 6, closed form of Eq. 7 over arclength) at
 * every pixel centre of planes k0 .. k0+nk-1 (Sec. 4).
 *
 * field: [nk][H][W] of the lattice dtype (required).  bits: optional
 * [nk][H][ceil(W/32)] uint32, bit (i % 32) of word i/32 set where
 * field >= C (the binary image of Sec. 4).  Per pixel the sum runs over the
 * struts that can reach the pixel's 8x8 block in that plane, in edge-list
 * order; terms outside the support are exactly zero.  float32 sums add runs
 * of eight consecutive terms and compensate once per run (the Gaussian
 * variant and float64 compensate every term); the candidates of a block and
 * plane, hence the field's bits, do not depend on the tile, slab depth or
 * group split.  Builds missing groups
 * (stream-ordered, no synchronisation).  Errors: LSL_EINVAL (range outside
 * [0, n_slices)), LSL_ENOMEM, LSL_EDEVICE.
 * ------------------------------------------------------------------------- */
lsl_status slice_field(lattice_bins* bins, int32_t k0, int32_t nk, void* field,
                       uint32_t* bits, void* stream);

/* Candidate and useful (non-zero term) pixel-strut pair counts of the field
 * evaluation of planes k0 .. k0+nk-1 (the work slice_field does).  counts is
 * [host] int64[3]: candidates, useful, pixels.  Synchronises `stream`. */
lsl_status slice_field_stats(lattice_bins* bins, int32_t k0, int32_t nk,
                             int64_t* counts, void* stream);

/* ---------------------------------------------------------------------------
 * slice_contours -- marching squares on the binary images of nk planes
 * (Sec. 4: rough boundary curves from the binary image).
 *
 * field: [nk][H][W] lattice dtype, inside where field >= C.  Cell (i,j),
 * i < W-1, j < H-1, has corners (i,j), (i+1,j), (i+1,j+1), (i,j+1) with bits
 * b0..b3 and case b0 | b1<<1 | b2<<2 | b3<<3.  Segments join edge midpoints,
 * in grid units (pixel (i,j) at (i,j)), with the inside on the left; the two
 * saddle cases keep the inside corners apart.  Cells are emitted row by row
 * (j outer, i inner), a cell's segments in a fixed table order.
 *
 * segs: [capacity][4] float32 (x0, y0, x1, y1).  offsets: [nk + 1] int64,
 * offsets[k] = first segment of plane k, offsets[nk] = total.  case_codes:
 * optional [nk][H-1][W-1] uint8.  *total [host] receives the total.
 * Synchronises `stream` (reads the total).  If total > capacity no segment
 * is written, offsets and case codes are, and LSL_ECAPACITY is returned.
 * ------------------------------------------------------------------------- */
lsl_status slice_contours(const lattice_bins* bins, int32_t nk,
                          const void* field, float* segs, int64_t capacity,
                          int64_t* offsets, uint8_t* case_codes, int64_t* total,
                          void* stream);

/* ---------------------------------------------------------------------------
 * slice_polylines -- sub-pixel contours and their chaining into polylines
 * (the step after Sec. 4's boundary curves, toward toolpaths).
 *
 * Same planes, cells, segment count, order, offsets and capacity rules as
 * slice_contours (without case codes), except that each segment end sits
 * where g - C, interpolated linearly along its cell edge from the edge's
 * lower-(j, i) grid point P to the other point Q, vanishes:
 * P + t (Q - P), t = (C - g(P)) / (g(Q) - g(P)) (exactly one of P, Q is
 * inside).  Both segments meeting on an edge compute the point identically.
 *
 * chain, rank: optional (both or neither) [capacity] int32, per plane.  The
 * segment that follows s starts on the edge where s ends (the inside stays on
 * the left).  A chain starts at a segment with no predecessor (where a contour
 * enters from the grid border) or, for a closed loop, at its smallest segment
 * index.  chain[s] is that start's index within the plane, rank[s] the steps
 * from it.  Sorting a plane's segments by (chain, rank) gives its polylines.
 * Bitwise deterministic.  Synchronises `stream` (reads the offsets).
 * LSL_ECAPACITY as in slice_contours; LSL_EINVAL beyond 2^30 segments.
 * ------------------------------------------------------------------------- */
lsl_status slice_polylines(const lattice_bins* bins, int32_t nk, const void* field,
                           float* segs, int64_t capacity, int64_t* offsets,
                           int32_t* chain, int32_t* rank, int64_t* total,
                           void* stream);

/* ---------------------------------------------------------------------------
 * slice_density -- per-voxel material density of the sliced solid
 * (Sec. 5, Eq. 9), by Monte-Carlo integration of the inside test.
 *
 * The samples are the pixel centres of the slice planes (a stratified
 * sample on the slicing grid).  `field` is [nk][H][W] in the lattice dtype
 * (from slice_field or slice_batch); voxel (l, j, i) holds its planes
 * [l vz, (l+1) vz), rows [j vy, (j+1) vy) and columns [i vx, (i+1) vx),
 * clipped at the field's last plane, row and column, so a field that starts
 * at plane k0 gives voxels aligned to k0.  density: [nz][ny][nx] float32,
 * nz = ceil(nk / vz), ny = ceil(H / vy), nx = ceil(W / vx): the fraction of
 * the voxel's samples with g >= C, C rounded to the field's dtype, computed
 * as count / samples in float64 and rounded once to float32.  Bitwise
 * deterministic.  Stream-ordered, no allocation.  LSL_EINVAL on extents < 1.
 * ------------------------------------------------------------------------- */
lsl_status slice_density(const lattice_bins* bins, int32_t nk, const void* field,
                         int32_t vx, int32_t vy, int32_t vz, float* density,
                         void* stream);

/* ---------------------------------------------------------------------------
 * slice_density_loss -- a smooth voxel-density loss and its field gradient,
 * the forward half of a density-matching step by gradient descent on the
 * strut weights (Sec. 5.3 tunes the radii toward per-voxel targets).
 *
 * Voxels and field as in slice_density; the inside test is replaced by
 * s = sigmoid((g - C) / tau), tau > 0.  soft_density = per-voxel mean of s.
 * loss = sum_v (soft_density_v - target_v)^2 (one float64 on the device).
 * grad_field = dL/dg = 2 (soft_density_v - target_v) / n_v * s (1 - s) / tau
 * at every pixel ([nk][H][W], lattice dtype; n_v the voxel's sample count),
 * ready for slice_field_backward.  target: [nz][ny][nx] float32 on the
 * device.  soft_density ([nz][ny][nx] float32), grad_field and loss are each
 * optional (NULL: not written).  Sums run in a fixed order (bitwise
 * repeatable).  Stream-ordered; keeps a scratch buffer of one float64 per
 * voxel on the bins handle (it grows, synchronising `stream`, when a call
 * needs more).  LSL_EINVAL on extents < 1 or tau <= 0.
 * ------------------------------------------------------------------------- */
lsl_status slice_density_loss(const lattice_bins* bins, int32_t nk, const void* field,
                              int32_t vx, int32_t vy, int32_t vz, const float* target,
                              double tau, float* soft_density, void* grad_field,
                              double* loss, void* stream);

/* ---------------------------------------------------------------------------
 * slice_occupancy_loss -- a per-pixel soft-occupancy loss of a sliced field
 * and its gradient, the input of slice_field_backward (the radius tuning of
 * Sec. 5.3 needs a differentiable stand-in for the inside test).
 *
 * field, target: [nk][H][W] of the lattice dtype.  With s = sigmoid((g - C)
 * / tau), tau > 0: loss = sum over pixels of (s - target)^2 (one float64 on
 * the device), grad_field = dL/dg = 2 (s - target) s (1 - s) / tau
 * ([nk][H][W], lattice dtype).  Either output may be NULL.  One pass over
 * field and target; the sum has a fixed order (bitwise repeatable).
 * Stream-ordered; shares the scratch of slice_density_loss (it grows,
 * synchronising `stream`, when a call needs more).  LSL_EINVAL on nk < 1 or
 * tau <= 0.
 * ------------------------------------------------------------------------- */
lsl_status slice_occupancy_loss(const lattice_bins* bins, int32_t nk, const void* field,
                                const void* target, double tau, void* grad_field,
                                double* loss, void* stream);

/* ---------------------------------------------------------------------------
 * slice_occupancy_loss_static -- slice_occupancy_loss for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, kernels and results,
 * with the per-block partial sums in a static device array of the library
 * (8192 doubles, 64 KB per GPU, held until the process ends) instead of the
 * handle's growable scratch.  Allocates nothing and never synchronises.
 * Calls that overlap on one GPU share the array and race.  LSL_ECAPACITY if
 * a call would need more partial sums than the array holds (the loss uses at
 * most 8192 blocks, so none does); otherwise as slice_occupancy_loss.
 * ------------------------------------------------------------------------- */
lsl_status slice_occupancy_loss_static(const lattice_bins* bins, int32_t nk, const void* field,
                                       const void* target, double tau, void* grad_field,
                                       double* loss, void* stream);

/* ---------------------------------------------------------------------------
 * slice_field_backward -- gradient of a loss of the sliced field.
 *
 * Given grad_field = dL/dg at the pixels of planes k0 .. k0+nk-1
 * ([nk][H][W], lattice dtype), computes dL/dr_j = sum_p dL/dg(p) I_j(p) and
 * dL/dv for every node by the chain rule through Eq. (6)-(7); the
 * radius-tuning step of Sec. 5.3 adjusts exactly these weights.  Per-pixel
 * fields are recomputed, not stored.  Reductions run in a fixed order
 * (results are bitwise repeatable).
 *
 * grad_weight: [n_edges] lattice dtype (struts not binned get 0; zero-weight
 * struts are binned, and get sum_p dL/dg I_j, when the lattice sets
 * keep_zero_weight).
 * grad_nodes: [n_nodes][3] lattice dtype.  Either may be NULL.
 * accumulate: 0 overwrites the outputs, 1 adds to them.  Stream-ordered.
 * Covers the quartic kernel, with one support or per-strut supports (held
 * fixed); a handle of the Gaussian kernel gives LSL_EINVAL.
 * ------------------------------------------------------------------------- */
lsl_status slice_field_backward(lattice_bins* bins, int32_t k0, int32_t nk,
                                const void* grad_field, void* grad_weight,
                                void* grad_nodes, int32_t accumulate,
                                void* stream);

/* ---------------------------------------------------------------------------
 * slice_batch -- planes k0 .. k0+nk-1 end to end (field, binary image,
 * contours) with one persistent field launch per slab group: work items
 * (slab, tile) are taken from a device queue in descending cost order, so
 * planes with very different strut counts share the GPU evenly (Sec. 6.4:
 * slicing time follows the number of struts meeting a plane).  Each group's
 * launches run as three HIP graphs through the process's graph cache (see
 * lsl_graph_cache_stats): recorded per call, instantiated once per launch
 * shape and updated in place afterwards.
 *
 * field: optional [nk][H][W]; when NULL the field is not written (the
 * binary image is built in library scratch, one slab group at a time).
 * bits (optional), segs, offsets, *total: as in slice_field /
 * slice_contours.  Synchronises `stream` once at the end.  If the total
 * exceeds capacity, LSL_ECAPACITY is returned with offsets and *total
 * written and only the segments that fit below capacity stored.
 * ------------------------------------------------------------------------- */
lsl_status slice_batch(lattice_bins* bins, int32_t k0, int32_t nk, void* field,
                       uint32_t* bits, float* segs, int64_t capacity,
                       int64_t* offsets, int64_t* total, void* stream);

/* ---------------------------------------------------------------------------
 * slice_autotune -- choose tile and slab sizes by binning with each
 * candidate and timing the binning (to the end of its device work, the
 * faster of two runs, after one untimed warm-up binning), the binning of the
 * later slab groups in order (as one pass over all planes does it) and
 * slice_batch's field launch on three sampled windows of 64 planes of this
 * lattice and grid (the field time scaled to all planes).  params is [host] in/out:
 * nonzero fields are kept, zero fields are filled.  cache_path (optional,
 * [host] C string) is a JSON file of earlier choices keyed by problem shape
 * and kernel variant;
 * a hit skips the timing.  Synchronises `stream`.  The field values do not
 * depend on the choice (the same struts reach each pixel in the same order).
 * ------------------------------------------------------------------------- */
lsl_status slice_autotune(const lsl_lattice* lattice, const lsl_grid* grid,
                          lsl_bin_params* params, const char* cache_path,
                          void* stream);

/* ---------------------------------------------------------------------------
 * lattice_support -- self-support metrics of a lattice (Sec. 5.2) and the
 * gradient of Gamma for the vertex position optimisation.
 *
 * For edge j with unit direction u_j, length L_j and weight r_j (the radius
 * stored on the edge), theta_j = arccos |u_j . t| (Eq. 11), t = print_dir
 * normalised; the edge is self-supported when theta_j <= pi/4 (the paper's
 * alpha).  g(theta) is the paper's polynomial for alpha = pi/4 (Eq. 12):
 * sum_i a_i theta^i, a = (-0.02, -0.31, 1.44, -1.11, 0.58, -0.16), for
 * theta > pi/4, else 0.  Gamma = sum over unsupported edges of r L g /
 * sum over all edges of r L (Eq. 13); Psi = 100 * supported length / total
 * length (Eq. 14).  Zero-length edges add nothing.  Sums are float64 in a
 * fixed order (bitwise repeatable).
 *
 * print_dir: [host] double[3], finite, non-zero.  out: [host].  grad_nodes:
 * optional [n_nodes][3] lattice dtype, receives dGamma/dv (overwritten; the
 * step of g at pi/4 contributes no derivative).  R and C of the lattice are
 * not used.  Synchronises `stream`.  Errors: LSL_EINVAL (bad argument, edge
 * index out of range), LSL_ENOMEM, LSL_EDEVICE.
 * ------------------------------------------------------------------------- */
typedef struct lsl_support {
    double gamma;             /* Eq. (13)                                      */
    double psi;               /* Eq. (14), percent                             */
    double risky_area;        /* sum over unsupported edges of r L g(theta)     */
    double area;              /* sum over edges of r L                         */
    double supported_length;  /* sum over supported edges of L                 */
    double length;            /* sum over edges of L                           */
    int64_t n_supported;
} lsl_support;

lsl_status lattice_support(const lsl_lattice* lattice, const double* print_dir,
                           lsl_support* out, void* grad_nodes, void* stream);

/* Static text for a status code. */
const char* lsl_status_string(lsl_status s);
/* Message of the calling thread's last failed call ("" if none). */
const char* lsl_last_error(void);
/* Library version string. */
const char* lsl_version(void);

/* ---------------------------------------------------------------------------
 * Diagnostics: vector-ALU throughput of the GPU, the ceiling against which
 * the field and adjoint kernels are measured.  Not part of the slicing path.
 *
 * lsl_probe_valu runs one probe kernel on `stream` (16 blocks of 256 threads
 * per compute unit, `iters` iterations) and returns its duration in *ms and
 * the lane operations it issued in *lane_ops:
 *   mode 0  FP32 multiply-add with register operands (v_fmac_f32),
 *           16 independent chains per lane          -> 1 lane-op = 2 FLOP
 *   mode 1  FP32 multiply-add with scalar-register operands (v_fma_f32)
 *   mode 2  FP32 square root (v_sqrt_f32)
 *   mode 3  FP64 multiply-add
 *   mode 4  the field kernel's per-pair term and compensated add, from 64
 *           staged struts in LDS                   -> 1 lane-op = 1 pair
 *   mode 5  FP32 multiply-add, three-operand form with register operands
 *           (v_fma_f32)
 *   mode 6  FP32 clamp (v_med3_f32 with a negated bound)
 * The probe allocates and frees its own small device buffers and
 * synchronizes the stream.  LSL_EINVAL for a bad mode or iters < 1.
 * ------------------------------------------------------------------------- */
lsl_status lsl_probe_valu(int32_t mode, int32_t iters, float* ms, double* lane_ops,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LSL_H */
