/*
 * pvl.h -- pseudo-Verlet (sorted cell-pair) SPH density loop on AMD gfx950.
 *
 * C ABI of libpvl.so.  Every entry point takes plain pointers and sizes; no C++
 * types or exceptions cross it.  Particle arrays are device pointers owned by
 * the caller.  Cell structures (pv_cells) and scratch memory are owned by the
 * library.  All calls are asynchronous on the context's HIP stream unless
 * stated otherwise.  A context is not thread-safe; use one per host thread.
 *
 * What is computed (Willis et al., "An Efficient SIMD Implementation of
 * Pseudo-Verlet Lists for Neighbour Interactions in Particle-Based Codes"):
 * the density loop of Fig. 1's caption -- each particle's density as a
 * kernel-weighted sum over every neighbour closer than its cut-off -- found
 * with the cell list of Section 2 (cells of edge >= cut-off) and the
 * pseudo-Verlet pruning of Section 2 / Listing 2 (project both cells on the
 * axis joining their centres, sort, and test only pairs whose projected
 * separation is below the receiver's cut-off), with the loop bounds of
 * Section 3.3 and the cache of Section 3.2.
 *
 * Conventions shared by every entry point:
 *   - h is the SPH smoothing length; the cut-off radius is H = 1.825742 h
 *     (cubic-spline support in 3D).  The paper's own "h" is this cut-off.
 *   - W(r, H) = 8 / (pi H^3) w(r/H) with the M4 cubic spline
 *     w(u) = 1 - 6u^2 + 6u^3 (u < 1/2), 2 (1-u)^3 (1/2 <= u < 1), 0 otherwise.
 *   - A pair is in range when r_ij < H_i (strict, as in Listings 1-2); the
 *     receiver's own cut-off decides (gather form).
 *   - Boxes are periodic with the minimum-image convention; positions may lie
 *     anywhere and are wrapped into [0, L).
 *   - Arithmetic is fp32.  Positions are stored relative to their cell's
 *     origin before any difference is taken (Section 3.2's shift-then-convert,
 *     with the cell origin in place of the pair centre).
 */
#ifndef PVL_H
#define PVL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pv_ctx pv_ctx;
typedef struct pv_cells pv_cells;

typedef enum {
    PV_OK = 0,
    PV_EINVAL = -1,     /* bad argument (NULL pointer, n < 0, box <= 0, ...)         */
    PV_ENOMEM = -2,     /* device allocation failed                                  */
    PV_EHIP = -3,       /* a HIP runtime call failed; pv_last_error has the text      */
    PV_EGRID = -4,      /* fewer than 3 cells on an axis, or a cell edge < max cut-off */
    PV_EOVERFLOW = -5,  /* a cell holds more particles than PV_MAX_CELL               */
    PV_ESTATE = -6      /* call out of order (e.g. density before sort_cells)         */
} pv_status;

typedef enum {
    PV_SORTED_PAIR = 0, /* pseudo-Verlet sweep over the 13 sorted axes (Section 2-3)  */
    PV_PLAIN_CELL = 1   /* plain 27-cell brute force (Listing 1), the comparator       */
} pv_algo;

/* Largest supported cell occupancy (particles in one cell). */
#define PV_MAX_CELL 8192
/* Largest supported number of cells per axis. */
#define PV_MAX_GRID 1024

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context.
 * device = -1 creates an argument-checking context that touches no device:
 * every entry point validates its arguments as usual and then returns
 * PV_ESTATE (useful on hosts without a GPU). */
pv_status pv_create(int device, void *hip_stream, pv_ctx **out);

/* Release the context and its scratch memory.  NULL is accepted. */
void pv_destroy(pv_ctx *ctx);

/* Change the stream later calls are issued on. */
pv_status pv_set_stream(pv_ctx *ctx, void *hip_stream);

/* Text of the last error on this context ("" if none).  Owned by the context. */
const char *pv_last_error(const pv_ctx *ctx);

/* Bin particles into cells (Section 2: the domain is cut into cells of edge
 * >= the cut-off and each cell's particles are stored together).
 *
 *   n         particles in the box, n >= 0
 *   pos       device, n x 3 fp32, array of structures (x0 y0 z0 x1 ...)
 *   h         device, n fp32 smoothing lengths (> 0)
 *   mass      device, n fp32 masses
 *   box       host, 3 doubles, box edge per axis (> 0)
 *   grid      host, 3 ints: cells per axis, or NULL / {0,0,0} for the finest
 *             legal grid floor(L / H_max) (this reads H_max back: one
 *             stream synchronisation)
 *   cells     in/out.  *cells == NULL: a new pv_cells is allocated.  Otherwise
 *             the given one is rebuilt in place, re-using its memory when it is
 *             large enough (no allocation then, so the call can be captured in a
 *             HIP graph together with sort_cells and density).
 *
 * Errors: PV_EINVAL, PV_EGRID (grid < 3 per axis, > PV_MAX_GRID, or edge below
 * the largest cut-off -- checked on the host in auto mode, on the device
 * otherwise and then reported by pv_check), PV_EOVERFLOW (reported by pv_check
 * or by the auto-grid read-back), PV_ENOMEM, PV_EHIP.
 * The input arrays are read during the call's kernels only. */
pv_status pv_build_cells(pv_ctx *ctx, int64_t n, const float *pos, const float *h,
                         const float *mass, const double box[3], const int grid[3],
                         pv_cells **cells);

/* Same for nbox independent periodic boxes in one structure.  Box b owns
 * particles [offsets[b], offsets[b+1]) of the concatenated device arrays.
 *   offsets   host, nbox + 1 int64, offsets[0] = 0, non-decreasing
 *   box       host, nbox x 3 doubles
 *   grid      host, nbox x 3 ints, or NULL for the finest legal grid per box
 *             (one stream synchronisation) */
pv_status pv_build_cells_batched(pv_ctx *ctx, int nbox, const int64_t *offsets,
                                 const float *pos, const float *h, const float *mass,
                                 const double *box, const int *grid, pv_cells **cells);

/* Sort every cell's particles by their projection on each of the 13 unique
 * cell-pair axes (Section 2: the dist and index arrays, pre-computed for the 13
 * directions left once the +-symmetry of the 26 neighbours is used).  Axis s
 * joins the centres of a cell and its neighbour at offset d_s, where d_s runs
 * over the offsets in {-1,0,1}^3 whose first non-zero component is positive. */
pv_status pv_sort_cells(pv_ctx *ctx, pv_cells *cells);

/* Density loop.  Outputs are device arrays of n fp32 (int32 for ncount) in the
 * caller's original particle order; any of them may be NULL.
 *   rho       sum_j m_j W(r_ij, H_i) over r_ij < H_i, j = i included
 *   wcount    sum_j W(r_ij, H_i), j = i included (units of 1 / volume)
 *   drho_dh   d rho_i / d h_i = -8/(pi H_i^3 h_i) sum_j m_j [3 w(u) + u w'(u)]
 *   ncount    #{ j != i : r_ij < H_i }
 * PV_SORTED_PAIR needs pv_sort_cells first (else PV_ESTATE). */
pv_status pv_density(pv_ctx *ctx, const pv_cells *cells, pv_algo algo, float *rho,
                     float *wcount, float *drho_dh, int32_t *ncount);

/* Adjoint of rho: given grad_rho = dL/drho (device, n fp32, original order),
 * write grad_pos = dL/dx (device, n x 3 fp32) and grad_h = dL/dh (device, n
 * fp32), either may be NULL:
 *   dL/dh_k = G_k drho_dh_k
 *   dL/dx_k = sum_{j != k} [G_k m_j W_r(r_kj, H_k) + G_j m_k W_r(r_kj, H_j)]
 *             (x_k - x_j) / r_kj,   W_r = 8 / (pi H^4) w'(r/H),
 * i.e. the pair set is the union r < max(H_k, H_j).  Uses the sorted lists
 * (pv_sort_cells first).  Masses are treated as constants. */
pv_status pv_density_backward(pv_ctx *ctx, const pv_cells *cells, const float *grad_rho,
                              float *grad_pos, float *grad_h);

/* Synchronise the context's stream and report device-detected errors raised
 * since the last check: PV_EOVERFLOW (a crowded cell), PV_EGRID (a cut-off
 * above the cell edge, or h <= 0), PV_ESTATE (particles moved by pv_drift
 * farther than the cells allow). */
pv_status pv_check(pv_ctx *ctx);

/* Describe a cell structure (host outputs, any may be NULL; box 0 for grid).
 * max_occupancy and hmax need a synchronisation. */
pv_status pv_cells_info(pv_ctx *ctx, const pv_cells *cells, int grid[3], int64_t *ncell,
                        int32_t *max_occupancy, float *hmax, int *nbox, int64_t *n);

/* Copy the cell-ordered layout to caller device buffers (tests and tools):
 * cell_start (ncell + 1 int32), order (n int32: original index of each
 * cell-ordered slot), sorted (13 x n uint16: in-cell rank lists per axis).
 * Any may be NULL. */
pv_status pv_cells_export(pv_ctx *ctx, const pv_cells *cells, int32_t *cell_start,
                          int32_t *order, uint16_t *sorted);

/* Candidate census of the last pv_density call made with census enabled
 * (host array of 3):
 *   counts[0]  pairs tested by the distance check under the method's exact
 *              per-receiver bounds: Section 3.3's bounds on the 26 neighbour
 *              cells and, in the receiver's own cell, the particles whose x
 *              lies within the receiver's cut-off (sorted), or every particle
 *              of the 27-cell stencil (plain), self excluded;
 *   counts[1]  pairs in range (self excluded);
 *   counts[2]  pair slots the production (tiled) sweep executes: 16 x 16 per
 *              source tile of each task of 16 receivers, including the slots
 *              of padding lanes and of pairs the tiles' coarser bounds admit.
 * pv_set_census(ctx, 1) enables counting: pv_density then runs scalar kernels
 * that test exactly the pairs of counts[0], followed by the tiled sweep
 * (whose outputs are the ones returned); slower. */
pv_status pv_set_census(pv_ctx *ctx, int enable);
pv_status pv_census(pv_ctx *ctx, int64_t counts[3]);

/* Tuning parameters of the sweep kernels (all results are identical up to
 * floating-point summation order; only speed changes).  Values persist on
 * the context; the sorted-pair density sweep, the adjoint sweep and the
 * plain cell-list sweep keep separate sets: add PV_PARAM_ADJOINT or
 * PV_PARAM_PLAIN to a parameter to address theirs (e.g. PV_PARAM_ADJOINT +
 * PV_PARAM_CHUNK).  pv_autotune picks them per workload.
 *   PV_PARAM_REACH_ORDER  1: order each direction's receivers by the reach of
 *                         their cut-off past the shared face before blocking
 *                         them into rows of 16 (tighter loop bounds, costs a
 *                         sort per cell); 0: use the key order.  Default 0.
 *                         The adjoint and plain sweeps ignore it.
 *   PV_PARAM_TASK_SORT    1: run row tasks longest first so the rows of a wave
 *                         finish together; 0: natural order.  Default 1.
 *   PV_PARAM_QUEUE_WGS    persistent workgroups per compute unit of the
 *                         work-queue sweeps (1..8).  Default 5, as many
 *                         as fit a compute unit (4 fit with
 *                         PV_PARAM_SYM_SELF set).
 *   PV_PARAM_CHUNK        receivers per work item, i.e. per workgroup's LDS
 *                         accumulator tile: a multiple of 16 in 32..256.
 *                         Cells with more particles are split into x-slabs
 *                         of this many receivers.  Default 256.
 *   PV_PARAM_TAIL_PARTS   the last cells of the work queue run as this many
 *                         work items each (1, 2 or 4), every item a share of
 *                         the cell's row tasks, so that the last items are
 *                         short and the workgroups finish together; the
 *                         shares are added in a fixed order afterwards
 *                         (1: no split).  Default 2.
 *   PV_PARAM_TAIL_CELLS   how many cells are split: the single-chunk cells
 *                         among the last this many cells of the grid
 *                         (1..2048), or 0: a quarter of the sweep's
 *                         persistent workgroups when there are at least
 *                         twice as many cells as workgroups, else none.
 *                         Default 0.
 *   PV_PARAM_GROUP        small cells per work item, at most (1..8): each
 *                         row of cells along z is cut into blocks of this
 *                         many cells, and consecutive single-chunk cells of a
 *                         block whose particles fit one chunk together run as
 *                         one work item (1: one cell per item).  0: automatic,
 *                         8 with at least 16 cells per persistent workgroup,
 *                         4 with at least 2, 2 with at least 1, else 1.
 *                         Results may differ in the last bits, since the
 *                         receivers' sums are taken in another order.  The
 *                         plain sweep always takes one cell per item.
 *                         Default 0.
 *   PV_PARAM_SYM_SELF     1: the receiver's own cell by the symmetric pair
 *                         update (Section 3.3's update of both particles of
 *                         a pair from one distance test): each unordered
 *                         pair of the cell is tested once and adds to both
 *                         particles, in items of whole cells (cells of at
 *                         most PV_PARAM_CHUNK particles); the adjoint sweep,
 *                         and the density sweep where masses are equal;
 *                         0: every receiver gathers from its own cell.
 *                         Default 0.
 *   PV_PARAM_XCD_RANGES   1: the work queue's single-chunk items are cut into
 *                         eight ranges of consecutive cells, one per
 *                         accelerator complex die (XCD: its own L2 cache;
 *                         workgroups go to the dies in turn by index), and a
 *                         workgroup takes items from its die's range first,
 *                         then from the next ranges, so that each L2 holds
 *                         the neighbourhood of one region; 0: one queue in
 *                         cell order for all.  The symmetric density form
 *                         (PV_PARAM_SYM_SELF) always takes the one queue.
 *                         Default 0.
 *   PV_PARAM_TAIL_SPLIT   how a split tail cell (PV_PARAM_TAIL_PARTS) is
 *                         shared: 0: every part takes every
 *                         PV_PARAM_TAIL_PARTS-th group of the cell's row
 *                         tasks, over all its receivers, and the shares are
 *                         added afterwards; 1: every part takes a range of
 *                         the cell's receivers (whole tiles of 16) and
 *                         writes their outputs itself, doing the set-up for
 *                         its receivers alone.  Default 0.
 * Out-of-range values return PV_EINVAL and leave the setting unchanged. */
typedef enum {
    PV_PARAM_REACH_ORDER = 1,
    PV_PARAM_TASK_SORT = 2,
    PV_PARAM_QUEUE_WGS = 3,
    PV_PARAM_CHUNK = 4,
    PV_PARAM_TAIL_PARTS = 5,
    PV_PARAM_TAIL_CELLS = 6,
    PV_PARAM_GROUP = 7,
    PV_PARAM_SYM_SELF = 8,
    PV_PARAM_XCD_RANGES = 9,
    PV_PARAM_TAIL_SPLIT = 10,
    PV_PARAM_ADJOINT = 16,
    PV_PARAM_PLAIN = 32
} pv_param;
pv_status pv_set_param(pv_ctx *ctx, int param, int value);
pv_status pv_get_param(pv_ctx *ctx, int param, int *value);

/* Kernel timing.  With enable != 0 the context records a pair of HIP events
 * on its stream right before and after every launch of the persistent
 * sweep kernel (the work-queue kernel of pv_density, pv_density_backward and
 * pv_lj, without the queue set-up and the tail combine before and after
 * it), in a ring of the last PV_KTIME_RING launches; nothing is recorded
 * while the stream is being captured into a graph.  Enabling (again) or
 * disabling clears the ring; the first enable creates the events.
 * pv_kernel_times synchronises the stream and writes to ms (host, *count
 * floats) the durations in milliseconds of the most recent launches, at
 * most *count of them, oldest first, and sets *count to how many it wrote.
 * For measurement (a bench's per-kernel rate); the events add a few
 * microseconds per launch.  Errors: PV_EINVAL, PV_ESTATE (argument-checking
 * context), PV_EHIP. */
#define PV_KTIME_RING 64
pv_status pv_set_kernel_timing(pv_ctx *ctx, int enable);
pv_status pv_kernel_times(pv_ctx *ctx, float *ms, int *count);

/* Autotuner.  Times the sorted-pair density sweep (PV_TUNE_DENSITY), the
 * adjoint sweep (PV_TUNE_ADJOINT, for the upstream gradient grad_rho, device,
 * n floats in original order) or the plain cell-list sweep (PV_TUNE_PLAIN)
 * on `cells` for every combination of the
 * parameters above (chunk 64/128/256, 1..8 workgroups per compute unit, task
 * order, receiver order), then the tail split (2 or 4 parts of the last 256,
 * 512 or 1024 cells, by task groups or by receivers) and then the
 * small-cell groups (1, 2, 4 or 8 cells per
 * item; not for the plain sweep) on top of the best, `reps` timed runs each
 * after one warm-up, and keeps the fastest on the context.  times_ms (host, may be NULL) receives the mean
 * time of the setting in place before the call and of the chosen one.  The
 * kernels write into temporary device buffers that the call allocates and
 * frees; the call synchronises the context's stream and must not be
 * captured.  Errors: PV_ESTATE if the cells are not sorted (density and
 * adjoint). */
typedef enum { PV_TUNE_DENSITY = 0, PV_TUNE_ADJOINT = 1, PV_TUNE_PLAIN = 2 } pv_tune_target;
pv_status pv_autotune(pv_ctx *ctx, const pv_cells *cells, int target, const float *grad_rho,
                      int reps, float times_ms[2]);

/* Grid autotuner.  The finest legal grid (floor(L / largest cut-off) per
 * axis) minimises the cell volume but not always the time: with few particles
 * per cell the 16-wide tiles run mostly empty.  Times a step (build with an
 * explicit grid + sort + sorted-pair density, `reps` runs after one warm-up)
 * for every box's finest grid scaled by 1, 0.85, 0.7, 0.6, 0.5, 0.42, 0.35 and
 * 0.3 (at least 3 cells per axis), stopping at the first grid with a cell above
 * PV_MAX_CELL or after two slower grids in a row, and writes the fastest to
 * grid_out (host, 3 * nbox ints) for the caller's later builds.  Arguments as
 * for pv_build_cells_batched.  times_ms (host, may be NULL): the step time at
 * the finest grid and at the chosen one.  Allocates temporary device memory,
 * synchronises, must not be captured. */
pv_status pv_autotune_grid(pv_ctx *ctx, int nbox, const int64_t *offsets, const float *pos,
                           const float *h, const float *mass, const double *box, int reps,
                           int *grid_out, float times_ms[2]);

/* Lennard-Jones forces and energies over the same neighbour sets (the
 * method serves molecular dynamics as well as SPH): for every pair with
 * r_ij < H_i (the receiver's cut-off; build the cells with h = r_c / gamma for
 * one cut-off r_c),
 *   force_i  = sum_j (24 eps / r^2) [2 (sigma/r)^12 - (sigma/r)^6] (x_i - x_j)
 *   energy_i = 1/2 sum_j 4 eps [(sigma/r)^12 - (sigma/r)^6]   (unshifted)
 * force: device n x 3, energy: device n, input order; either may be NULL.
 * Sorted-pair sweep with the density's tuning parameters; coincident
 * particles are skipped.  Requires pv_sort_cells. */
pv_status pv_lj(pv_ctx *ctx, const pv_cells *cells, float eps, float sigma, float *force,
                float *energy);

/* Move the particles of sorted cells without rebuilding them (Section 2: the
 * sorted lists can be reused over several time steps when every projected
 * bound is widened by the particles' displacement).  disp: device, n x 3, input
 * order, added to the stored positions (the caller's pos arrays are not
 * touched).  Each cell accumulates a bound on its particles' displacement since
 * the build; later pv_density / pv_density_backward calls widen their bounds by
 * the bounds of the two cells of each pair, so the results are those of the
 * moved positions.  The cells stay usable while largest cut-off + the two
 * displacement bounds fit the cell edge; past that the sweeps flag the error
 * word and pv_check returns PV_ESTATE (rebuild with pv_build_cells).  After a
 * drift, pv_sort_cells is refused (PV_ESTATE): rebuild instead. */
pv_status pv_drift(pv_ctx *ctx, pv_cells *cells, const float *disp);

/* Smoothing lengths from the density (the h-iteration around the density
 * loop of an SPH code; not part of the paper's method).  Solves, for every
 * particle, rho_i(h_i) h_i^3 = m_i eta^3 with eta^3 = 3 ngb / (4 pi gamma^3),
 * rho_i taken with the particle's own cut-off gamma h_i; with equal masses this
 * is the weighted neighbour number (4 pi / 3) H_i^3 wcount_i = ngb.  Each
 * iteration builds the cells (auto grid), sorts them, runs the sorted-pair
 * density for rho and drho_dh, and takes one Newton step per particle (steps
 * limited to a factor 1.5).  The boxes are given as for
 * pv_build_cells_batched (offsets host, nbox + 1; box host, 3 * nbox).
 *   pos, mass  device, input order (pos n x 3)
 *   h          device, n: the initial guess on entry, on return the last
 *              evaluated h (the one whose residual is reported)
 *   tol        stop when max_i |rho_i h_i^3 - m_i eta^3| / (m_i eta^3) <= tol
 *   iters      host, may be NULL: density evaluations made
 *   resid      host, may be NULL: that largest relative residual
 * Returns PV_OK when the iterations ran (compare *resid with tol to see
 * whether it converged within max_iter), or the error of a build (PV_EGRID when
 * a cut-off outgrows a third of the box, PV_EOVERFLOW for a crowded cell).
 * Synchronises every iteration; not for graph capture.  Its working set (a
 * cell structure and 3 n floats) stays on the context for the next call and
 * grows when a call needs more; pv_destroy frees it. */
pv_status pv_solve_h(pv_ctx *ctx, int nbox, const int64_t *offsets, const float *pos,
                     const float *mass, float *h, const double *box, float ngb, float tol,
                     int max_iter, int *iters, float *resid);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * density of one periodic box -- pv_build_cells with an explicit grid,
 * pv_sort_cells (sorted-pair only) and pv_density -- in one call that
 * allocates nothing and does not synchronise.  The cell structure and all
 * scratch memory of the binning, the per-cell sorts and the work-queue sweep
 * live in one static device array of 30 MiB, which every GPU the library runs
 * on holds until the process ends; a context looks up its device's copy when
 * it is created.  Inputs and outputs are the caller's, as for pv_build_cells
 * and pv_density:
 *   n          0 <= n <= PV_STATIC_MAX_N
 *   pos, h, mass  device, input order (pos n x 3)
 *   box        host, 3 doubles (> 0)
 *   grid       host, 3 ints, required: 3..PV_MAX_GRID cells per axis and at
 *              most PV_STATIC_MAX_CELLS cells in all
 *   algo, rho, wcount, drho_dh, ncount   as for pv_density
 * Results are those of pv_build_cells (same grid) + pv_sort_cells +
 * pv_density up to floating-point summation order (the split of the work
 * queue's last cells is limited to 512 cell parts here).  Errors:
 * PV_EINVAL (NULL pointer, n or the cell count above the limits, no grid),
 * PV_EGRID (fewer than 3 or more than PV_MAX_GRID cells per axis), PV_EHIP;
 * a cut-off above the cell edge or a crowded cell is detected on the device
 * and reported by pv_check, as for pv_build_cells.  Every call on one GPU uses
 * that GPU's one array and leaves its contents behind: calls that overlap on
 * one GPU (other contexts, streams or host threads on the same device) race,
 * and the caller must serialise them. */
#define PV_STATIC_MAX_N 131072
#define PV_STATIC_MAX_CELLS 32768
pv_status pv_density_static(pv_ctx *ctx, int64_t n, const float *pos, const float *h,
                            const float *mass, const double box[3], const int grid[3],
                            pv_algo algo, float *rho, float *wcount, float *drho_dh,
                            int32_t *ncount);

/* Release a cell structure.  NULL is accepted. */
pv_status pv_free_cells(pv_ctx *ctx, pv_cells *cells);

#ifdef __cplusplus
}
#endif
#endif /* PVL_H */
