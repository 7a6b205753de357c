// Internal declarations shared by the libpvl translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pvl.h"

namespace pvl {

// Cut-off over smoothing length of the cubic spline in 3D (H = GAMMA h).
constexpr float kGamma = 1.825742f;
constexpr float kPi = 3.14159265358979f;
// Threads per workgroup of the per-cell kernels.
constexpr int kBlock = 256;
// Device error bits.
constexpr int kErrOverflow = 1;
constexpr int kErrGrid = 2;
constexpr int kErrDrift = 4;   // particles moved farther than the cells allow

// One periodic box of a (possibly batched) cell structure, as the kernels see it.
struct BoxDesc {
    float L[3];         // box edge per axis
    float edge[3];      // cell edge L / g (fp32)
    float inv_edge[3];  // g / L
    int g[3];           // cells per axis
    int cell_off;       // first global cell of this box
    int part_off;       // first particle of this box (input and cell order)
    int n;              // particles in the box
    int nblk;           // binning chunks of the box (rows of its count matrix)
    int moff;           // first entry of the box's count matrix
    int pad[3];
};

// The 13 canonical cell offsets: those d in {-1,0,1}^3 \ 0 whose first
// non-zero component is positive.  A neighbour at offset d uses axis s with
// d_s = +d or d_s = -d.
__host__ __device__ inline void dir_offset(int s, int d[3])
{
    // s = 0..8: x = +1, (y, z) in {-1,0,1}^2; s = 9..11: x = 0, y = +1, z in {-1,0,1};
    // s = 12: (0, 0, 1)
    if (s < 9) { d[0] = 1; d[1] = s / 3 - 1; d[2] = s % 3 - 1; }
    else if (s < 12) { d[0] = 0; d[1] = 1; d[2] = s - 10; }
    else { d[0] = 0; d[1] = 0; d[2] = 1; }
}

// Map an offset d != 0 to (axis s, sign): d = sign * d_s.
__host__ __device__ inline int dir_canon(int dx, int dy, int dz, int *sign)
{
    int sx = dx, sy = dy, sz = dz;
    int sg = 1;
    if (dx < 0 || (dx == 0 && (dy < 0 || (dy == 0 && dz < 0)))) {
        sx = -dx; sy = -dy; sz = -dz; sg = -1;
    }
    *sign = sg;
    if (sx == 1) return (sy + 1) * 3 + (sz + 1);
    if (sy == 1) return 10 + sz;
    return 12;
}

// Unit axis of direction s: d_s / |d_s|.
__host__ __device__ inline void dir_axis(int s, float e[3])
{
    int d[3];
    dir_offset(s, d);
    int nz = (d[0] != 0) + (d[1] != 0) + (d[2] != 0);
    float inv = nz == 1 ? 1.0f : (nz == 2 ? 0.70710678118654752f : 0.57735026918962576f);
    e[0] = d[0] * inv; e[1] = d[1] * inv; e[2] = d[2] * inv;
}

// Device-side buffers of one cell structure.
struct DevCells {
    BoxDesc *box = nullptr;       // nbox
    int32_t *cell_box = nullptr;  // ncell: owning box
    int32_t *cell_start = nullptr;// ncell + 1: first slot (global, cell order)
    uint32_t *cell_hmax = nullptr;// ncell: max cut-off in the cell (fp32 bits)
    int32_t *cellid = nullptr;    // n: global cell of each input particle
    int32_t *slot = nullptr;      // n: arrival rank of the particle within its cell
    float4 *stage = nullptr;      // 2n: per particle (x, y, z, H) wrapped, (m, index bits, -, -)
    float4 *xyzm = nullptr;       // n: cell-relative position and mass
    float *H = nullptr;           // n: cut-off radius
    int32_t *orig = nullptr;      // n: original index
    uint16_t *sidx = nullptr;     // 13 x n: in-cell rank lists, ascending key
    float *gcell = nullptr;       // n: upstream gradient in cell order (adjoint)
    int2 *items = nullptr;        // work queue of (cell, receiver chunk)
    float4 *partial = nullptr;    // per-part sums of the split tail cells
    int *qcount = nullptr;        // kQueueCounters: large-cell chunks, cells, head, tail cells
    uint32_t *box_hmax = nullptr; // nbox: max cut-off per box (fp32 bits)
    int32_t *scan_tmp = nullptr;  // scan_scratch_words(matrix entries): tile sums / offsets
    int32_t *binm = nullptr;      // binning count matrix (chunks x cells per box)
    int32_t *big = nullptr;       // kCellLists lists of ncell + 1 (see cell_list)
                                  // particles (written by the cell finish, any order)
    // Tile summaries of the sorted lists, written by the per-cell sorts: for
    // axis s and tile slot t = cell_start[c] / 16 + c + j of tile j of cell c,
    //   tiles[kTileTS(s)] key of position 16 j        (first of tile j from the start)
    //   tiles[kTileTE(s)] key of position na-1-16 j   (first of tile j from the end)
    // and for the x axis (the cell order) the last key and the largest H of
    // each tile.
    float *tiles = nullptr;       // kTileArrays x tslots
    // the queue sweeps' per-workgroup receiver lists (kRecvListBytes per
    // persistent workgroup, for rlist_wgs of them): kept in memory rather
    // than LDS so that five density workgroups fit a compute unit
    uint8_t *rlist = nullptr;
    int64_t rlist_wgs = 0;
    int64_t tslots = 0;
    float *cell_m = nullptr;      // ncell: the mass shared by all particles of the cell,
                                  // NaN if they differ, +inf if the cell is empty
    float *cell_dx = nullptr;     // ncell: accumulated largest displacement since the build
    uint32_t *dx_all = nullptr;   // largest cell_dx of the structure (fp32 bits)
    int4 *bin_blocks = nullptr;   // binning chunks: (box, chunk in box, first, end particle)
};

// Chunking of the binning count sort (see plan_binning).
struct BinPlan {
    int chunk = 16384;     // particles per chunk
    int64_t mtot = 0;      // entries of the count matrices
    int64_t nblocks = 0;   // chunks (workgroups of the counting kernel)
};

// Largest cell sorted with one particle per thread; larger cells are listed
// and sorted one axis per workgroup.
constexpr int kSortSmallMax = 512;

// Largest cell of the large-cell sort's smaller LDS class.
constexpr int kSortLargeMax = 4096;

// Cell lists made during a build (by the binning's column pass), each a count
// followed by cell indices with room for every cell: the cells above 256
// particles, then of those the cells of 257..kSortSmallMax, of
// kSortSmallMax+1..kSortLargeMax and larger ones up to PV_MAX_CELL.
// The kernels that take a list run a fixed grid of at most kListWgs
// workgroups over it.
constexpr int kListLarge = 0, kListMid = 1, kListBig = 2, kListHuge = 3, kCellLists = 4;
constexpr int64_t kListWgs = 1024;
__host__ __device__ inline int32_t *cell_list(int32_t *lists, int64_t ncell, int k)
{
    return lists + k * (ncell + 1);
}

// Mean cell occupancy from which the per-cell kernels fold their rare size
// classes into their neighbours' launches.
constexpr int64_t kDenseCells = 128;

// Tile-summary arrays (see DevCells::tiles).
constexpr int kTileArrays = 2 * 13 + 2;
constexpr int kTileAxisX = 4;   // d = (1, 0, 0): the sorted list is the cell order
__host__ __device__ inline int64_t tile_slot(int32_t cell_start, int64_t cell, int j)
{
    return (int64_t)(cell_start >> 4) + cell + j;
}
__host__ __device__ inline int64_t tile_slots(int64_t n, int64_t ncell) { return n / 16 + ncell + 1; }
__host__ __device__ inline int64_t kTileTS(int s) { return s; }
__host__ __device__ inline int64_t kTileTE(int s) { return 13 + s; }
constexpr int64_t kTileTLX = 26;   // x axis: key of the tile's last position
constexpr int64_t kTileBHX = 27;   // x axis: largest H of the tile

// Launch wrappers (each lives next to its kernels).
hipError_t launch_box_hmax(hipStream_t st, const DevCells &c, int nbox, int64_t n,
                           const float *h);
// Fill BoxDesc::nblk / moff of every box (whose g, n and part_off are set)
// and the chunk table.
BinPlan plan_binning(std::vector<BoxDesc> &boxes, std::vector<int4> &blocks);
hipError_t launch_bin(hipStream_t st, const DevCells &c, const BinPlan &plan, int nbox, int64_t n,
                      int64_t ncell, const float *pos, const float *h, const float *mass,
                      int *dflags);
hipError_t launch_sort13(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell);
hipError_t launch_zero(hipStream_t st, void *p, int64_t words);
// Cells per tile of the cell-count scan, and the words of scratch the scan
// needs for ncell cells (tile sums and offsets).
constexpr int kScanTile = 8192;
constexpr int64_t scan_scratch_words(int64_t ncell) { return ncell / kScanTile + 2; }
// Sweep tuning (see pv_param).
struct SweepTuning {
    int reach_order = 0;
    int task_sort = 1;
    int queue_wgs_per_cu = 4;   // persistent workgroups per compute unit (1..kQueueWgsMax)
    int chunk = 256;            // receivers per work item (multiple of 16, 32..256)
    int tail_parts = 2;         // the queue's last cells run as this many items (1, 2, 4)
    int tail_cells = 0;         // how many cells (0: automatic)
    int group = 0;              // small cells per work item, at most (1..8; 0: automatic)
    int sym_self = 0;           // own cells by the symmetric pair update
    int xcd_ranges = 0;         // each XCD first takes its own eighth of the queue
    int tail_split = 0;         // tail parts: 0 share the task groups, 1 the receivers
    int num_cu = 256;           // compute units of the device
    // events recorded on the launch stream right before and after the
    // persistent sweep kernel (kernel timing; both null: none)
    hipEvent_t kt_start = nullptr, kt_stop = nullptr;
};

// Small cells per work item of the sweeps, at most.
constexpr int kGroupMax = 8;

// Tail split of the work queue: at most kTailMaxCells cells, kTailMaxParts
// parts each, kTailRecv receivers per cell (the largest chunk).
constexpr int kTailMaxCells = 2048;
constexpr int kTailMaxParts = 4;
constexpr int kTailRecv = 256;
// Compacted receiver lists of one work item: a byte per receiver of the
// largest chunk, per neighbour direction.
constexpr int64_t kRecvListBytes = 26 * kTailRecv;
// Persistent workgroups per compute unit of the queue sweeps, at most.
constexpr int kQueueWgsMax = 8;

// Smallest receivers per work item (sizes the work queue).
constexpr int kChunkMin = 32;
// Entries of the work queue for n particles in ncell cells: the items, then
// a tail region of kTailMaxCells entries.
constexpr int64_t queue_main(int64_t n, int64_t ncell) { return ncell + n / kChunkMin + 1; }
constexpr int64_t queue_capacity(int64_t n, int64_t ncell)
{
    return queue_main(n, ncell) + kTailMaxCells;
}
// Persistent workgroups of a queue sweep, and the cells of its split tail.
inline SweepTuning tuning_with_wgs(int wgs)
{
    SweepTuning t;
    t.queue_wgs_per_cu = wgs;
    return t;
}
int64_t queue_grid(const SweepTuning &tune, int64_t ncell);
int tail_cells_of(const SweepTuning &tune, int64_t ncell);
// Work-queue counters: large-cell chunks, single-chunk cells, the head of the
// dynamic queue, the split tail cells, then (XCD ranges) the heads of the
// large-cell chunks, of the tail items and of the kXcds ranges of the
// single-chunk items.
constexpr int kXcds = 8;   // accelerator complex dies of the device
constexpr int kQueueCounters = 6 + kXcds;

hipError_t launch_sweep(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell, int algo,
                        float *rho, float *wcount, float *drho_dh, int32_t *ncount,
                        int *dflags, unsigned long long *census, const SweepTuning &tune);
// slots (may be NULL): adds the pair slots the sweep executes (16 x 16 per
// source tile of each row task)
hipError_t launch_sweep_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                              float *rho, float *wcount, float *drho_dh, int32_t *ncount,
                              int *dflags, const SweepTuning &tune, bool plain,
                              unsigned long long *slots = nullptr);
hipError_t launch_lj_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                           float eps, float sigma, float *force, float *energy, int *dflags,
                           const SweepTuning &tune);
hipError_t launch_backward_tiled(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                                 float *grad_pos, float *grad_h, int *dflags,
                                 const SweepTuning &tune);
hipError_t launch_backward(hipStream_t st, const DevCells &c, int64_t n, int64_t ncell,
                           const float *grad_rho, float *grad_pos, float *grad_h,
                           int *dflags, const SweepTuning &tune);

// Allocation-free density (pv_density_static): the static scratch of
// kStaticBytes per device, its address looked up once per device (with the
// device current) and kept, and the launches of one call.
constexpr int64_t kStaticBytes = 30ll << 20;
hipError_t static_scratch_init(int device);
unsigned char *static_scratch(int device);
hipError_t launch_density_static(hipStream_t st, unsigned char *base, int64_t n,
                                 const float *pos, const float *h, const float *mass,
                                 const double box[3], const int grid[3], int algo, float *rho,
                                 float *wcount, float *drho_dh, int32_t *ncount, int *dflags,
                                 SweepTuning tune);

hipError_t launch_drift(hipStream_t st, const DevCells &c, int64_t ncell, const float *disp);
hipError_t launch_h_newton(hipStream_t st, int64_t n, const float *rho, const float *drho_dh,
                           const float *mass, const float *h, float eta3, float *h_next,
                           uint32_t *resid);
hipError_t launch_copy_f32(hipStream_t st, int64_t n, const float *src, float *dst);

}  // namespace pvl
