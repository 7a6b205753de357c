// Allocation-free density (pv_density_static): build_cells + sort_cells +
// density for one periodic box, for callers that cannot allocate device
// memory.  The cell structure and every scratch buffer of the binning, the
// per-cell sorts and the work-queue sweep live in one static device array of
// fixed size, `scratch`; each device holds its own copy, whose address a
// context looks up once when it is created (static_scratch_init).  The
// kernels are the ones the allocating entry points launch: only the memory
// differs.
#include <algorithm>
#include <mutex>

#include "pvl_internal.h"

namespace pvl {

namespace {

constexpr int64_t kSN = PV_STATIC_MAX_N;        // particles, at most
constexpr int64_t kSC = PV_STATIC_MAX_CELLS;    // cells, at most
constexpr int kSChunk = 16384;                  // binning chunk (one count-matrix row)
constexpr int kSBlocks = (int)((kSN + kSChunk - 1) / kSChunk);
// split tail: cells x parts, at most (the tail sums hold one chunk per part)
constexpr int kSTailSlots = 512;
// persistent workgroups of a sweep, at most (each has its receiver lists)
constexpr int kSRlistWgs = 1280;

constexpr int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Byte offsets of the arrays in the static scratch (each 256-byte aligned),
// sized for kSN particles in kSC cells.
struct StaticLayout {
    int64_t box, box_hmax, bin_blocks, qcount, dx_all;
    int64_t cell_box, cell_start, cell_hmax, cell_dx, cell_m, big, binm, scan_tmp;
    int64_t cellid, slot, stage, xyzm, H, orig, sidx, tiles, items, partial, rlist;
    int64_t total;
};

constexpr StaticLayout static_layout()
{
    StaticLayout o{};
    int64_t p = 0;
    auto take = [&p](int64_t bytes) {
        const int64_t at = p;
        p = align256(p + bytes);
        return at;
    };
    o.box = take(sizeof(BoxDesc));
    o.box_hmax = take(4);
    o.bin_blocks = take(16 * kSBlocks);
    o.qcount = take(4 * kQueueCounters);
    o.dx_all = take(4);
    o.cell_box = take(4 * kSC);
    o.cell_start = take(4 * (kSC + 1));
    o.cell_hmax = take(4 * kSC);
    o.cell_dx = take(4 * kSC);
    o.cell_m = take(4 * kSC);
    o.big = take(4 * kCellLists * (kSC + 1));
    o.binm = take(4 * kSC * kSBlocks);
    o.scan_tmp = take(4 * scan_scratch_words(kSC));
    o.cellid = take(4 * kSN);
    o.slot = take(4 * kSN);
    o.stage = take(32 * kSN);
    o.xyzm = take(16 * kSN);
    o.H = take(4 * kSN);
    o.orig = take(4 * kSN);
    o.sidx = take(2 * 13 * kSN);
    o.tiles = take(4 * kTileArrays * (kSN / 16 + kSC + 1));
    o.items = take(8 * queue_capacity(kSN, kSC));
    o.partial = take(16 * (int64_t)kSTailSlots * kTailRecv);
    o.rlist = take(kRecvListBytes * kSRlistWgs);
    o.total = p;
    return o;
}

constexpr StaticLayout kLayout = static_layout();
static_assert(kLayout.total <= kStaticBytes, "the static scratch holds the largest input");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};

// The box descriptor and the binning chunks of one call, as kernel arguments.
struct StaticSetup {
    BoxDesc box;
    int4 blocks[kSBlocks];
    int nblocks;
};

__global__ void k_static_setup(StaticSetup s, BoxDesc *__restrict__ box, int4 *__restrict__ blocks)
{
    const int t = threadIdx.x;
    if (t == 0) *box = s.box;
    if (t < s.nblocks) blocks[t] = s.blocks[t];
}

}  // namespace

// The static scratch.  In host code this name is only a stand-in for the
// symbol, not a device address: kernels are given the address that
// static_scratch_init looks up on each device.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Device address of the static scratch on `device` (current): looked up once
// per device and kept.
hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = (unsigned char *)p;
    return hipSuccess;
}

unsigned char *static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

// Launches of one allocation-free density call (arguments already checked).
hipError_t launch_density_static(hipStream_t st, unsigned char *base, int64_t n,
                                 const float *pos, const float *h, const float *mass,
                                 const double box[3], const int grid[3], int algo, float *rho,
                                 float *wcount, float *drho_dh, int32_t *ncount, int *dflags,
                                 SweepTuning tune)
{
    const StaticLayout &o = kLayout;
    DevCells d;
    d.box = (BoxDesc *)(base + o.box);
    d.box_hmax = (uint32_t *)(base + o.box_hmax);
    d.bin_blocks = (int4 *)(base + o.bin_blocks);
    d.qcount = (int *)(base + o.qcount);
    d.dx_all = (uint32_t *)(base + o.dx_all);
    d.cell_box = (int32_t *)(base + o.cell_box);
    d.cell_start = (int32_t *)(base + o.cell_start);
    d.cell_hmax = (uint32_t *)(base + o.cell_hmax);
    d.cell_dx = (float *)(base + o.cell_dx);
    d.cell_m = (float *)(base + o.cell_m);
    d.big = (int32_t *)(base + o.big);
    d.binm = (int32_t *)(base + o.binm);
    d.scan_tmp = (int32_t *)(base + o.scan_tmp);
    d.cellid = (int32_t *)(base + o.cellid);
    d.slot = (int32_t *)(base + o.slot);
    d.stage = (float4 *)(base + o.stage);
    d.xyzm = (float4 *)(base + o.xyzm);
    d.H = (float *)(base + o.H);
    d.orig = (int32_t *)(base + o.orig);
    d.sidx = (uint16_t *)(base + o.sidx);
    d.tiles = (float *)(base + o.tiles);
    d.tslots = tile_slots(kSN, kSC);
    d.items = (int2 *)(base + o.items);
    d.partial = (float4 *)(base + o.partial);
    d.rlist = base + o.rlist;
    d.rlist_wgs = kSRlistWgs;

    // one box: cell and binning plan as pv_build_cells makes them
    StaticSetup s = {};
    BoxDesc &B = s.box;
    for (int a = 0; a < 3; ++a) {
        B.L[a] = (float)box[a];
        B.g[a] = grid[a];
        B.edge[a] = (float)(box[a] / grid[a]);
        B.inv_edge[a] = (float)(grid[a] / box[a]);
    }
    const int64_t ncell = (int64_t)grid[0] * grid[1] * grid[2];
    B.cell_off = 0;
    B.part_off = 0;
    B.n = (int)n;
    B.nblk = n > 0 ? (int)((n + kSChunk - 1) / kSChunk) : 1;
    B.moff = 0;
    s.nblocks = B.nblk;
    for (int j = 0; j < B.nblk; ++j) {
        const int lo = (int)std::min<int64_t>(n, (int64_t)j * kSChunk);
        const int hi = (int)std::min<int64_t>(n, (int64_t)(j + 1) * kSChunk);
        s.blocks[j] = make_int4(0, j, lo, hi);
    }
    BinPlan plan;
    plan.chunk = kSChunk;
    plan.mtot = ncell * B.nblk;
    plan.nblocks = B.nblk;
    hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(64), 0, st, s, d.box, d.bin_blocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_bin(st, d, plan, 1, n, ncell, pos, h, mass, dflags);
    if (e == hipSuccess && algo == PV_SORTED_PAIR) e = launch_sort13(st, d, n, ncell);
    if (e != hipSuccess) return e;
    // the persistent workgroups' receiver lists must fit their static share
    tune.queue_wgs_per_cu =
        std::max(1, std::min(tune.queue_wgs_per_cu, kSRlistWgs / std::max(1, tune.num_cu)));
    // the split tail's sums must fit their static share
    const int tc = tail_cells_of(tune, ncell);
    if (tune.tail_parts > 1) {
        const int cap = kSTailSlots / tune.tail_parts;
        if (tc <= 0) {
            tune.tail_parts = 1;
        } else {
            tune.tail_cells = std::min(tc, cap);
        }
    }
    return launch_sweep(st, d, n, ncell, algo, rho, wcount, drho_dh, ncount, dflags, nullptr,
                        tune);
}

}  // namespace pvl
