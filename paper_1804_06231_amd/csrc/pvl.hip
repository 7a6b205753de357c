// Host side of the C ABI declared in include/pvl.h: argument checks, grid
// choice, memory of the cell structures, kernel launches on the context's
// stream, error reporting.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "pvl_internal.h"

using pvl::BoxDesc;
using pvl::DevCells;

struct pv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int *dflags = nullptr;                  // [0] sticky error bits, [1] max occupancy
    unsigned long long *dcensus = nullptr;  // [0] pairs tested, [1] pairs in range,
                                            // [2] pair slots of the tiled sweep
    int census_on = 0;
    int *hpinned = nullptr;                 // pinned read-back area (64 bytes)
    // per sweep; five persistent workgroups per compute unit, as many as fit
    pvl::SweepTuning tune = pvl::tuning_with_wgs(5);        // density and LJ sweeps
    pvl::SweepTuning tune_adj = pvl::tuning_with_wgs(5);    // adjoint sweep
    pvl::SweepTuning tune_plain = pvl::tuning_with_wgs(5);  // plain cell-list sweep
    // pv_solve_h's working set, kept for the next call: its cells, and rho,
    // drho_dh, the next h (3 x hbuf_n floats) and the residual word
    pv_cells *hcells = nullptr;
    float *hbuf = nullptr;
    int64_t hbuf_n = 0;
    uint32_t *hres = nullptr;
    // kernel timing (pv_set_kernel_timing): a ring of event pairs, one pair
    // per launch of the persistent sweep kernel
    int kt_on = 0;
    std::vector<hipEvent_t> kt_ev;   // 2 * PV_KTIME_RING: start, stop, start, ...
    int kt_next = 0, kt_count = 0;
};

struct pv_cells {
    int nbox = 0;
    int64_t n = 0;
    int64_t ncell = 0;
    std::vector<BoxDesc> hbox;
    std::vector<BoxDesc> uploaded;  // what d.box currently holds
    std::vector<int4> hblocks;      // binning chunks
    std::vector<int4> uploaded_blocks;
    pvl::BinPlan plan;
    DevCells d;
    int64_t cap_n = 0, cap_cell = 0, cap_box = 0, cap_m = 0, cap_blocks = 0;
    bool sorted = false;
    bool drifted = false;   // positions moved by pv_drift since the build
};

namespace {

pv_status fail(pv_ctx *ctx, pv_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

#define HIPCHK(ctx, expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((ctx), PV_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
hipError_t dev_alloc(T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc((void **)p, sizeof(T) * (size_t)count);
}

void free_dev(DevCells &d)
{
    void *ptrs[] = {d.box, d.cell_box, d.cell_start, d.cell_hmax, d.cellid, d.slot, d.stage,
                    d.xyzm, d.H, d.orig, d.sidx, d.gcell, d.box_hmax,
                    d.items, d.qcount, d.scan_tmp, d.binm, d.bin_blocks, d.cell_dx, d.dx_all,
                    d.partial, d.cell_m, d.tiles, d.big, d.rlist};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = DevCells();
}

pv_status ensure_capacity(pv_ctx *ctx, pv_cells *c, int64_t n, int64_t ncell, int nbox,
                          int64_t mtot, int64_t nblocks)
{
    if (n <= c->cap_n && ncell <= c->cap_cell && nbox <= c->cap_box && mtot <= c->cap_m &&
        nblocks <= c->cap_blocks)
        return PV_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    free_dev(c->d);
    c->uploaded.clear();
    c->uploaded_blocks.clear();
    int64_t N = std::max<int64_t>(n, c->cap_n), C = std::max<int64_t>(ncell, c->cap_cell);
    int64_t Bx = std::max<int64_t>(nbox, c->cap_box);
    int64_t M = std::max<int64_t>(mtot, c->cap_m), NB = std::max<int64_t>(nblocks, c->cap_blocks);
    DevCells &d = c->d;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, cnt) if (e == hipSuccess) e = dev_alloc(&ptr, cnt)
    ALLOC(d.box, Bx);
    ALLOC(d.box_hmax, Bx);
    ALLOC(d.cell_box, C);
    ALLOC(d.cell_start, C + 1);
    ALLOC(d.cell_hmax, C);
    ALLOC(d.cellid, N);
    ALLOC(d.slot, N);
    ALLOC(d.stage, 2 * N);
    ALLOC(d.xyzm, N);
    ALLOC(d.H, N);
    ALLOC(d.orig, N);
    ALLOC(d.sidx, 13 * N);
    ALLOC(d.gcell, N);
    ALLOC(d.items, pvl::queue_capacity(N, C));
    ALLOC(d.qcount, pvl::kQueueCounters);
    ALLOC(d.scan_tmp, pvl::scan_scratch_words(C));
    ALLOC(d.binm, M);
    ALLOC(d.bin_blocks, NB);
    ALLOC(d.cell_dx, C);
    ALLOC(d.cell_m, C);
    ALLOC(d.big, pvl::kCellLists * (C + 1));
    d.tslots = pvl::tile_slots(N, C);
    ALLOC(d.tiles, pvl::kTileArrays * d.tslots);
    // receiver lists for the most persistent workgroups a sweep may launch
    d.rlist_wgs = (int64_t)pvl::kQueueWgsMax * std::max(1, ctx->tune.num_cu);
    ALLOC(d.rlist, pvl::kRecvListBytes * d.rlist_wgs);
    ALLOC(d.dx_all, 1);
    ALLOC(d.partial, (int64_t)pvl::kTailMaxCells * pvl::kTailMaxParts * pvl::kTailRecv);
#undef ALLOC
    if (e != hipSuccess) {
        free_dev(c->d);
        c->cap_n = c->cap_cell = c->cap_box = c->cap_m = c->cap_blocks = 0;
        return fail(ctx, PV_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    c->cap_n = N;
    c->cap_cell = C;
    c->cap_box = Bx;
    c->cap_m = M;
    c->cap_blocks = NB;
    return PV_OK;
}

bool boxes_equal(const std::vector<BoxDesc> &a, const std::vector<BoxDesc> &b)
{
    return a.size() == b.size() && (a.empty() || memcmp(a.data(), b.data(), sizeof(BoxDesc) * a.size()) == 0);
}

pv_status upload_boxes(pv_ctx *ctx, pv_cells *c)
{
    const bool same_blocks =
        c->hblocks.size() == c->uploaded_blocks.size() &&
        (c->hblocks.empty() ||
         memcmp(c->hblocks.data(), c->uploaded_blocks.data(), sizeof(int4) * c->hblocks.size()) == 0);
    if (boxes_equal(c->hbox, c->uploaded) && same_blocks) return PV_OK;
    HIPCHK(ctx, hipMemcpyAsync(c->d.box, c->hbox.data(), sizeof(BoxDesc) * c->hbox.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    if (!c->hblocks.empty())
        HIPCHK(ctx, hipMemcpyAsync(c->d.bin_blocks, c->hblocks.data(), sizeof(int4) * c->hblocks.size(),
                                   hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    c->uploaded = c->hbox;
    c->uploaded_blocks = c->hblocks;
    return PV_OK;
}

}  // namespace

extern "C" {

pv_status pv_create(int device, void *hip_stream, pv_ctx **out)
{
    if (!out) return PV_EINVAL;
    *out = nullptr;
    if (device == -1) {
        // argument-checking context: every entry point validates its
        // arguments and then returns PV_ESTATE instead of touching a device
        pv_ctx *ctx = new pv_ctx();
        ctx->device = -1;
        *out = ctx;
        return PV_OK;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PV_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return PV_EHIP;
    pv_ctx *ctx = new pv_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void **)&ctx->dflags, 4 * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&ctx->dcensus, 3 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->hpinned, 64, hipHostMallocDefault) != hipSuccess) {
        pv_destroy(ctx);
        return PV_ENOMEM;
    }
    // the device address of the allocation-free entry point's static scratch
    if (pvl::static_scratch_init(device) != hipSuccess) {
        pv_destroy(ctx);
        return PV_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->tune.num_cu = ctx->tune_adj.num_cu = ctx->tune_plain.num_cu =
            prop.multiProcessorCount;
    if (hipMemset(ctx->dflags, 0, 4 * sizeof(int)) != hipSuccess ||
        hipMemset(ctx->dcensus, 0, 3 * sizeof(unsigned long long)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        pv_destroy(ctx);
        return PV_EHIP;
    }
    *out = ctx;
    return PV_OK;
}

void pv_destroy(pv_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->device < 0) {
        delete ctx;
        return;
    }
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->hcells) pv_free_cells(ctx, ctx->hcells);
    if (ctx->hbuf) (void)hipFree(ctx->hbuf);
    if (ctx->hres) (void)hipFree(ctx->hres);
    if (ctx->dflags) (void)hipFree(ctx->dflags);
    if (ctx->dcensus) (void)hipFree(ctx->dcensus);
    if (ctx->hpinned) (void)hipHostFree(ctx->hpinned);
    for (hipEvent_t ev : ctx->kt_ev) (void)hipEventDestroy(ev);
    delete ctx;
}

pv_status pv_set_stream(pv_ctx *ctx, void *hip_stream)
{
    if (!ctx) return PV_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return PV_OK;
}

const char *pv_last_error(const pv_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

pv_status pv_build_cells_batched(pv_ctx *ctx, int nbox, const int64_t *offsets,
                                 const float *pos, const float *h, const float *mass,
                                 const double *box, const int *grid, pv_cells **cells)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (nbox < 1) return fail(ctx, PV_EINVAL, "nbox < 1");
    if (!offsets || !box) return fail(ctx, PV_EINVAL, "offsets or box is NULL");
    if (offsets[0] != 0) return fail(ctx, PV_EINVAL, "offsets[0] != 0");
    for (int b = 0; b < nbox; ++b)
        if (offsets[b + 1] < offsets[b]) return fail(ctx, PV_EINVAL, "offsets decrease");
    const int64_t n = offsets[nbox];
    if (n > 0x7fffffffLL) return fail(ctx, PV_EINVAL, "more than 2^31-1 particles");
    if (n > 0 && (!pos || !h || !mass)) return fail(ctx, PV_EINVAL, "NULL particle array");
    for (int b = 0; b < 3 * nbox; ++b)
        if (!(box[b] > 0.0) || !isfinite(box[b])) return fail(ctx, PV_EINVAL, "box edge <= 0");
    bool autogrid = (grid == nullptr);
    if (!autogrid) {
        bool allzero = true;
        for (int b = 0; b < 3 * nbox; ++b) allzero &= (grid[b] == 0);
        autogrid = allzero;
    }
    if (!autogrid)
        for (int b = 0; b < 3 * nbox; ++b)
            if (grid[b] < 3 || grid[b] > PV_MAX_GRID)
                return fail(ctx, PV_EGRID, "grid must have 3.." + std::to_string(PV_MAX_GRID) +
                                               " cells per axis");

    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    pv_cells *c = *cells;
    bool fresh = (c == nullptr);
    if (fresh) c = new pv_cells();
    c->hbox.assign(nbox, BoxDesc());
    for (int b = 0; b < nbox; ++b) {
        BoxDesc &B = c->hbox[b];
        for (int a = 0; a < 3; ++a) {
            B.L[a] = (float)box[3 * b + a];
            B.g[a] = 3;
        }
        B.part_off = (int)offsets[b];
        B.n = (int)(offsets[b + 1] - offsets[b]);
    }
    // cell counts are needed to size memory; with an auto grid the largest
    // cut-off of every box is read back first
    std::vector<int> g(3 * nbox);
    if (!autogrid) {
        for (int b = 0; b < 3 * nbox; ++b) g[b] = grid[b];
    }
    auto ncell_of = [&](const std::vector<int> &gg) {
        int64_t t = 0;
        for (int b = 0; b < nbox; ++b) t += (int64_t)gg[3 * b] * gg[3 * b + 1] * gg[3 * b + 2];
        return t;
    };
    pv_status st;
    if (autogrid) {
        c->hblocks.clear();
        st = ensure_capacity(ctx, c, n, std::max<int64_t>(c->cap_cell, 27 * nbox), nbox, 0, 0);
        if (st != PV_OK) { if (fresh) { pv_free_cells(ctx, c); } return st; }
        c->n = n;
        if ((st = upload_boxes(ctx, c)) != PV_OK) { if (fresh) pv_free_cells(ctx, c); return st; }
        hipError_t e = pvl::launch_zero(ctx->stream, c->d.box_hmax, nbox);
        if (e == hipSuccess) e = pvl::launch_box_hmax(ctx->stream, c->d, nbox, n, h);
        std::vector<uint32_t> hm(nbox);
        if (e == hipSuccess) e = hipMemcpyAsync(hm.data(), c->d.box_hmax, sizeof(uint32_t) * nbox,
                                                hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            if (fresh) pv_free_cells(ctx, c);
            return fail(ctx, PV_EHIP, std::string("H_max read-back: ") + hipGetErrorString(e));
        }
        for (int b = 0; b < nbox; ++b) {
            float Hm;
            memcpy(&Hm, &hm[b], 4);
            if (!(Hm >= 0.0f) || !isfinite(Hm)) {
                if (fresh) pv_free_cells(ctx, c);
                return fail(ctx, PV_EINVAL, "non-finite or negative h");
            }
            for (int a = 0; a < 3; ++a) {
                double L = box[3 * b + a];
                int64_t gg = Hm > 0.0f ? (int64_t)floor(L / ((double)Hm * (1.0 + 4e-6))) : PV_MAX_GRID;
                if (gg > PV_MAX_GRID) gg = PV_MAX_GRID;
                if (gg < 3) {
                    if (fresh) pv_free_cells(ctx, c);
                    return fail(ctx, PV_EGRID, "box " + std::to_string(b) +
                                                   ": largest cut-off leaves fewer than 3 cells per axis");
                }
                g[3 * b + a] = (int)gg;
            }
        }
    }
    const int64_t ncell = ncell_of(g);
    if (ncell > 0x7fffffffLL / 2) {
        if (fresh) pv_free_cells(ctx, c);
        return fail(ctx, PV_EGRID, "too many cells");
    }
    int coff = 0;
    for (int b = 0; b < nbox; ++b) {
        BoxDesc &B = c->hbox[b];
        for (int a = 0; a < 3; ++a) {
            B.g[a] = g[3 * b + a];
            double L = box[3 * b + a];
            B.edge[a] = (float)(L / B.g[a]);
            B.inv_edge[a] = (float)(B.g[a] / L);
        }
        B.cell_off = coff;
        coff += B.g[0] * B.g[1] * B.g[2];
    }
    c->plan = pvl::plan_binning(c->hbox, c->hblocks);
    st = ensure_capacity(ctx, c, n, ncell, nbox, c->plan.mtot, c->plan.nblocks);
    if (st != PV_OK) { if (fresh) pv_free_cells(ctx, c); return st; }
    c->nbox = nbox;
    c->n = n;
    c->ncell = ncell;
    c->sorted = false;
    if ((st = upload_boxes(ctx, c)) != PV_OK) { if (fresh) pv_free_cells(ctx, c); return st; }
    c->drifted = false;
    // (the binning also clears the displacement bounds and the occupancy word)
    hipError_t e = pvl::launch_bin(ctx->stream, c->d, c->plan, nbox, n, ncell, pos, h, mass,
                                   ctx->dflags);
    if (e != hipSuccess) {
        if (fresh) pv_free_cells(ctx, c);
        return fail(ctx, PV_EHIP, std::string("binning launch: ") + hipGetErrorString(e));
    }
    if (autogrid) {
        // the auto path synchronises anyway: report occupancy overflow now
        e = hipMemcpyAsync(ctx->hpinned, ctx->dflags, 2 * sizeof(int), hipMemcpyDeviceToHost,
                           ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            if (fresh) pv_free_cells(ctx, c);
            return fail(ctx, PV_EHIP, std::string("occupancy read-back: ") + hipGetErrorString(e));
        }
        if (ctx->hpinned[0] & pvl::kErrOverflow) {
            // reported here, so cleared from the sticky flags
            e = pvl::launch_zero(ctx->stream, ctx->dflags, 1);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            *cells = c;
            return fail(ctx, PV_EOVERFLOW, "a cell holds " + std::to_string(ctx->hpinned[1]) +
                                               " particles (max " + std::to_string(PV_MAX_CELL) + ")");
        }
    }
    *cells = c;
    ctx->err.clear();
    return PV_OK;
}

pv_status pv_build_cells(pv_ctx *ctx, int64_t n, const float *pos, const float *h,
                         const float *mass, const double box[3], const int grid[3],
                         pv_cells **cells)
{
    if (!ctx) return PV_EINVAL;
    if (n < 0) return fail(ctx, PV_EINVAL, "n < 0");
    int64_t off[2] = {0, n};
    return pv_build_cells_batched(ctx, 1, off, pos, h, mass, box, grid, cells);
}

pv_status pv_sort_cells(pv_ctx *ctx, pv_cells *cells)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    if (cells->drifted)
        return fail(ctx, PV_ESTATE, "cells moved by pv_drift are rebuilt, not re-sorted");
    HIPCHK(ctx, pvl::launch_sort13(ctx->stream, cells->d, cells->n, cells->ncell));
    cells->sorted = true;
    return PV_OK;
}

namespace {
// The sweep tuning with the next event pair of the timing ring filled in
// when kernel timing is on and the stream is not being captured.
pvl::SweepTuning timed(pv_ctx *ctx, const pvl::SweepTuning &t)
{
    pvl::SweepTuning r = t;
    if (!ctx->kt_on) return r;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return r;
    r.kt_start = ctx->kt_ev[2 * ctx->kt_next];
    r.kt_stop = ctx->kt_ev[2 * ctx->kt_next + 1];
    ctx->kt_next = (ctx->kt_next + 1) % PV_KTIME_RING;
    ctx->kt_count = std::min(ctx->kt_count + 1, PV_KTIME_RING);
    return r;
}
}  // namespace

pv_status pv_set_kernel_timing(pv_ctx *ctx, int enable)
{
    if (!ctx) return PV_EINVAL;
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    if (enable && ctx->kt_ev.empty()) {
        ctx->kt_ev.assign(2 * PV_KTIME_RING, nullptr);
        for (hipEvent_t &ev : ctx->kt_ev) HIPCHK(ctx, hipEventCreate(&ev));
    }
    ctx->kt_on = enable ? 1 : 0;
    ctx->kt_next = 0;
    ctx->kt_count = 0;
    return PV_OK;
}

pv_status pv_kernel_times(pv_ctx *ctx, float *ms, int *count)
{
    if (!ctx || !count || *count < 0 || (*count > 0 && !ms)) return PV_EINVAL;
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    const int k = std::min(*count, ctx->kt_count);
    *count = 0;
    if (k == 0) return PV_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < k; ++i) {
        // the k most recent pairs, oldest first
        const int slot = ((ctx->kt_next - k + i) % PV_KTIME_RING + PV_KTIME_RING) % PV_KTIME_RING;
        HIPCHK(ctx, hipEventElapsedTime(&ms[i], ctx->kt_ev[2 * slot], ctx->kt_ev[2 * slot + 1]));
    }
    *count = k;
    return PV_OK;
}

pv_status pv_density(pv_ctx *ctx, const pv_cells *cells, pv_algo algo, float *rho,
                     float *wcount, float *drho_dh, int32_t *ncount)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (algo != PV_SORTED_PAIR && algo != PV_PLAIN_CELL) return fail(ctx, PV_EINVAL, "bad algo");
    if (algo == PV_SORTED_PAIR && !cells->sorted)
        return fail(ctx, PV_ESTATE, "pv_sort_cells must run before a sorted-pair density");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    if (ctx->census_on) HIPCHK(ctx, pvl::launch_zero(ctx->stream, ctx->dcensus, 6));
    HIPCHK(ctx, pvl::launch_sweep(ctx->stream, cells->d, cells->n, cells->ncell, (int)algo, rho,
                                  wcount, drho_dh, ncount, ctx->dflags,
                                  ctx->census_on ? ctx->dcensus : nullptr,
                                  timed(ctx, algo == PV_PLAIN_CELL ? ctx->tune_plain : ctx->tune)));
    return PV_OK;
}

pv_status pv_density_backward(pv_ctx *ctx, const pv_cells *cells, const float *grad_rho,
                              float *grad_pos, float *grad_h)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (!grad_rho && cells->n > 0) return fail(ctx, PV_EINVAL, "grad_rho is NULL");
    if (!cells->sorted) return fail(ctx, PV_ESTATE, "pv_sort_cells must run before the adjoint");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    HIPCHK(ctx, pvl::launch_backward(ctx->stream, cells->d, cells->n, cells->ncell, grad_rho,
                                     grad_pos, grad_h, ctx->dflags, timed(ctx, ctx->tune_adj)));
    return PV_OK;
}

pv_status pv_check(pv_ctx *ctx)
{
    if (!ctx) return PV_EINVAL;
    if (ctx->device < 0) return PV_OK;
    HIPCHK(ctx, hipMemcpyAsync(ctx->hpinned, ctx->dflags, 2 * sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    int bits = ctx->hpinned[0];
    if (bits) {
        HIPCHK(ctx, pvl::launch_zero(ctx->stream, ctx->dflags, 1));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (bits & pvl::kErrOverflow)
            return fail(ctx, PV_EOVERFLOW, "a cell held " + std::to_string(ctx->hpinned[1]) +
                                               " particles (max " + std::to_string(PV_MAX_CELL) + ")");
        if (bits & pvl::kErrDrift)
            return fail(ctx, PV_ESTATE, "particles moved farther since the build than the cell "
                                        "edge leaves room for (largest cut-off + twice the "
                                        "displacement > edge): rebuild the cells");
        return fail(ctx, PV_EGRID, "a cut-off exceeded the cell edge (grid too fine) or h <= 0");
    }
    return PV_OK;
}

pv_status pv_cells_info(pv_ctx *ctx, const pv_cells *cells, int grid[3], int64_t *ncell,
                        int32_t *max_occupancy, float *hmax, int *nbox, int64_t *n)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (grid)
        for (int a = 0; a < 3; ++a) grid[a] = cells->hbox.empty() ? 0 : cells->hbox[0].g[a];
    if (ncell) *ncell = cells->ncell;
    if (nbox) *nbox = cells->nbox;
    if (n) *n = cells->n;
    if (max_occupancy || hmax) {
        HIPCHK(ctx, hipMemcpyAsync(ctx->hpinned, ctx->dflags, 2 * sizeof(int),
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (max_occupancy) *max_occupancy = ctx->hpinned[1];
        if (hmax) {
            std::vector<uint32_t> v((size_t)std::max<int64_t>(cells->ncell, 1));
            if (cells->ncell > 0)
                HIPCHK(ctx, hipMemcpy(v.data(), cells->d.cell_hmax, sizeof(uint32_t) * cells->ncell,
                                      hipMemcpyDeviceToHost));
            uint32_t m = 0;
            for (int64_t i = 0; i < cells->ncell; ++i) m = std::max(m, v[i]);
            float f;
            memcpy(&f, &m, 4);
            *hmax = f;
        }
    }
    return PV_OK;
}

pv_status pv_cells_export(pv_ctx *ctx, const pv_cells *cells, int32_t *cell_start,
                          int32_t *order, uint16_t *sorted)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (cell_start)
        HIPCHK(ctx, hipMemcpyAsync(cell_start, cells->d.cell_start, sizeof(int32_t) * (cells->ncell + 1),
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (order && cells->n > 0)
        HIPCHK(ctx, hipMemcpyAsync(order, cells->d.orig, sizeof(int32_t) * cells->n,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (sorted && cells->n > 0) {
        if (!cells->sorted) return fail(ctx, PV_ESTATE, "cells are not sorted");
        HIPCHK(ctx, hipMemcpyAsync(sorted, cells->d.sidx, sizeof(uint16_t) * 13 * cells->n,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    }
    return PV_OK;
}

pv_status pv_set_census(pv_ctx *ctx, int enable)
{
    if (!ctx) return PV_EINVAL;
    ctx->census_on = enable ? 1 : 0;
    return PV_OK;
}

pv_status pv_census(pv_ctx *ctx, int64_t counts[3])
{
    if (!ctx || !counts) return PV_EINVAL;
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    unsigned long long v[3];
    HIPCHK(ctx, hipMemcpyAsync(v, ctx->dcensus, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    counts[0] = (int64_t)v[0];
    counts[1] = (int64_t)v[1];
    counts[2] = (int64_t)v[2];
    return PV_OK;
}

namespace {
// The parameter set a pv_param value addresses, and the parameter within it.
pvl::SweepTuning *param_set(pv_ctx *ctx, int &param)
{
    if (param >= PV_PARAM_PLAIN) {
        param -= PV_PARAM_PLAIN;
        return &ctx->tune_plain;
    }
    if (param >= PV_PARAM_ADJOINT) {
        param -= PV_PARAM_ADJOINT;
        return &ctx->tune_adj;
    }
    return &ctx->tune;
}
}  // namespace

pv_status pv_set_param(pv_ctx *ctx, int param, int value)
{
    if (!ctx) return PV_EINVAL;
    pvl::SweepTuning &t = *param_set(ctx, param);
    switch (param) {
    case PV_PARAM_REACH_ORDER: t.reach_order = value ? 1 : 0; return PV_OK;
    case PV_PARAM_TASK_SORT: t.task_sort = value ? 1 : 0; return PV_OK;
    case PV_PARAM_QUEUE_WGS:
        if (value < 1 || value > pvl::kQueueWgsMax)
            return fail(ctx, PV_EINVAL, "queue_wgs must be 1.." + std::to_string(pvl::kQueueWgsMax));
        t.queue_wgs_per_cu = value;
        return PV_OK;
    case PV_PARAM_CHUNK:
        if (value < 32 || value > 256 || value % 16 != 0)
            return fail(ctx, PV_EINVAL, "chunk must be a multiple of 16 in 32..256");
        t.chunk = value;
        return PV_OK;
    case PV_PARAM_TAIL_PARTS:
        if (value != 1 && value != 2 && value != 4)
            return fail(ctx, PV_EINVAL, "tail_parts must be 1, 2 or 4");
        t.tail_parts = value;
        return PV_OK;
    case PV_PARAM_TAIL_CELLS:
        if (value < 0 || value > pvl::kTailMaxCells)
            return fail(ctx, PV_EINVAL, "tail_cells must be in 0..2048");
        t.tail_cells = value;
        return PV_OK;
    case PV_PARAM_GROUP:
        if (value < 0 || value > pvl::kGroupMax)
            return fail(ctx, PV_EINVAL, "group must be 0..8");
        t.group = value;
        return PV_OK;
    case PV_PARAM_SYM_SELF: t.sym_self = value ? 1 : 0; return PV_OK;
    case PV_PARAM_XCD_RANGES: t.xcd_ranges = value ? 1 : 0; return PV_OK;
    case PV_PARAM_TAIL_SPLIT: t.tail_split = value ? 1 : 0; return PV_OK;
    }
    return fail(ctx, PV_EINVAL, "unknown parameter");
}

pv_status pv_get_param(pv_ctx *ctx, int param, int *value)
{
    if (!ctx || !value) return PV_EINVAL;
    const pvl::SweepTuning &t = *param_set(ctx, param);
    switch (param) {
    case PV_PARAM_REACH_ORDER: *value = t.reach_order; return PV_OK;
    case PV_PARAM_TASK_SORT: *value = t.task_sort; return PV_OK;
    case PV_PARAM_QUEUE_WGS: *value = t.queue_wgs_per_cu; return PV_OK;
    case PV_PARAM_CHUNK: *value = t.chunk; return PV_OK;
    case PV_PARAM_TAIL_PARTS: *value = t.tail_parts; return PV_OK;
    case PV_PARAM_TAIL_CELLS: *value = t.tail_cells; return PV_OK;
    case PV_PARAM_GROUP: *value = t.group; return PV_OK;
    case PV_PARAM_SYM_SELF: *value = t.sym_self; return PV_OK;
    case PV_PARAM_XCD_RANGES: *value = t.xcd_ranges; return PV_OK;
    case PV_PARAM_TAIL_SPLIT: *value = t.tail_split; return PV_OK;
    }
    return fail(ctx, PV_EINVAL, "unknown parameter");
}

pv_status pv_autotune(pv_ctx *ctx, const pv_cells *cells, int target, const float *grad_rho,
                      int reps, float times_ms[2])
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (target != PV_TUNE_DENSITY && target != PV_TUNE_ADJOINT && target != PV_TUNE_PLAIN)
        return fail(ctx, PV_EINVAL, "bad tuning target");
    const bool adj = target == PV_TUNE_ADJOINT;
    const bool plain = target == PV_TUNE_PLAIN;
    if (adj && !grad_rho && cells->n > 0) return fail(ctx, PV_EINVAL, "grad_rho is NULL");
    if (reps < 1 || reps > 100) return fail(ctx, PV_EINVAL, "reps must be 1..100");
    if (!plain && !cells->sorted)
        return fail(ctx, PV_ESTATE, "pv_sort_cells must run before tuning");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    pvl::SweepTuning &cur = adj ? ctx->tune_adj : (plain ? ctx->tune_plain : ctx->tune);
    if (cells->n == 0) {
        if (times_ms) times_ms[0] = times_ms[1] = 0.0f;
        return PV_OK;
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // scratch outputs: 4 words per particle either way
    void *scratch = nullptr;
    HIPCHK(ctx, hipMalloc(&scratch, sizeof(float) * 4 * (size_t)cells->n));
    float *f = (float *)scratch;
    const int64_t n = cells->n;
    auto run = [&](const pvl::SweepTuning &t) -> hipError_t {
        if (adj)
            return pvl::launch_backward(ctx->stream, cells->d, n, cells->ncell, grad_rho, f,
                                        f + 3 * n, ctx->dflags, t);
        return pvl::launch_sweep(ctx->stream, cells->d, n, cells->ncell,
                                 plain ? PV_PLAIN_CELL : PV_SORTED_PAIR, f, f + n,
                                 f + 2 * n, (int32_t *)(f + 3 * n), ctx->dflags, nullptr, t);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto time_of = [&](const pvl::SweepTuning &t, float *ms) -> hipError_t {
        hipError_t r = run(t);
        if (r == hipSuccess) r = hipEventRecord(e0, ctx->stream);
        for (int k = 0; k < reps && r == hipSuccess; ++k) r = run(t);
        if (r == hipSuccess) r = hipEventRecord(e1, ctx->stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
        *ms /= (float)reps;
        return r;
    };
    float before = 0.0f, best_ms = 0.0f;
    pvl::SweepTuning best = cur;
    if (e == hipSuccess) e = time_of(cur, &before);
    best_ms = before;
    static const int chunks[] = {64, 128, 256};
    static const int wgs[] = {1, 2, 3, 4, 5, 6, 8};
    for (int ch : chunks)
        for (int w : wgs)
            for (int ts = 0; ts < 2; ++ts)
                for (int ro = 0; ro < (adj || plain ? 1 : 2); ++ro) {
                    if (e != hipSuccess) break;
                    pvl::SweepTuning t = cur;
                    t.chunk = ch;
                    t.queue_wgs_per_cu = w;
                    t.task_sort = ts;
                    t.reach_order = ro;
                    float ms = 0.0f;
                    e = time_of(t, &ms);
                    if (e == hipSuccess && ms < best_ms) {
                        best_ms = ms;
                        best = t;
                    }
                }
    // then the tail split on top of the best setting
    {
        const pvl::SweepTuning base = best;
        static const int parts[] = {2, 4};
        static const int tails[] = {256, 512, 1024};
        for (int sp = 0; sp < 2; ++sp)
            for (int p : parts)
                for (int tc : tails) {
                    if (e != hipSuccess) break;
                    pvl::SweepTuning t = base;
                    t.tail_parts = p;
                    t.tail_cells = tc;
                    t.tail_split = sp;
                    float ms = 0.0f;
                    e = time_of(t, &ms);
                    if (e == hipSuccess && ms < best_ms) {
                        best_ms = ms;
                        best = t;
                    }
                }
    }
    // then the small-cell groups (the plain sweep takes one cell per item)
    if (!plain) {
        const pvl::SweepTuning base = best;
        static const int groups[] = {1, 2, 4, 8};
        for (int gsz : groups) {
            if (e != hipSuccess || gsz == base.group) continue;
            pvl::SweepTuning t = base;
            t.group = gsz;
            float ms = 0.0f;
            e = time_of(t, &ms);
            if (e == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (e != hipSuccess) return fail(ctx, PV_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    cur = best;
    if (times_ms) {
        times_ms[0] = before;
        times_ms[1] = best_ms;
    }
    return PV_OK;
}

pv_status pv_autotune_grid(pv_ctx *ctx, int nbox, const int64_t *offsets, const float *pos,
                           const float *h, const float *mass, const double *box, int reps,
                           int *grid_out, float times_ms[2])
{
    if (!ctx) return PV_EINVAL;
    if (nbox < 1 || !offsets || !box || !grid_out)
        return fail(ctx, PV_EINVAL, "nbox < 1 or a NULL host array");
    if (reps < 1 || reps > 100) return fail(ctx, PV_EINVAL, "reps must be 1..100");
    const int64_t n = offsets[nbox];
    if (n > 0 && (!pos || !h || !mass)) return fail(ctx, PV_EINVAL, "NULL particle array");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // the finest legal grid of every box (auto grid)
    pv_cells *cells = nullptr;
    pv_status st = pv_build_cells_batched(ctx, nbox, offsets, pos, h, mass, box, nullptr, &cells);
    if (st != PV_OK && st != PV_EOVERFLOW) {
        if (cells) pv_free_cells(ctx, cells);
        return st;
    }
    std::vector<int> finest(3 * nbox);
    for (int b = 0; b < nbox; ++b)
        for (int a = 0; a < 3; ++a) finest[3 * b + a] = cells->hbox[b].g[a];
    float *out = nullptr;
    if (hipMalloc((void **)&out, sizeof(float) * 4 * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
        pv_free_cells(ctx, cells);
        return fail(ctx, PV_ENOMEM, "autotune_grid: device allocation failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    // candidate grids: fractions of the finest grid (at least 3 cells per axis)
    static const float fractions[] = {1.0f, 0.85f, 0.7f, 0.6f, 0.5f, 0.42f, 0.35f, 0.3f};
    std::vector<int> g(3 * nbox), best;
    float best_ms = INFINITY, finest_ms = INFINITY;
    int worse = 0;
    for (float f : fractions) {
        for (int k = 0; k < 3 * nbox; ++k) g[k] = std::max(3, (int)floorf(f * (float)finest[k]));
        if (!best.empty() && g == best) continue;
        auto step = [&]() -> pv_status {
            pv_status s2 = pv_build_cells_batched(ctx, nbox, offsets, pos, h, mass, box, g.data(),
                                                  &cells);
            if (s2 == PV_OK) s2 = pv_sort_cells(ctx, cells);
            if (s2 == PV_OK)
                s2 = pv_density(ctx, cells, PV_SORTED_PAIR, out, out + n, out + 2 * n,
                                (int32_t *)(out + 3 * n));
            return s2;
        };
        st = step();
        if (st == PV_OK) st = pv_check(ctx);
        if (st == PV_EOVERFLOW) {   // too coarse: a cell above the limit
            st = PV_OK;
            break;
        }
        if (st != PV_OK) break;
        (void)hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < reps && st == PV_OK; ++r) st = step();
        (void)hipEventRecord(e1, ctx->stream);
        if (st == PV_OK) st = pv_check(ctx);
        if (st != PV_OK) break;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (f == 1.0f) finest_ms = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = g;
            worse = 0;
        } else if (++worse == 2) {
            break;   // two coarser grids in a row were slower
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    pv_free_cells(ctx, cells);
    if (st != PV_OK) return st;
    if (best.empty())
        return fail(ctx, PV_EOVERFLOW, "even the finest grid has a cell above the limit");
    for (int k = 0; k < 3 * nbox; ++k) grid_out[k] = best[k];
    if (times_ms) {
        times_ms[0] = finest_ms;
        times_ms[1] = best_ms;
    }
    ctx->err.clear();
    return PV_OK;
}

pv_status pv_lj(pv_ctx *ctx, const pv_cells *cells, float eps, float sigma, float *force,
                float *energy)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (!(eps > 0.0f) || !(sigma > 0.0f)) return fail(ctx, PV_EINVAL, "eps and sigma must be > 0");
    if (!cells->sorted) return fail(ctx, PV_ESTATE, "pv_sort_cells must run before pv_lj");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    HIPCHK(ctx, pvl::launch_lj_tiled(ctx->stream, cells->d, cells->n, cells->ncell, eps, sigma,
                                     force, energy, ctx->dflags, timed(ctx, ctx->tune)));
    return PV_OK;
}

pv_status pv_drift(pv_ctx *ctx, pv_cells *cells, const float *disp)
{
    if (!ctx) return PV_EINVAL;
    if (!cells) return fail(ctx, PV_EINVAL, "cells is NULL");
    if (!disp && cells->n > 0) return fail(ctx, PV_EINVAL, "disp is NULL");
    if (!cells->sorted) return fail(ctx, PV_ESTATE, "pv_sort_cells must run before pv_drift");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    HIPCHK(ctx, pvl::launch_drift(ctx->stream, cells->d, cells->ncell, disp));
    cells->drifted = true;
    return PV_OK;
}

pv_status pv_solve_h(pv_ctx *ctx, int nbox, const int64_t *offsets, const float *pos,
                     const float *mass, float *h, const double *box, float ngb, float tol,
                     int max_iter, int *iters, float *resid)
{
    if (!ctx) return PV_EINVAL;
    if (!(ngb > 0.0f) || !(tol > 0.0f)) return fail(ctx, PV_EINVAL, "ngb and tol must be > 0");
    if (max_iter < 1 || max_iter > 1000) return fail(ctx, PV_EINVAL, "max_iter must be 1..1000");
    if (nbox < 1 || !offsets) return fail(ctx, PV_EINVAL, "nbox < 1 or offsets is NULL");
    const int64_t n = offsets[nbox];
    if (n > 0 && (!pos || !mass || !h)) return fail(ctx, PV_EINVAL, "NULL particle array");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const float g = pvl::kGamma;
    const float eta3 = 3.0f * ngb / (4.0f * pvl::kPi * g * g * g);
    // the working set of the last call, grown when n is larger
    if (n > ctx->hbuf_n || !ctx->hbuf) {
        if (ctx->hbuf) (void)hipStreamSynchronize(ctx->stream);
        if (ctx->hbuf) (void)hipFree(ctx->hbuf);
        ctx->hbuf = nullptr;
        ctx->hbuf_n = 0;
        if (hipMalloc((void **)&ctx->hbuf, sizeof(float) * 3 * (size_t)std::max<int64_t>(n, 1)) !=
            hipSuccess) {
            ctx->hbuf = nullptr;
            return fail(ctx, PV_ENOMEM, "solve_h: device allocation failed");
        }
        ctx->hbuf_n = std::max<int64_t>(n, 1);
    }
    if (!ctx->hres && hipMalloc((void **)&ctx->hres, sizeof(uint32_t)) != hipSuccess) {
        ctx->hres = nullptr;
        return fail(ctx, PV_ENOMEM, "solve_h: device allocation failed");
    }
    float *buf = ctx->hbuf;     // rho, drho_dh, h_next
    uint32_t *dres = ctx->hres;
    float *rho = buf, *drho = buf + n, *hnext = buf + 2 * n;
    pv_cells *&cells = ctx->hcells;
    pv_status st = PV_OK;
    float r = INFINITY;
    int it = 0;
    while (it < max_iter) {
        ++it;
        st = pv_build_cells_batched(ctx, nbox, offsets, pos, h, mass, box, nullptr, &cells);
        if (st == PV_OK) st = pv_sort_cells(ctx, cells);
        if (st == PV_OK) st = pv_density(ctx, cells, PV_SORTED_PAIR, rho, nullptr, drho, nullptr);
        if (st == PV_OK) st = pv_check(ctx);
        if (st != PV_OK) break;
        hipError_t e = pvl::launch_zero(ctx->stream, dres, 1);
        if (e == hipSuccess)
            e = pvl::launch_h_newton(ctx->stream, n, rho, drho, mass, h, eta3, hnext, dres);
        uint32_t rb = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->hpinned, dres, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            st = fail(ctx, PV_EHIP, std::string("solve_h: ") + hipGetErrorString(e));
            break;
        }
        rb = (uint32_t)ctx->hpinned[0];
        memcpy(&r, &rb, sizeof(r));
        // h stays the last evaluated one when the loop ends
        if (r <= tol || it == max_iter) break;
        e = pvl::launch_copy_f32(ctx->stream, n, hnext, h);
        if (e != hipSuccess) {
            st = fail(ctx, PV_EHIP, std::string("solve_h: ") + hipGetErrorString(e));
            break;
        }
    }
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (st == PV_OK) ctx->err.clear();
    return st;
}

pv_status pv_density_static(pv_ctx *ctx, int64_t n, const float *pos, const float *h,
                            const float *mass, const double box[3], const int grid[3],
                            pv_algo algo, float *rho, float *wcount, float *drho_dh,
                            int32_t *ncount)
{
    if (!ctx) return PV_EINVAL;
    if (n < 0 || n > PV_STATIC_MAX_N)
        return fail(ctx, PV_EINVAL, "n must be 0.." + std::to_string(PV_STATIC_MAX_N) +
                                        " (the size of the static scratch)");
    if (n > 0 && (!pos || !h || !mass)) return fail(ctx, PV_EINVAL, "NULL particle array");
    if (!box) return fail(ctx, PV_EINVAL, "box is NULL");
    for (int a = 0; a < 3; ++a)
        if (!(box[a] > 0.0) || !isfinite(box[a])) return fail(ctx, PV_EINVAL, "box edge <= 0");
    if (!grid) return fail(ctx, PV_EINVAL, "an explicit grid is required");
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 3 || grid[a] > PV_MAX_GRID)
            return fail(ctx, PV_EGRID, "grid must have 3.." + std::to_string(PV_MAX_GRID) +
                                           " cells per axis");
    if ((int64_t)grid[0] * grid[1] * grid[2] > PV_STATIC_MAX_CELLS)
        return fail(ctx, PV_EINVAL, "more than " + std::to_string(PV_STATIC_MAX_CELLS) +
                                        " cells (the size of the static scratch)");
    if (algo != PV_SORTED_PAIR && algo != PV_PLAIN_CELL) return fail(ctx, PV_EINVAL, "bad algo");
    if (ctx->device < 0) return fail(ctx, PV_ESTATE, "argument-checking context has no device");
    unsigned char *base = pvl::static_scratch(ctx->device);
    if (!base) return fail(ctx, PV_ESTATE, "the static scratch of this device is not set up");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, pvl::launch_density_static(ctx->stream, base, n, pos, h, mass, box, grid,
                                           (int)algo, rho, wcount, drho_dh, ncount, ctx->dflags,
                                           algo == PV_PLAIN_CELL ? ctx->tune_plain : ctx->tune));
    return PV_OK;
}

pv_status pv_free_cells(pv_ctx *ctx, pv_cells *cells)
{
    if (!cells) return PV_OK;
    if (ctx && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    free_dev(cells->d);
    delete cells;
    return PV_OK;
}

}  // extern "C"
