// sweep.hip -- launch of the wavefront-per-line banded solves (sweep_kernels.h).
#include "sweep_win.h"

namespace iga {

static SweepFn pick_fn(bool fp32, int P, int mm, bool diry)
{
    if (fp32) {
        if (P == 1) return pick_sweep_f1(mm, diry);
        if (P == 2) return pick_sweep_f2(mm, diry);
        if (P == 3) return pick_sweep_f3(mm, diry);
    } else {
        if (P == 1) return pick_sweep_d1(mm, diry);
        if (P == 2) return pick_sweep_d2(mm, diry);
        if (P == 3) return pick_sweep_d3(mm, diry);
    }
    return nullptr;
}

int sweep_capacity(int m)
{
    static const int caps[] = {4, 8, 12, 17};
    for (int c : caps)
        if (m <= c) return c;
    return 0;
}

static size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

static size_t stage_stride(int N, int dir) { return dir ? (size_t)N : (size_t)(N | 1); }

// LDS of one workgroup: the staged lines, the largest table set a job of this
// direction stages (two factored operators with their refinement rows and
// chunk transfer matrices, and one band) and the line exchange slots.
size_t sweep_lds_bytes(const iga_plan *pl, int dir, int lines, int wpl)
{
    const size_t w = pl->wsize;
    const int N = dir ? pl->Ny : pl->Nx;
    const int P = pl->P, RS = 2 * P + 2, PP = P * P;
    const size_t scan = (size_t)64 * wpl * PP * w;
    size_t b = align16((size_t)lines * stage_stride(N, dir) * w);
    int maxrows = 0;
    for (int op = 0; op < NOPS; ++op)
        if (op_dir(op) == dir) maxrows = std::max(maxrows, pl->op_host[op].nrows);
    for (int bd = 0; bd < NBANDS; ++bd)
        if ((bd == BAND_BX ? 0 : 1) == dir) maxrows = std::max(maxrows, pl->band_host[bd].nrows);
    if (maxrows == 0) maxrows = 96;   // before factorisation: a typical interior-compressed size
    const size_t op_bytes = align16((size_t)maxrows * RS * w) +
                            (pl->fp32 ? align16((size_t)maxrows * RS * 8) : 0) + 2 * align16(scan);
    b += 2 * op_bytes + align16((size_t)maxrows * RS * w);
    b += align16((size_t)lines * 2 * wpl * (PP + P) * w) + align16((size_t)lines * 2 * wpl * 2 * P * w);
    return b;
}

iga_status sweep_prepare(const iga_plan *pl, int dir)
{
    const Schedule &sc = pl->sched[dir];
    SweepFn fn = pick_fn(pl->fp32, pl->P, sc.mm, dir == 1);
    if (!fn) return fail(IGA_EUNSUPPORTED, "line-solve kernel not compiled for this schedule");
    IGA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    return IGA_OK;
}

static SweepBatchFn pick_batch_fn(bool fp32, int P, int mm, bool diry)
{
    if (fp32) {
        if (P == 1) return pick_sweep_batch_f1(mm, diry);
        if (P == 2) return pick_sweep_batch_f2(mm, diry);
        if (P == 3) return pick_sweep_batch_f3(mm, diry);
    } else {
        if (P == 1) return pick_sweep_batch_d1(mm, diry);
        if (P == 2) return pick_sweep_batch_d2(mm, diry);
        if (P == 3) return pick_sweep_batch_d3(mm, diry);
    }
    return nullptr;
}

static iga_status build_params(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs,
                               SweepParams &prm)
{
    if (njobs < 1 || njobs > MAXJOBS) return fail(IGA_EINVAL, "bad sweep job count");
    const Schedule &sc = pl->sched[dir];
    std::memset(&prm, 0, sizeof prm);
    for (int j = 0; j < njobs; ++j) {
        prm.jobs[j] = jobs[j];
        prm.jobs[j].zero_skip = 0;   // not used by the chunk-scan kernels
        if (jobs[j].op0 >= 0 && op_dir(jobs[j].op0) != dir) return fail(IGA_EINVAL, "operator direction");
        if (jobs[j].op1 >= 0 && op_dir(jobs[j].op1) != dir) return fail(IGA_EINVAL, "operator direction");
    }
    for (int op = 0; op < NOPS; ++op) {
        const OpHost &o = pl->op_host[op];
        prm.ops[op] = OpTab{pl->op_rows[op].ptr, pl->op_a64c[op].as<double>(), pl->op_tf[op].ptr,
                            pl->op_tb[op].ptr, o.K0, o.NK, o.nrows};
    }
    for (int b = 0; b < NBANDS; ++b) {
        const BandHost &o = pl->band_host[b];
        prm.bands[b] = BandTab{pl->band_rows[b].ptr, o.K0, o.NK, o.nrows};
    }
    prm.N = dir ? pl->Ny : pl->Nx;
    prm.nlines = dir ? pl->Nx : pl->Ny;
    prm.ld = pl->Ny;
    prm.Ns = (int)stage_stride(prm.N, dir);
    prm.W = sc.lines;
    prm.WPL = sc.wpl;
    prm.njobs = njobs;
    return IGA_OK;
}

// ---------------------------------------------------------------------------
// windowed solves
// ---------------------------------------------------------------------------
static WSweepFn pick_wfn(bool fp32, int P, int mm, bool diry, bool one)
{
    if (fp32) {
        if (P == 1) return pick_wsweep_f1(mm, diry, one);
        if (P == 2) return pick_wsweep_f2(mm, diry, one);
        if (P == 3) return pick_wsweep_f3(mm, diry, one);
    } else {
        if (P == 1) return pick_wsweep_d1(mm, diry, one);
        if (P == 2) return pick_wsweep_d2(mm, diry, one);
        if (P == 3) return pick_wsweep_d3(mm, diry, one);
    }
    return nullptr;
}

static WSweepBatchFn pick_wbatch_fn(bool fp32, int P, int mm, bool diry, bool one)
{
    if (fp32) {
        if (P == 1) return pick_wsweep_batch_f1(mm, diry, one);
        if (P == 2) return pick_wsweep_batch_f2(mm, diry, one);
        if (P == 3) return pick_wsweep_batch_f3(mm, diry, one);
    } else {
        if (P == 1) return pick_wsweep_batch_d1(mm, diry, one);
        if (P == 2) return pick_wsweep_batch_d2(mm, diry, one);
        if (P == 3) return pick_wsweep_batch_d3(mm, diry, one);
    }
    return nullptr;
}

int wsweep_max_block(bool fp32, int mm) { return (mm >= 25 || (!fp32 && mm >= 17)) ? 512 : 1024; }

static int wline_stride(int H, int wpl, int mm) { return 2 * H + 64 * wpl * mm; }

// LDS of one windowed workgroup: two line buffers per line, and the tables
// its job stages (nops factored operators with their refinement rows,
// nbands bands); the launch takes the largest over its jobs.
static size_t wlds(const iga_plan *pl, const WinGeom &g, int lines, int wpl, int mm, int nops,
                   int nbands, int compact)
{
    const size_t w = pl->wsize;
    const int RS = 2 * pl->P + 2;
    size_t b = align16((size_t)(compact ? 1 : 2) * lines * wline_stride(g.H, wpl, mm) * w);
    const size_t op = align16((size_t)g.nrows * RS * w) + (pl->fp32 ? align16((size_t)g.anrows * RS * 8) : 0);
    if (compact) nops = std::min(nops, 1);
    return b + 16 + 64 + nops * op + nbands * align16((size_t)g.anrows * RS * w);
}

// The largest job of a direction: x sweeps solve one operator; y sweeps may
// solve, apply the Crank-Nicolson band and solve again (Strang S1 with S2).
size_t wsweep_lds_bytes(const iga_plan *pl, int dir, int lines, int wpl, int mm, int compact)
{
    const WinGeom g = window_geometry(pl, dir, mm, wpl);
    if (g.H <= 0) return ~(size_t)0;
    return dir == 0 ? wlds(pl, g, lines, wpl, mm, 1, 0, compact)
                    : wlds(pl, g, lines, wpl, mm, 2, 1, compact);
}

static size_t wsweep_lds_jobs(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs)
{
    const Schedule &sc = pl->sched[dir];
    size_t b = 0;
    for (int j = 0; j < njobs; ++j)
        b = std::max(b, wlds(pl, pl->wgeom[dir], sc.lines, sc.wpl, sc.mm,
                             (jobs[j].op0 >= 0) + (jobs[j].op1 >= 0), jobs[j].band >= 0, sc.compact));
    return b;
}

// Also picks the compact form (one line buffer, tables staged in turn) where
// it lets more workgroups share a compute unit than the two-buffer form:
// both compute the same values in the same order, and the compact form
// costs a few barriers, so it only pays where LDS limits residency.
iga_status wsweep_prepare(iga_plan *pl, int dir)
{
    Schedule &sc = pl->sched[dir];
    const int block = sc.lines * sc.wpl * 64;
    int resident[2] = {0, 0};
    for (int one = 0; one < 2; ++one) {
        WSweepFn fn = pick_wfn(pl->fp32, pl->P, sc.mm, dir == 1, one != 0);
        if (!fn) return fail(IGA_EUNSUPPORTED, "windowed line-solve kernel not compiled for this schedule");
        IGA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        const size_t lds = wsweep_lds_bytes(pl, dir, sc.lines, sc.wpl, sc.mm, one);
        if (lds <= 160 * 1024)
            IGA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident[one], fn, block, lds));
    }
    const int req = pl->win_buffers[dir];
    sc.compact = req == 1 ? 1 : req == 2 ? 0 : (resident[1] > resident[0] ? 1 : 0);
    return IGA_OK;
}

static bool zero_skip_valid(const SweepJob &j)
{
    return j.op0 >= 0 && j.band < 0 && j.op1 < 0 &&
           ((j.base == nullptr && j.dst == j.src) || (j.base != nullptr && j.base == j.dst));
}

static iga_status build_wparams(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs,
                                WSweepParams &prm)
{
    if (njobs < 1 || njobs > MAXJOBS) return fail(IGA_EINVAL, "bad sweep job count");
    const Schedule &sc = pl->sched[dir];
    std::memset(&prm, 0, sizeof prm);
    for (int j = 0; j < njobs; ++j) {
        prm.jobs[j] = jobs[j];
        if (jobs[j].zero_skip && !zero_skip_valid(jobs[j]))
            return fail(IGA_EINVAL, "zero_skip on a job whose result is not its destination");
        if (jobs[j].op0 >= 0 && op_dir(jobs[j].op0) != dir) return fail(IGA_EINVAL, "operator direction");
        if (jobs[j].op1 >= 0 && op_dir(jobs[j].op1) != dir) return fail(IGA_EINVAL, "operator direction");
    }
    for (int op = 0; op < NOPS; ++op)
        prm.ops[op] = WinOpTab{pl->op_wrows[op].ptr, pl->op_wa64[op].as<double>()};
    for (int b = 0; b < NBANDS; ++b) prm.bands[b] = WinBandTab{pl->band_wrows[b].ptr};
    prm.g = pl->wgeom[dir];
    prm.N = dir ? pl->Ny : pl->Nx;
    prm.nlines = dir ? pl->Nx : pl->Ny;
    prm.ld = pl->Ny;
    prm.Lb = wline_stride(prm.g.H, sc.wpl, sc.mm);
    prm.W = sc.lines;
    prm.WPL = sc.wpl;
    prm.njobs = njobs;
    prm.compact = sc.compact;
    return IGA_OK;
}


iga_status launch_sweep(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs, hipStream_t s)
{
    const Schedule &sc = pl->sched[dir];
    if (sc.col) {
        if (dir != 0) return fail(IGA_EINVAL, "column-wave schedules are for x-lines");
        return launch_csweep(pl, jobs, njobs, s);
    }
    if (sc.win) {
        WSweepFn fn = pick_wfn(pl->fp32, pl->P, sc.mm, dir == 1, sc.compact != 0);
        if (!fn) return fail(IGA_EUNSUPPORTED, "windowed line-solve kernel not compiled for this schedule");
        WSweepParams prm;
        iga_status st = build_wparams(pl, dir, jobs, njobs, prm);
        if (st) return st;
        const int nblk = (prm.nlines + sc.lines - 1) / sc.lines;
        const size_t lds = wsweep_lds_jobs(pl, dir, jobs, njobs);
        if (lds > 160 * 1024) return fail(IGA_EUNSUPPORTED, "line-solve buffers do not fit in LDS");
        hipLaunchKernelGGL(fn, dim3(nblk, njobs), dim3(sc.lines * sc.wpl * 64), lds, s, prm);
        IGA_HIP(hipGetLastError());
        return IGA_OK;
    }
    SweepFn fn = pick_fn(pl->fp32, pl->P, sc.mm, dir == 1);
    if (!fn) return fail(IGA_EUNSUPPORTED, "line-solve kernel not compiled for this schedule");
    SweepParams prm;
    iga_status st = build_params(pl, dir, jobs, njobs, prm);
    if (st) return st;
    const int nblk = (prm.nlines + sc.lines - 1) / sc.lines;
    const size_t lds = sweep_lds_bytes(pl, dir, sc.lines, sc.wpl);
    if (lds > 160 * 1024) return fail(IGA_EUNSUPPORTED, "line-solve tables do not fit in LDS");
    hipLaunchKernelGGL(fn, dim3(nblk, njobs), dim3(sc.lines * sc.wpl * 64), lds, s, prm);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

// Batched sweeps of one direction over several plans: members are grouped by
// schedule (rows per lane, lines per workgroup, wavefronts per line), one
// launch per group.
iga_status build_sweep_batch(const std::vector<iga_plan *> &pls, int dir,
                             const std::vector<std::vector<SweepJob>> &jobs,
                             std::vector<BatchLaunch> &out)
{
    out.clear();
    if (pls.empty() || jobs.size() != pls.size()) return fail(IGA_EINVAL, "sweep batch: members");
    std::vector<int> done(pls.size(), 0);
    for (size_t m0 = 0; m0 < pls.size(); ++m0) {
        if (done[m0]) continue;
        const Schedule key = pls[m0]->sched[dir];
        if (key.col) return fail(IGA_EUNSUPPORTED, "column-wave schedules are not batched");
        std::vector<SweepParams> prms;
        std::vector<WSweepParams> wprms;
        std::vector<int2> info;
        int maxjobs = 1;
        size_t lds = 0;
        for (size_t m = m0; m < pls.size(); ++m) {
            const Schedule &sc = pls[m]->sched[dir];
            // one launch per workgroup shape: members whose lines need fewer
            // wavefronts join with proportionally more lines per workgroup
            if (done[m] || sc.mm != key.mm || sc.lines * sc.wpl != key.lines * key.wpl ||
                sc.win != key.win || (key.win && sc.compact != key.compact))
                continue;
            done[m] = 1;
            int nlines, njobs;
            if (key.win) {
                WSweepParams prm;
                iga_status st = build_wparams(pls[m], dir, jobs[m].data(), (int)jobs[m].size(), prm);
                if (st) return st;
                nlines = prm.nlines;
                njobs = prm.njobs;
                wprms.push_back(prm);
                lds = std::max(lds, wsweep_lds_jobs(pls[m], dir, jobs[m].data(), (int)jobs[m].size()));
            } else {
                SweepParams prm;
                iga_status st = build_params(pls[m], dir, jobs[m].data(), (int)jobs[m].size(), prm);
                if (st) return st;
                nlines = prm.nlines;
                njobs = prm.njobs;
                prms.push_back(prm);
                lds = std::max(lds, sweep_lds_bytes(pls[m], dir, sc.lines, sc.wpl));
            }
            const int member = (int)(key.win ? wprms.size() : prms.size()) - 1;
            const int nblk = (nlines + sc.lines - 1) / sc.lines;
            for (int b = 0; b < nblk; ++b) info.push_back(int2{member, b});
            maxjobs = std::max(maxjobs, njobs);
        }
        if (lds > 160 * 1024) return fail(IGA_EUNSUPPORTED, "line-solve tables do not fit in LDS");
        const void *fn = key.win
            ? reinterpret_cast<const void *>(pick_wbatch_fn(pls[m0]->fp32, pls[m0]->P, key.mm, dir == 1,
                                                                  key.compact != 0))
            : reinterpret_cast<const void *>(pick_batch_fn(pls[m0]->fp32, pls[m0]->P, key.mm, dir == 1));
        if (!fn) return fail(IGA_EUNSUPPORTED, "line-solve kernel not compiled for this schedule");
        IGA_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        out.emplace_back();
        BatchLaunch &bl = out.back();
        bl.fn = fn;
        bl.nblk = (int)info.size();
        bl.njobs = maxjobs;
        bl.block = key.lines * key.wpl * 64;
        bl.lds = lds;
        const size_t pbytes = key.win ? wprms.size() * sizeof(WSweepParams) : prms.size() * sizeof(SweepParams);
        IGA_HIP(bl.prm.alloc(pbytes));
        IGA_HIP(bl.info.alloc(info.size() * sizeof(int2)));
        IGA_HIP(hipMemcpy(bl.prm.ptr, key.win ? (const void *)wprms.data() : (const void *)prms.data(),
                          pbytes, hipMemcpyHostToDevice));
        IGA_HIP(hipMemcpy(bl.info.ptr, info.data(), info.size() * sizeof(int2),
                          hipMemcpyHostToDevice));
    }
    return IGA_OK;
}

iga_status launch_batch(const BatchLaunch &b, hipStream_t s)
{
    void *prm = b.prm.ptr, *info = b.info.ptr;
    void *args[] = {&prm, &info};
    IGA_HIP(hipLaunchKernel(b.fn, dim3(b.nblk, b.njobs), dim3(b.block), args, b.lds, s));
    return IGA_OK;
}

}  // namespace iga
