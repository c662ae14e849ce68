// sweep.hip -- launch of the wavefront-per-line banded solves (sweep_kernels.h).
#include "sweep_kernels.h"

namespace iga {

static SweepFn pick_fn(bool fp32, int P, int mm, bool diry)
{
    if (fp32) {
        if (P == 2) return pick_sweep_f2(mm, diry);
        if (P == 3) return pick_sweep_f3(mm, diry);
    } else {
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
        if (P == 2) return pick_sweep_batch_f2(mm, diry);
        if (P == 3) return pick_sweep_batch_f3(mm, diry);
    } else {
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

iga_status launch_sweep(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs, hipStream_t s)
{
    const Schedule &sc = pl->sched[dir];
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
        std::vector<SweepParams> prms;
        std::vector<int2> info;
        int maxjobs = 1;
        size_t lds = 0;
        for (size_t m = m0; m < pls.size(); ++m) {
            const Schedule &sc = pls[m]->sched[dir];
            if (done[m] || sc.mm != key.mm || sc.lines != key.lines || sc.wpl != key.wpl) continue;
            done[m] = 1;
            SweepParams prm;
            iga_status st = build_params(pls[m], dir, jobs[m].data(), (int)jobs[m].size(), prm);
            if (st) return st;
            const int nblk = (prm.nlines + sc.lines - 1) / sc.lines;
            for (int b = 0; b < nblk; ++b) info.push_back(int2{(int)prms.size(), b});
            prms.push_back(prm);
            maxjobs = std::max(maxjobs, prm.njobs);
            lds = std::max(lds, sweep_lds_bytes(pls[m], dir, sc.lines, sc.wpl));
        }
        if (lds > 160 * 1024) return fail(IGA_EUNSUPPORTED, "line-solve tables do not fit in LDS");
        SweepBatchFn fn = pick_batch_fn(pls[m0]->fp32, pls[m0]->P, key.mm, dir == 1);
        if (!fn) return fail(IGA_EUNSUPPORTED, "line-solve kernel not compiled for this schedule");
        IGA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        out.emplace_back();
        BatchLaunch &bl = out.back();
        bl.fn = reinterpret_cast<const void *>(fn);
        bl.nblk = (int)info.size();
        bl.njobs = maxjobs;
        bl.block = key.lines * key.wpl * 64;
        bl.lds = lds;
        IGA_HIP(bl.prm.alloc(prms.size() * sizeof(SweepParams)));
        IGA_HIP(bl.info.alloc(info.size() * sizeof(int2)));
        IGA_HIP(hipMemcpy(bl.prm.ptr, prms.data(), prms.size() * sizeof(SweepParams),
                          hipMemcpyHostToDevice));
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
