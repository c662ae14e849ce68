// sweep.hip -- dispatch of the batched line-solve kernels (sweep_kernels.h).
#include "sweep_kernels.h"

namespace iga {

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
static SweepFn pick_fn(bool fp32, int P, int lw, int mm, bool diry)
{
    if (fp32) {
        if (P == 2) return pick_sweep_f2(lw, mm, diry);
        if (P == 3) return pick_sweep_f3(lw, mm, diry);
    } else {
        if (P == 2) return pick_sweep_d2(lw, mm, diry);
        if (P == 3) return pick_sweep_d3(lw, mm, diry);
    }
    return nullptr;
}

bool sweep_compiled(int P, int lw, int mm)
{
    return pick_fn(false, P, lw, mm, false) != nullptr;
}

size_t sweep_lds_bytes(const iga_plan *pl, int dir, const Schedule &sc)
{
    const size_t w = pl->wsize;
    size_t scan = (size_t)sc.chunks * sc.lw * pl->P * w;
    size_t xch = (size_t)sc.chunks * sc.lw * 2 * pl->P * w;
    size_t b = scan + xch;
    if (dir == 1) {
        size_t stage = (size_t)sc.lw * pl->Ny * w;
        b = std::max(b, stage);
    }
    return b;
}

iga_status sweep_prepare(const iga_plan *pl, int dir)
{
    const Schedule &sc = pl->sched[dir];
    SweepFn fn = pick_fn(pl->fp32, pl->P, sc.lw, sc.mm, dir == 1);
    if (!fn) return fail(IGA_EUNSUPPORTED, "line-solve kernel not compiled for this schedule");
    const size_t lds = sweep_lds_bytes(pl, dir, sc);
    IGA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return IGA_OK;
}

iga_status launch_sweep(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs, hipStream_t s)
{
    if (njobs < 1 || njobs > MAXJOBS) return fail(IGA_EINVAL, "bad sweep job count");
    const Schedule &sc = pl->sched[dir];
    SweepFn fn = pick_fn(pl->fp32, pl->P, sc.lw, sc.mm, dir == 1);
    if (!fn) return fail(IGA_EUNSUPPORTED, "line-solve kernel not compiled for this schedule");
    SweepParams prm;
    std::memset(&prm, 0, sizeof prm);
    for (int j = 0; j < njobs; ++j) prm.jobs[j] = jobs[j];
    for (int op = 0; op < NOPS; ++op) prm.ops[op] = op_dev(pl, op);
    for (int b = 0; b < NBANDS; ++b) prm.bands[b] = pl->cn_dev[b].ptr;
    prm.N = dir ? pl->Ny : pl->Nx;
    prm.nlines = dir ? pl->Nx : pl->Ny;
    prm.ld = pl->Ny;
    prm.m = sc.m;
    prm.C = sc.chunks;
    prm.D = sc.levels;
    const int nblk = (prm.nlines + sc.lw - 1) / sc.lw;
    const size_t lds = sweep_lds_bytes(pl, dir, sc);
    hipLaunchKernelGGL(fn, dim3(nblk, njobs), dim3(sc.waves * 64), lds, s, prm);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

}  // namespace iga
