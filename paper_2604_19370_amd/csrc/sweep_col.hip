// sweep_col.hip -- launcher of the column-wave x-line solves (sweep_col.h).
#include "sweep_col.h"

namespace iga {

#define IGA_CSWEEP_MMS(X) X(16) X(32)

using CSweepFn = void (*)(CSweepParams);

static CSweepFn pick_cfn(int P, int mm)
{
#define IGA_CPICK(M)                                              \
    if (mm == M) {                                                \
        if (P == 1) return k_csweep<1, M>;                        \
        if (P == 2) return k_csweep<2, M>;                        \
        if (P == 3) return k_csweep<3, M>;                        \
    }
    IGA_CSWEEP_MMS(IGA_CPICK)
#undef IGA_CPICK
    return nullptr;
}

bool csweep_rows_ok(int mm) { return mm == 16 || mm == 32; }

// Column waves need FP32 plans and x operators that decay within the
// kernel's compiled warm-ups.
bool csweep_ok(const iga_plan *pl)
{
    if (!pl->fp32) return false;
    int hh = 0, hc = 0;
    if (pl->P == 1) { hh = ColHalo<1>::HH; hc = ColHalo<1>::HC; }
    if (pl->P == 2) { hh = ColHalo<2>::HH; hc = ColHalo<2>::HC; }
    if (pl->P == 3) { hh = ColHalo<3>::HH; hc = ColHalo<3>::HC; }
    for (int op = 0; op < NOPS; ++op) {
        if (op_dir(op) != 0) continue;
        const OpHost &o = pl->op_host[op];
        if (o.H <= 0 || o.Hc <= 0 || o.H > hh || o.Hc > hc) return false;
    }
    return true;
}

iga_status launch_csweep(const iga_plan *pl, const SweepJob *jobs, int njobs, hipStream_t s)
{
    const Schedule &sc = pl->sched[0];
    CSweepFn fn = pick_cfn(pl->P, sc.mm);
    if (!fn) return fail(IGA_EUNSUPPORTED, "column-wave line-solve kernel not compiled for this schedule");
    if (njobs < 1 || njobs > CMAXJOBS) return fail(IGA_EINVAL, "column-wave sweep: 1 or 2 jobs");
    CSweepParams prm;
    std::memset(&prm, 0, sizeof prm);
    for (int i = 0; i < njobs; ++i) {
        const SweepJob &j = jobs[i];
        if (j.op0 < 0 || j.band >= 0 || j.op1 >= 0 || j.base)
            return fail(IGA_EINVAL, "column-wave sweep: single solves only");
        if (j.src == j.dst) return fail(IGA_EINVAL, "column-wave sweep: solves are out of place");
        if (op_dir(j.op0) != 0) return fail(IGA_EINVAL, "column-wave sweep: x operators only");
        const OpHost &o = pl->op_host[j.op0];
        prm.jobs[i].src = static_cast<const float *>(j.src);
        prm.jobs[i].dst = static_cast<float *>(j.dst);
        prm.jobs[i].zero_skip = j.zero_skip;
        prm.jobs[i].op.rows = pl->op_rows[j.op0].as<float>();
        prm.jobs[i].op.a64 = pl->op_a64c[j.op0].as<double>();
        // compressed rows: [0, K0), the canonical row K0, [NK, N), identity
        prm.jobs[i].op.K0 = o.K0;
        prm.jobs[i].op.NK = o.NK;
        prm.jobs[i].op.ID = o.nrows - 1;
    }
    prm.N = pl->Nx;
    prm.nlines = pl->Ny;
    prm.ld = pl->Ny;
    prm.ncg = (pl->Ny + 63) / 64;
    prm.nchunks = (pl->Nx + sc.mm - 1) / sc.mm;
    prm.njobs = njobs;
    // chunks whose rows (with their warm-ups) leave the canonical interior of
    // some job's operator: the first lo_end and those from hi_start on
    {
        int hh = 0;
        if (pl->P == 1) hh = ColHalo<1>::HH + ColHalo<1>::HC + 1;
        if (pl->P == 2) hh = ColHalo<2>::HH + ColHalo<2>::HC + 2;
        if (pl->P == 3) hh = ColHalo<3>::HH + ColHalo<3>::HC + 3;
        int k0 = 0, nk = pl->Nx;
        for (int i = 0; i < njobs; ++i) {
            k0 = std::max(k0, prm.jobs[i].op.K0);
            nk = std::min(nk, prm.jobs[i].op.NK);
        }
        const int lo = std::min(prm.nchunks, (k0 + hh + sc.mm - 1) / sc.mm);
        const int top = nk - sc.mm - hh;   // last canonical chunk starts at or below this row
        const int hi = top >= 0 ? top / sc.mm + 1 : 0;
        prm.lo_end = lo;
        prm.hi_start = std::min(prm.nchunks, std::max(lo, hi));
    }
    // one wavefront per workgroup: the waves share nothing, and single-wave
    // workgroups retire independently
    const int nblk = prm.ncg * prm.nchunks;
    hipLaunchKernelGGL(fn, dim3(nblk, njobs), dim3(64), 0, s, prm);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

}  // namespace iga
