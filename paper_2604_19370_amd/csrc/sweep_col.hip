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

// Edge windows (ColEdge) of every x operator for chunks of mm rows.  The
// edge chunks are those whose windows leave the canonical interior of some
// x operator, so one range serves any mix of jobs.  A line row r maps to
// the stored row min(r, K0) + max(0, r - NK + 1) of the compressed tables
// (the interior shares row K0), rows outside [0, N) to the identity row;
// factor values are rounded to float as in the state-precision tables.
template <int P, int MM> static iga_status column_edges(iga_plan *pl)
{
    using E = ColEdge<P, MM>;
    constexpr int RS = 2 * P + 2, W = 2 * P + 1, HS = E::HH + E::HC + P;
    const int N = pl->Nx, nchunks = (N + MM - 1) / MM;
    int k0 = 0, nk = N;
    for (int op = 0; op < NOPS; ++op)
        if (op_dir(op) == 0) {
            k0 = std::max(k0, pl->op_host[op].K0);
            nk = std::min(nk, pl->op_host[op].NK);
        }
    const int lo = std::min(nchunks, (k0 + HS + MM - 1) / MM);
    const int top = nk - MM - HS;   // the last interior chunk starts at or below this row
    const int hi = std::min(nchunks, std::max(lo, top >= 0 ? top / MM + 1 : 0));
    const int nedge = lo + nchunks - hi;
    // built aside and moved into the plan only when every table is on the
    // device, so a failure leaves the current schedule's tables intact
    DevBuf ef[NOPS], ed[NOPS];
    for (int op = 0; op < NOPS; ++op) {
        if (op_dir(op) != 0) continue;
        const OpHost &o = pl->op_host[op];
        auto row = [&](int r) -> int {   // stored row of line row r
            if (r < 0 || r >= N) return o.nrows - 1;
            return std::min(r, o.K0) + std::max(0, r - o.NK + 1);
        };
        std::vector<float> f((size_t)std::max(1, nedge) * E::NFLT, 0.f);
        std::vector<double> d((size_t)std::max(1, nedge) * E::NDBL, 0.0);
        for (int e = 0; e < nedge; ++e) {
            const int c = e < lo ? e : hi + (e - lo);
            const int rf = c * MM - HS;   // window row 0
            float *fe = &f[(size_t)e * E::NFLT];
            double *de = &d[(size_t)e * E::NDBL];
            auto fr = [&](int w) { return &o.rows[(size_t)row(rf + w) * RS]; };
            for (int w = 0; w < E::NF; ++w)
                for (int q = 0; q < P; ++q) fe[E::FL + w * P + q] = (float)fr(w)[q];
            for (int k = 0; k < E::NY; ++k)
                for (int q = 0; q <= P; ++q) fe[E::BU + k * (P + 1) + q] = (float)fr(E::HH + k)[P + q];
            for (int m = 0; m < E::NR; ++m) {
                for (int q = 0; q < P; ++q) fe[E::CL + m * P + q] = (float)fr(E::IB + m)[q];
                for (int q = 0; q <= P; ++q) fe[E::CU + m * (P + 1) + q] = (float)fr(E::IB + m)[P + q];
                const double *a = &o.a64[(size_t)row(rf + E::IB + m) * RS];
                for (int q = 0; q < W; ++q) de[m * W + q] = a[q];
            }
        }
        IGA_HIP(ef[op].alloc(f.size() * sizeof(float)));
        IGA_HIP(hipMemcpy(ef[op].ptr, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
        IGA_HIP(ed[op].alloc(d.size() * sizeof(double)));
        IGA_HIP(hipMemcpy(ed[op].ptr, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    for (int op = 0; op < NOPS; ++op) {
        if (op_dir(op) != 0) continue;
        pl->col_edge_f[op] = std::move(ef[op]);
        pl->col_edge_d[op] = std::move(ed[op]);
    }
    pl->col_lo = lo;
    pl->col_hi = hi;
    return IGA_OK;
}

iga_status build_column_edges(iga_plan *pl, int mm)
{
#define IGA_CEDGE(M)                                                \
    if (mm == M) {                                                  \
        if (pl->P == 1) return column_edges<1, M>(pl);              \
        if (pl->P == 2) return column_edges<2, M>(pl);              \
        if (pl->P == 3) return column_edges<3, M>(pl);              \
    }
    IGA_CSWEEP_MMS(IGA_CEDGE)
#undef IGA_CEDGE
    return fail(IGA_EUNSUPPORTED, "column-wave edge windows: no kernel for this schedule");
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
        prm.jobs[i].op.ef = pl->col_edge_f[j.op0].as<float>();
        prm.jobs[i].op.ed = pl->col_edge_d[j.op0].as<double>();
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
    prm.lo_end = pl->col_lo;
    prm.hi_start = pl->col_hi;
    // one wavefront per workgroup: the waves share nothing, and single-wave
    // workgroups retire independently
    const int nblk = prm.ncg * prm.nchunks;
    hipLaunchKernelGGL(fn, dim3(nblk, njobs), dim3(64), 0, s, prm);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

}  // namespace iga
