// iga_internal.h -- private declarations shared by the host plan, the C ABI
// and the HIP kernels of the wildfire stepper.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/iga.h"

namespace iga {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
iga_status fail(iga_status st, const std::string &msg);
iga_status hip_fail(hipError_t e, const char *what);
#define IGA_HIP(call)                                                  \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::iga::hip_fail(e_, #call);       \
    } while (0)

// ---------------------------------------------------------------------------
// device buffer (RAII)
// ---------------------------------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes)
    {
        o.ptr = nullptr;
        o.bytes = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            ptr = o.ptr;
            bytes = o.bytes;
            o.ptr = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    hipError_t alloc(size_t n) {
        release();
        bytes = n;
        return n ? hipMalloc(&ptr, n) : hipSuccess;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// ---------------------------------------------------------------------------
// banded operators and line-solve schedules
// ---------------------------------------------------------------------------
enum OpId { OP_AX = 0, OP_MX = 1, OP_AY = 2, OP_MY = 3, NOPS = 4 };
enum BandId { BAND_BX = 0, BAND_BY = 1, NBANDS = 2 };

inline int op_dir(int op) { return (op == OP_AX || op == OP_MX) ? 0 : 1; }

// Schedule of the line solves in one direction: a workgroup owns `lines`
// lines, each worked by `wpl` wavefronts; each lane holds a chunk of mm
// consecutive rows (64*wpl chunks per line, lines padded to 64*wpl*mm rows).
struct Schedule {
    int lines = 4, wpl = 1, mm = 17;
    int win = 0;   // 1: windowed solves (see WinGeom), 0: exact chunk scan
    int col = 0;   // 1 (x-lines, FP32): column waves, mm rows per chunk (sweep_col.h)
    int compact = 0;   // windowed: one line buffer per line (see WSweepParams)
};

// Windowed line solves (truncated partition): each lane restarts forward and
// backward substitution from a zero state H rows outside its chunk.  Lanes
// read their coefficient windows from strip tables at a per-lane base row:
//   lane c < nhead               head strip, base off_head + c*mm
//   tail0 <= c < tail1           tail strip, base off_tail + (c - tail0)*mm
//   c >= tail1 (rows >= N only)  identity window at off_id
//   otherwise                    canonical window at off_canon
// Factor tables hold windows of H + mm + H rows (window row j is line row
// c*mm - H + j); refinement rows (A, double) and explicit bands hold windows
// of mm rows (the lane's own rows), with their own offsets (a*).
struct WinGeom {
    int H = 0;    // warm-up rows (and window margin) of a solve
    int Hc = 0;   // warm-up rows of the refinement's correction solve (<= H)
    int nhead = 0, tail0 = 0, tail1 = 0;
    int off_head = 0, off_tail = 0, off_canon = 0, off_id = 0, nrows = 0;
    int aoff_head = 0, aoff_tail = 0, aoff_canon = 0, aoff_id = 0, anrows = 0;
};

// Compressed coefficient tables of one banded operator (host copy).  Rows
// [0, K0) and [NK, N) are kept, the interior rows [K0, NK) -- equal to
// rounding on a uniform mesh -- share the canonical row K0.
//   rows[i*RS + j]      j < P: L(r, r-1-j);  rows[i*RS + P] = 1/U(r,r);
//                       rows[i*RS + P + 1 + j] = U(r, r+1+j)/U(r,r)
//   a64[i*RS + j]       A(r, r-P+j), j <= 2P (the operator, for refinement)
//   tf[c*P*P]           forward transfer matrix of chunk c (64*wpl chunks of mm rows)
//   tb[c*P*P]           backward transfer matrix of chunk c
struct OpHost {
    int K0 = 0, NK = 0, nrows = 0;
    int H = 0;    // warm-up rows of windowed solves (0: decay too slow)
    int Hc = 0;   // warm-up rows of the FP32 refinement's correction solve
    std::vector<double> rows, a64, tf, tb;
    std::vector<double> wrows, wa64;   // windowed strip tables (WinGeom)
};
struct BandHost {
    int K0 = 0, NK = 0, nrows = 0;
    std::vector<double> rows;   // band row r-P .. r+P
    std::vector<double> wrows;  // windowed strip table (mm-row windows)
};

struct DirHost {
    int n = 0, N = 0;
    double L = 0, h = 0;
    std::vector<double> knots;
    std::vector<double> bv, bd;   // [e][a][q] basis values / first derivatives
    std::vector<double> xq;       // [e][q] physical quadrature points
    std::vector<double> wq;       // [q] Gauss weight * h / 2
    std::vector<double> M, K, G;  // bands [N][2P+1]
};

// A captured sequence of `steps` steps bound to one (T, fuel) pair.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void *T = nullptr, *fuel = nullptr;
    int64_t steps = 0;
    void reset();
};

// iga_run keeps two graphs: the main chunk and the tail of the last call.
struct GraphCache {
    GraphEntry main, tail;
    void reset()
    {
        main.reset();
        tail.reset();
    }
};

}  // namespace iga

struct iga_plan {
    iga_plan_desc d;
    int P = 2, Nx = 0, Ny = 0;
    size_t ndof = 0;
    bool fp32 = false;
    bool delta = false;           // increment form (FP32 plans)
    size_t wsize = 8;             // bytes per state element
    iga::DirHost X, Y;
    std::vector<double> op_band[iga::NOPS];    // host FP64 operators
    std::vector<double> cn_band[iga::NBANDS];  // explicit CN operators (B, or B - A)
    iga::Schedule sched[2];
    int win_buffers[2] = {0, 0};   // requested windowed LDS form: 0 automatic, 1 or 2 buffers
    int asm_rows = 16;
    int asm_stack = 0;   // assembly tiles share halos within four-tile workgroups

    // device LU (input bands and factors, double)
    iga::DevBuf op_a64[iga::NOPS], op_lf64[iga::NOPS], op_uf64[iga::NOPS];
    // compressed tables used by the line solves
    iga::OpHost op_host[iga::NOPS];
    iga::BandHost band_host[iga::NBANDS];
    iga::DevBuf op_rows[iga::NOPS], op_a64c[iga::NOPS], op_tf[iga::NOPS], op_tb[iga::NOPS];
    iga::DevBuf band_rows[iga::NBANDS];
    // windowed solve tables of the current schedules
    iga::WinGeom wgeom[2];
    iga::DevBuf op_wrows[iga::NOPS], op_wa64[iga::NOPS], band_wrows[iga::NBANDS];
    // assembly tables
    iga::DevBuf asm_bx, asm_by;                // [e][2][P+1][P+1]  (val, der), state precision
    iga::DevBuf asm_wx, asm_wy;                // wind remainders at x-qps / y-qps
    iga::DevBuf scratch_r, scratch_rf;         // right-hand sides
    iga::DevBuf scratch_r2, scratch_rf2;       // x-solved right-hand sides (column waves)
    // column waves: edge windows of the x operators for the current chunk
    // size (ColEdge in sweep_col.h) and the edge chunks [0, col_lo), [col_hi, ..)
    iga::DevBuf col_edge_f[iga::NOPS], col_edge_d[iga::NOPS];
    int col_lo = 0, col_hi = 0;
    iga::DevBuf flag;                          // non-finite detector
    bool factored = false;
    iga::GraphCache graph;
};

namespace iga {

// host side (plan.cpp)
iga_status build_plan_host(iga_plan *pl);
iga_status upload_plan(iga_plan *pl);
iga_status choose_schedule(iga_plan *pl, int dir, int lines, int wpl);
iga_status build_solve_tables(iga_plan *pl);
iga_status build_scan_tables(iga_plan *pl, int dir);
int warmup_rows(const iga_plan *pl, int dir);   // 0 if a windowed solve is not accurate enough
WinGeom window_geometry(const iga_plan *pl, int dir, int mm, int wpl);
iga_status build_window_tables(iga_plan *pl, int dir);
iga_status choose_window_schedule(iga_plan *pl, int dir, int lines, int mm);
iga_status choose_column_schedule(iga_plan *pl, int mm);

// kernels (factor.hip)
iga_status launch_factor(iga_plan *pl, hipStream_t s);

// kernels (assemble.hip)
// src: optional source sampled at the quadrature points (forced steps)
iga_status launch_assemble(const iga_plan *pl, int substep, const void *T, const void *fuel,
                           void *rhs, void *rhs_fuel, hipStream_t s, const void *src = nullptr);

// kernels (sweep.hip)
struct SweepJob {
    const void *src;
    void *dst;
    int op0;          // first solve (-1: none)
    int band;         // explicit band applied after the first solve (-1: none)
    int op1;          // solve applied to the band product (-1: none)
    const void *base; // added after the first solve (increment form), or NULL
    int add_after;    // 1: result = x + op1^{-1} band x; 0: result = op1^{-1} band x
    // 1: a workgroup whose input lines are all zero leaves them untouched (set
    // only for single solves whose result then equals dst's content: in place
    // without base, or dst == base); the out-of-place column-wave kernel
    // writes the zeros instead of solving
    int zero_skip = 0;
};
iga_status launch_sweep(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs,
                        hipStream_t s);
// column-wave x-line solves (sweep_col.hip): out of place, single solves
bool csweep_ok(const iga_plan *pl);
bool csweep_rows_ok(int mm);
iga_status launch_csweep(const iga_plan *pl, const SweepJob *jobs, int njobs, hipStream_t s);
iga_status build_column_edges(iga_plan *pl, int mm);   // edge windows for chunks of mm rows
int sweep_capacity(int m);           // smallest compiled register capacity >= m (0: none)

// A prepared batched launch over ensemble members: kernel, per-member
// parameter records and the per-workgroup (member, block) table on the device.
struct BatchLaunch {
    const void *fn = nullptr;
    DevBuf prm, info;
    int nblk = 0, njobs = 1, block = 256;
    size_t lds = 0;
};
iga_status build_sweep_batch(const std::vector<iga_plan *> &pls, int dir,
                             const std::vector<std::vector<SweepJob>> &jobs,
                             std::vector<BatchLaunch> &out);
// assembly of substep substeps[m] for member m: (T, fuel) -> (R, R_fuel or NULL)
struct AsmArgs {
    int substep;
    const void *T, *fuel;
    void *R, *RF;
    const void *src = nullptr;   // forced steps only (never batched)
};
iga_status build_assemble_batch(const std::vector<iga_plan *> &pls, const std::vector<AsmArgs> &args,
                                BatchLaunch &out);
iga_status launch_batch(const BatchLaunch &b, hipStream_t s);
iga_status sweep_prepare(const iga_plan *pl, int dir);
size_t sweep_lds_bytes(const iga_plan *pl, int dir, int lines, int wpl);
size_t wsweep_lds_bytes(const iga_plan *pl, int dir, int lines, int wpl, int mm, int compact = 0);
int wsweep_max_block(bool fp32, int mm);   // largest workgroup the windowed kernel allows
iga_status wsweep_prepare(iga_plan *pl, int dir);

// kernels (util)
iga_status launch_nonfinite(const iga_plan *pl, const void *T, const void *fuel, int *flag,
                            hipStream_t s);

// Element rows marched per assembly wavefront that the autotuners try.  The
// list is fine-grained because the kernel time is set by the most loaded
// compute unit: on small meshes one more row per wavefront can remove a whole
// extra round of workgroups from some compute units.
#define ASSEMBLY_ROW_CANDIDATES {4, 5, 6, 7, 8, 9, 10, 11, 12, 14, 16, 20, 24, 28, 32, 40, 48, 64}

// the launches of one step of a plan on fields (T, fuel) (api.cpp)
struct StepPhases {
    AsmArgs a1, a2;
    std::vector<SweepJob> x1, y1, x2, y2;
    bool two = true;   // false: the step is a1, x1, y1 only (explicit scheme)
};
void step_phases(const iga_plan *pl, void *T, void *fuel, StepPhases &sp,
                 void *const *work = nullptr);
// one step of a plan in place (api.cpp); work as for step_phases
iga_status step_impl(const iga_plan *pl, void *T, void *fuel, hipStream_t s,
                     const void *src0 = nullptr, const void *src1 = nullptr,
                     void *const *work = nullptr);
iga_status check_desc(const iga_plan_desc *d);
iga_status check_field(const void *p, const char *name);

// Capture `steps` repetitions of one_step(stream) into g on a private stream
// (kernels only).
template <typename F> iga_status capture_graph(GraphEntry &g, int64_t steps, F &&one_step)
{
    g.reset();
    hipStream_t cs;
    IGA_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    iga_status cst = IGA_OK;
    for (int64_t k = 0; k < steps && !cst; ++k) cst = one_step(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (cst) {
        if (graph) (void)hipGraphDestroy(graph);
        return cst;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    g.graph = graph;
    g.exec = exec;
    g.steps = steps;
    return IGA_OK;
}

// Time `reps` launches of fn between HIP events on s; returns ms per launch
// (negative on failure).
template <typename F> float time_launches(hipStream_t s, int reps, F &&fn)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    float ms = -1.f;
    bool ok = fn() == IGA_OK;   // warm-up
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    for (int i = 0; i < reps && ok; ++i) ok = fn() == IGA_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms /= reps;
    else ms = -1.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace iga
