// iga_internal.h -- private declarations shared by the host plan, the C ABI
// and the HIP kernels of the wildfire stepper.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <cstdint>
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

// Schedule of the chunked line solve in one direction: a workgroup of `waves`
// wavefronts owns `lw` whole lines; lane (line l, chunk c) holds rows
// [c*m, c*m + m) of line l in registers (mm = compiled register capacity).
struct Schedule {
    int lw = 16, waves = 16, mm = 32, m = 0, chunks = 0, levels = 0;
};

// Device pointers of one factored operator (all arrays indexed by row r of
// the line, length N):
//   lf[r*P + j]      multiplier L(r, r-1-j) of the unit lower factor
//   uf[r*(P+1)]      1 / U(r, r);  uf[r*(P+1) + 1 + j] = U(r, r+1+j) / U(r, r)
//   tf[(d*C + c)*P*P] forward transfer of chunks c-2^d+1 .. c (scan level d)
//   tb[(d*C + c)*P*P] backward transfer of chunks c .. c+2^d-1
//   a64[r*(2P+1) + (k - r + P)]  the operator itself in double
struct OpDev {
    const void *lf, *uf, *tf, *tb;
    const double *a64;
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
    size_t wsize = 8;             // bytes per state element
    iga::DirHost X, Y;
    std::vector<double> op_band[iga::NOPS];    // host FP64 operators
    std::vector<double> cn_band[iga::NBANDS];  // explicit CN counterparts
    iga::Schedule sched[2];
    int asm_rows = 32;

    // device tables
    iga::DevBuf op_a64[iga::NOPS], op_lf64[iga::NOPS], op_uf64[iga::NOPS];
    iga::DevBuf op_tf64[iga::NOPS], op_tb64[iga::NOPS];
    iga::DevBuf op_lf32[iga::NOPS], op_uf32[iga::NOPS], op_tf32[iga::NOPS], op_tb32[iga::NOPS];
    iga::DevBuf cn_dev[iga::NBANDS];           // explicit bands, state precision
    iga::DevBuf asm_bx, asm_by;                // [e][2][P+1][P+1]  (val, der), state precision
    iga::DevBuf asm_wx, asm_wy;                // wind remainders at x-qps / y-qps
    iga::DevBuf scratch_r, scratch_rf;         // right-hand sides
    iga::DevBuf flag;                          // non-finite detector
    bool factored = false;
    iga::GraphCache graph;
};

namespace iga {

// host side (plan.cpp)
iga_status build_plan_host(iga_plan *pl);
iga_status upload_plan(iga_plan *pl);
iga_status choose_schedule(iga_plan *pl, int dir, int lw, int waves);
OpDev op_dev(const iga_plan *pl, int op);

// kernels (factor.hip)
iga_status launch_factor(iga_plan *pl, hipStream_t s);
iga_status launch_chunk_tables(iga_plan *pl, int op, hipStream_t s);

// kernels (assemble.hip)
iga_status launch_assemble(const iga_plan *pl, int substep, const void *T, const void *fuel,
                           void *rhs, void *rhs_fuel, hipStream_t s);

// kernels (sweep.hip)
struct SweepJob {
    const void *src;
    void *dst;
    int op0;    // first solve
    int band;   // explicit band applied after the first solve (-1: none)
    int op1;    // second solve (-1: none)
};
iga_status launch_sweep(const iga_plan *pl, int dir, const SweepJob *jobs, int njobs,
                        hipStream_t s);
bool sweep_compiled(int P, int lw, int mm);
iga_status sweep_prepare(const iga_plan *pl, int dir);
size_t sweep_lds_bytes(const iga_plan *pl, int dir, const Schedule &sc);

// kernels (util)
iga_status launch_nonfinite(const iga_plan *pl, const void *T, const void *fuel, int *flag,
                            hipStream_t s);

}  // namespace iga
