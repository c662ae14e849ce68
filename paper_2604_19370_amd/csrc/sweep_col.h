// sweep_col.h -- x-line solves with one line per lane ("column waves").
//
// The x-lines of a field (fixed column j, rows i = 0 .. Nx-1, dof (i, j) at
// i*Ny + j) are strided in memory.  Here a wavefront owns 64 consecutive
// columns -- one line per lane -- and a chunk of MM rows of them, so every row
// it touches is one coalesced 256-byte access, and no lane ever needs another
// lane's data: there is no LDS and no barrier.  All lanes work on the same
// row at the same time, so the factor coefficients are wavefront-uniform and
// live in scalar registers (one set for chunks whose rows are all canonical,
// per-row scalar loads near the line ends).
//
// The solve is the banded LU of Section 4 restarted from a zero state outside
// the chunk, as in the windowed kernels (the recurrences contract
// geometrically, by less than 2^-20 over HH rows and 2^-12 over HC rows for
// the operators this kernel accepts; the plan checks).  FP32 refined solve of
// the chunk [r0, r0 + MM):
//   1. x0 = LU^{-1} b on [r0 - HC - P, r0 + MM + HC + P): forward from a zero
//      state HH rows before that range and on through HH rows after it, then
//      backward from the top;
//   2. r = b - A x0 in double on [r0 - HC, r0 + MM + HC);
//   3. d = LU^{-1} r on [r0, r0 + MM) with HC-row warm-ups;
//   4. x = x0 + d.
// Neighbouring waves recompute the overlapping halo rows (read from L2); the
// result is written out of place (dst != src), since other waves still read
// the input rows around a chunk.
#pragma once
#include "sweep_kernels.h"

namespace iga {

constexpr int CMAXJOBS = 2;

struct CSweepOp {
    const float *rows;    // compressed factor rows [nrows][RS] (L, 1/U, U/U_rr)
    const double *a64;    // compressed operator rows [nrows][RS] (A(r, r-P .. r+P))
    const float *ef;      // edge windows (ColEdge): factor coefficients in pass order
    const double *ed;     // edge windows: operator rows of the residual
    int K0, NK, ID;       // rows [0, K0) and [NK, N) stored; interior -> row K0; ID identity row
};

struct CSweepJob {
    const float *src;
    float *dst;
    int zero_skip;        // all-zero input window -> write zeros, skip the solve
    CSweepOp op;
};

struct CSweepParams {
    CSweepJob jobs[CMAXJOBS];
    int N;         // line length (Nx)
    int nlines;    // lines (Ny)
    int ld;        // row stride of the field (Ny)
    int ncg;       // column groups of 64 lines
    int nchunks;   // chunks of MM rows per line
    int lo_end;    // chunks [0, lo_end) and [hi_start, nchunks) reach rows outside
    int hi_start;  // the canonical interior of some job's operator
    int njobs;
};

template <int P> struct ColHalo;
template <> struct ColHalo<1> { static constexpr int HH = 12, HC = 8; };
template <> struct ColHalo<2> { static constexpr int HH = 20, HC = 12; };
template <> struct ColHalo<3> { static constexpr int HH = 28, HC = 20; };

// Chunks whose windows reach rows outside an x operator's canonical interior
// (the first lo_end and those from hi_start on, "edge chunks") read their
// coefficients from edge windows the plan builds: for edge chunk e, the
// coefficients of each window row in the order the passes use them, so a
// pass reads them at compile-time offsets from one base (scalar loads of
// consecutive words).  Floats: forward l of window rows 0 .. NF-1 (P each),
// backward (1/U, u) of window rows HH .. HH+NY-1 (P+1 each), correction
// forward l and backward (1/U, u) of window rows IB .. IB+NR-1; doubles: the
// operator row A(r, r-P .. r+P) of the residual rows (2P+1 each).  Window
// row w is line row r0 - HC - P - HH + w; rows outside the line take the
// identity row.
template <int P, int MM> struct ColEdge {
    static constexpr int HH = ColHalo<P>::HH, HC = ColHalo<P>::HC;
    static constexpr int NY = MM + 2 * (HC + P) + HH, NR = MM + 2 * HC, NF = HH + NY;
    static constexpr int IB = HH + P;
    static constexpr int FL = 0, BU = FL + NF * P, CL = BU + NY * (P + 1), CU = CL + NR * P;
    static constexpr int NFLT = CU + NR * (P + 1);
    static constexpr int NDBL = NR * (2 * P + 1);
};

// The tables are read-only during a launch: read them through the constant
// address space, so uniform reads are scalar loads even after the kernel's
// own stores.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *col_const(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// factor coefficients of one row: l[j] = L(r, r-1-j), ui = 1/U(r,r),
// u[j] = U(r, r+1+j)/U(r,r); a[j] = A(r, r-P+j)
template <int P> struct ColCoef {
    float l[P], ui, u[P];
};
template <int P> struct ColA {
    double a[2 * P + 1];
};

template <int P>
__device__ __forceinline__ ColCoef<P> col_coef(const CSweepOp &o, int idx)
{
    constexpr int RS = 2 * P + 2;
    const auto c = col_const(o.rows) + (size_t)idx * RS;
    ColCoef<P> k;
#pragma unroll
    for (int j = 0; j < P; ++j) k.l[j] = c[j];
    k.ui = c[P];
#pragma unroll
    for (int j = 0; j < P; ++j) k.u[j] = c[P + 1 + j];
    return k;
}

template <int P>
__device__ __forceinline__ ColA<P> col_a(const CSweepOp &o, int idx)
{
    constexpr int RS = 2 * P + 2;
    const auto c = col_const(o.a64) + (size_t)idx * RS;
    ColA<P> k;
#pragma unroll
    for (int j = 0; j < 2 * P + 1; ++j) k.a[j] = c[j];
    return k;
}

// Keeps the compiler from moving instructions across this point (the loads
// of a chunk's window stay ahead of its arithmetic).
__device__ __forceinline__ void col_fence()
{
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
}

// Edge chunks read their coefficients with scalar loads: a fence every 8
// rows keeps them from all being issued (and held in scalar registers) at
// once.
template <bool CANON>
__device__ __forceinline__ void col_row_fence(int i)
{
    if constexpr (!CANON)
        if ((i & 7) == 7) col_fence();
}

// b value of row base + off of this lane's column, the row clamped to [0, N) (the
// caller zeroes rows outside [0, N) once the loads have returned, so no
// per-row flag is held while they are in flight).  Buffer loads: the lane's
// column (clamped to a valid one) is the per-lane byte offset, the row a
// uniform scalar offset, so every access is in bounds and needs no per-lane
// address register.  INSIDE: the row is known to lie in [0, N) (chunks whose
// rows are all canonical).
template <bool INSIDE>
__device__ __forceinline__ float col_load_row(__amdgpu_buffer_rsrc_t rs, int voff, int base, int off,
                                              int N, int ld)
{
    // row base + off: the base is pinned here, so the scalar offsets of the
    // window's rows are neither computed (and held) before the first load
    // nor kept for later passes
    asm volatile("" : "+s"(base));
    const int r = base + off;
    const int rc = INSIDE ? r : min(max(r, 0), N - 1);
    // the builtin returns the raw 32 bits
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, rc * ld * 4, 0));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t col_rsrc(const float *p, int N, int ld)
{
    // raw buffer over the field: num_records in bytes, default word 3
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, N * ld * 4,
                                             0x00020000);
}

// The refined solve of one chunk for this lane's column.  CANON: every row
// in reach uses the canonical coefficients (passed in kc, ka).
// ZS (zero-skip jobs): a wavefront whose whole input window is zero stores
// zeros and stops (the solve of zero data is exactly zero).
template <int P, int MM, bool CANON, bool ZS>
__device__ __forceinline__ void col_solve(const CSweepParams &prm, const CSweepJob &job,
                                          __amdgpu_buffer_rsrc_t rs, int r0, int j, bool jok,
                                          const ColCoef<P> &kc, const ColA<P> &ka, int edge)
{
    constexpr int HH = ColHalo<P>::HH, HC = ColHalo<P>::HC;
    constexpr int NY = MM + 2 * (HC + P) + HH;   // rows kept from the first forward pass
    constexpr int NR = MM + 2 * HC;              // rows of the residual / correction
    constexpr int NF = HH + NY;                  // rows of the first forward pass
    const int N = prm.N, ld = prm.ld;
    const CSweepOp &o = job.op;
    const int voff = min(j, prm.nlines - 1) * 4;   // in bounds for every lane
    // coefficients: the canonical set, or the chunk's edge window (ColEdge),
    // one accessor per pass, each at a compile-time offset
    using E = ColEdge<P, MM>;
    const auto ef = col_const(o.ef) + (size_t)(CANON ? 0 : edge) * E::NFLT;
    const auto ed = col_const(o.ed) + (size_t)(CANON ? 0 : edge) * E::NDBL;
    auto lrow = [&](int off) -> ColCoef<P> {   // forward: l only
        if constexpr (CANON) {
            return kc;
        } else {
            ColCoef<P> k = kc;
#pragma unroll
            for (int q = 0; q < P; ++q) k.l[q] = ef[off + q];
            return k;
        }
    };
    auto urow = [&](int off) -> ColCoef<P> {   // backward: 1/U and u
        if constexpr (CANON) {
            return kc;
        } else {
            ColCoef<P> k = kc;
            k.ui = ef[off];
#pragma unroll
            for (int q = 0; q < P; ++q) k.u[q] = ef[off + 1 + q];
            return k;
        }
    };
    auto acoef = [&](int m) -> ColA<P> {
        if constexpr (CANON) {
            return ka;
        } else {
            ColA<P> k;
#pragma unroll
            for (int q = 0; q < 2 * P + 1; ++q) k.a[q] = ed[m * (2 * P + 1) + q];
            return k;
        }
    };

    // 1. first solve.  Every row of the window is loaded before the first is
    //    used (one memory latency per chunk; the whole window fits in the
    //    registers at this occupancy); forward substitution then overwrites
    //    the loaded rows in place: v[HH + k] = y[k], the value of row ry + k
    const int ry = r0 - HC - P;   // row of y[0]
    const int rf = ry - HH;       // first row of the forward pass
    constexpr int IB = HH + P;    // residual rows r0 - HC .. r0 + MM + HC - 1 are v[IB ..]
    float v[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) v[i] = col_load_row<CANON>(rs, voff, rf, i, N, ld);
    col_fence();
    if constexpr (!CANON) {
        // rows outside [0, N): window rows below lo or from hi on
        const int lo = -rf, hi = N - rf;
#pragma unroll
        for (int i = 0; i < NF; ++i)
            if (i < lo || i >= hi) v[i] = 0.0f;
    }
    // b on the residual rows, kept for the residual and then overwritten in
    // place by it and by the correction
    float rr[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) rr[m] = v[IB + m];
    if constexpr (ZS) {
        bool nz = false;
#pragma unroll
        for (int i = 0; i < NF; ++i) nz = nz || v[i] != 0.0f;
        if (!__any(nz)) {
            if (jok) {
                float *dst = job.dst + j;
#pragma unroll
                for (int k = 0; k < MM; ++k)
                    if (r0 + k < N) dst[(size_t)(r0 + k) * ld] = 0.0f;
            }
            return;
        }
    }
    float s[P];
#pragma unroll
    for (int q = 0; q < P; ++q) s[q] = 0.0f;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const ColCoef<P> c = lrow(E::FL + i * P);
        float x = v[i];
#pragma unroll
        for (int q = P - 1; q >= 0; --q) x -= c.l[q] * s[q];
#pragma unroll
        for (int q = P - 1; q > 0; --q) s[q] = s[q - 1];
        s[0] = x;
        v[i] = x;
        col_row_fence<CANON>(i);
    }
    // backward from the top: rows NY - HH .. NY - 1 are the warm-up
    float t[P];
#pragma unroll
    for (int q = 0; q < P; ++q) t[q] = 0.0f;
#pragma unroll
    for (int k = NY - 1; k >= 0; --k) {
        const ColCoef<P> c = urow(E::BU + k * (P + 1));
        float x = v[HH + k] * c.ui;
#pragma unroll
        for (int q = P - 1; q >= 0; --q) x -= c.u[q] * t[q];
#pragma unroll
        for (int q = P - 1; q > 0; --q) t[q] = t[q - 1];
        t[0] = x;
        v[HH + k] = x;   // x0 for k < NY - HH
        col_row_fence<CANON>(k);
    }
    // 2. residual in double on rows r0 - HC .. r0 + MM + HC - 1 (x0 at row
    //    r - P + q is y[m + q]), over a sliding window of 2P+1 doubles
    const int rr0 = r0 - HC;
    {
        double w[2 * P + 1];
#pragma unroll
        for (int q = 0; q < 2 * P; ++q) w[q + 1] = (double)v[HH + q];
#pragma unroll
        for (int m = 0; m < NR; ++m) {
#pragma unroll
            for (int q = 0; q < 2 * P; ++q) w[q] = w[q + 1];
            w[2 * P] = (double)v[HH + m + 2 * P];
            const ColA<P> a = acoef(m);
            double acc = (double)rr[m];
#pragma unroll
            for (int q = 0; q < 2 * P + 1; ++q) acc -= a.a[q] * w[q];
            rr[m] = (float)acc;
            col_row_fence<CANON>(m);
        }
    }
    // 3. correction: forward from r0 - HC, backward from r0 + MM + HC - 1
#pragma unroll
    for (int q = 0; q < P; ++q) s[q] = 0.0f;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
        const ColCoef<P> c = lrow(E::CL + m * P);
        float x = rr[m];
#pragma unroll
        for (int q = P - 1; q >= 0; --q) x -= c.l[q] * s[q];
#pragma unroll
        for (int q = P - 1; q > 0; --q) s[q] = s[q - 1];
        s[0] = x;
        rr[m] = x;
        col_row_fence<CANON>(m);
    }
#pragma unroll
    for (int q = 0; q < P; ++q) t[q] = 0.0f;
#pragma unroll
    for (int m = NR - 1; m >= HC; --m) {
        const ColCoef<P> c = urow(E::CU + m * (P + 1));
        float x = rr[m] * c.ui;
#pragma unroll
        for (int q = P - 1; q >= 0; --q) x -= c.u[q] * t[q];
#pragma unroll
        for (int q = P - 1; q > 0; --q) t[q] = t[q - 1];
        t[0] = x;
        rr[m] = x;
        col_row_fence<CANON>(m);
    }
    // 4. x = x0 + d on the own rows
    if (jok) {
        float *dst = job.dst + j;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const int r = r0 + k;
            if (r < N) dst[(size_t)r * ld] = v[HH + HC + P + k] + rr[HC + k];
        }
    }
}

// One wavefront (the whole workgroup): column group and chunk from the
// block index in XCD-aware order, job blockIdx.y.
template <int P, int MM>
__device__ __forceinline__ void csweep_body(const CSweepParams &prm)
{
    const int lane = threadIdx.x & 63;
    // Edge chunks load every row's coefficients and take longest: they get
    // the first blocks, which the dispatcher spreads over the XCDs and
    // starts first.  The interior chunks follow; blocks
    // dispatched to one XCD take consecutive chunks of a column group, so
    // the halo rows neighbouring chunks share are in that XCD's L2.
    const int nlo = prm.lo_end, nedge = nlo + prm.nchunks - prm.hi_start;
    const int nint = prm.hi_start - nlo;
    const int b = blockIdx.x, e0 = prm.ncg * nedge;
    int cg, chunk;
    if (b < e0) {
        cg = b / nedge;
        const int e = b - cg * nedge;
        chunk = e < nlo ? e : prm.hi_start + (e - nlo);
    } else {
        const int L = xcd_remap(b - e0, gridDim.x - e0);
        cg = L / nint;
        chunk = nlo + (L - cg * nint);
    }
    const CSweepJob &job = prm.jobs[blockIdx.y];
    const int j = cg * 64 + lane;
    const bool jok = j < prm.nlines;
    const int r0 = chunk * MM;
    const int N = prm.N;
    const CSweepOp &o = job.op;
    // the buffer resource is built here, before the paths diverge, so it
    // stays in scalar registers
    const __amdgpu_buffer_rsrc_t rs = col_rsrc(job.src, N, prm.ld);
    // interior chunks use the canonical rows throughout (their windows lie in
    // every x operator's canonical interior); edge chunks their edge window
    const ColCoef<P> kc = col_coef<P>(o, o.K0);
    const ColA<P> ka = col_a<P>(o, o.K0);
    if (chunk >= prm.lo_end && chunk < prm.hi_start) {
        if (job.zero_skip) col_solve<P, MM, true, true>(prm, job, rs, r0, j, jok, kc, ka, 0);
        else col_solve<P, MM, true, false>(prm, job, rs, r0, j, jok, kc, ka, 0);
    } else {
        const int edge = chunk < prm.lo_end ? chunk : prm.lo_end + (chunk - prm.hi_start);
        col_solve<P, MM, false, false>(prm, job, rs, r0, j, jok, kc, ka, edge);
    }
}

// occupancy target: 3 wavefronts per SIMD (at most 168 VGPRs) where the
// chunk fits, else 2
template <int P, int MM> struct ColWaves {
    static constexpr int value = (P == 3 || MM == 32) ? 2 : 3;
};

template <int P, int MM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ColWaves<P, MM>::value)))
void k_csweep(CSweepParams prm)
{
    csweep_body<P, MM>(prm);
}

}  // namespace iga
