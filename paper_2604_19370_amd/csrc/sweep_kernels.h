// sweep_kernels.h -- batched banded line solves of the Kronecker-factored systems
// (Section 4: N_y independent solves of size N_x for an x substep, N_x of size
// N_y for a y substep).
//
// Schedule (one workgroup owns `LW` whole lines):
//   lane (line l, chunk c): rows [c*m, c*m + len) of line l in registers;
//   chunks per line C = waves * 64 / LW.
// Forward and backward substitution are linear recurrences with a p-vector
// state, affine over a chunk.  Each lane runs its chunk with a zero incoming
// state, the chunk end-states are combined across the C chunks of a line by a
// Hillis-Steele scan in LDS whose matrix parts (products of companion
// matrices, data independent) come precomputed from the factorisation, and
// each lane re-runs its chunk from the exact incoming state.  The result is
// the banded LU solve itself (no approximation), with C-fold parallelism per
// line.
//
// Direction x (lines strided by Ny): lanes of a line group read consecutive
// columns, so every row access is coalesced.  Direction y (lines contiguous):
// the workgroup stages its LW whole lines through LDS with contiguous loads
// and stores.
//
// FP32 plans: each solve is x0 = LU32^{-1} b, r = b - A64 x0 formed in double,
// x = x0 + LU32^{-1} r (one step of iterative refinement).
#pragma once
#include "iga_internal.h"

namespace iga {

constexpr int MAXJOBS = 4;

struct SweepParams {
    SweepJob jobs[MAXJOBS];
    OpDev ops[NOPS];
    const void *bands[NBANDS];
    int N;        // line length
    int nlines;   // lines
    int ld;       // row stride of the field (Ny)
    int m;        // rows per chunk
    int C;        // chunks per line
    int D;        // scan levels
};

// blockIdx -> line group with consecutive groups on the same XCD (workgroups
// are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <typename T, int P> struct Chunk {
    int c, ell, r0, len, C, D, LW;
};

// forward substitution over the chunk; s = incoming state (y_{r0-1}, ...),
// on exit the outgoing state.  WRITE: overwrite x with y.
template <typename T, int P, int MM, bool WRITE>
__device__ __forceinline__ void fwd(T (&x)[MM], int len, int r0, const T *__restrict__ lf,
                                    T (&s)[P])
{
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        if (k < len) {
            const T *L = lf + (size_t)(r0 + k) * P;
            T y = x[k];
#pragma unroll
            for (int j = 0; j < P; ++j) y -= L[j] * s[j];
#pragma unroll
            for (int j = P - 1; j > 0; --j) s[j] = s[j - 1];
            s[0] = y;
            if (WRITE) x[k] = y;
        }
    }
}

// backward substitution over the chunk; t = incoming state (x_{r0+len}, ...).
template <typename T, int P, int MM, bool WRITE>
__device__ __forceinline__ void bwd(T (&x)[MM], int len, int r0, const T *__restrict__ uf,
                                    T (&t)[P])
{
#pragma unroll
    for (int k = MM - 1; k >= 0; --k) {
        if (k < len) {
            const T *U = uf + (size_t)(r0 + k) * (P + 1);
            T v = x[k] * U[0];
#pragma unroll
            for (int j = 0; j < P; ++j) v -= U[1 + j] * t[j];
#pragma unroll
            for (int j = P - 1; j > 0; --j) t[j] = t[j - 1];
            t[0] = v;
            if (WRITE) x[k] = v;
        }
    }
}

// Inclusive scan of chunk end-states along a line; on exit v holds the state
// entering this chunk (from the left when FWD, from the right otherwise).
template <typename T, int P, bool FWD>
__device__ __forceinline__ void scan_states(T (&v)[P], int c, int ell, int LW, int C, int D,
                                            const T *__restrict__ tab, T *sb)
{
    constexpr int PP = P * P;
    for (int d = 0; d < D; ++d) {
        const int off = 1 << d;
#pragma unroll
        for (int j = 0; j < P; ++j) sb[(c * LW + ell) * P + j] = v[j];
        __syncthreads();
        const int nc = FWD ? c - off : c + off;
        if (nc >= 0 && nc < C) {
            T o[P];
#pragma unroll
            for (int j = 0; j < P; ++j) o[j] = sb[(nc * LW + ell) * P + j];
            const T *Mt = tab + ((size_t)d * C + c) * PP;
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
                for (int j = 0; j < P; ++j) v[i] += Mt[i * P + j] * o[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < P; ++j) sb[(c * LW + ell) * P + j] = v[j];
    __syncthreads();
    const int pc = FWD ? c - 1 : c + 1;
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = (pc >= 0 && pc < C) ? sb[(pc * LW + ell) * P + j] : T(0);
    __syncthreads();
}

// x <- A^{-1} x for the chunk, exact LU solve of the whole line.
template <typename T, int P, int MM>
__device__ __forceinline__ void chunk_solve(T (&x)[MM], const OpDev &op, int c, int ell, int r0,
                                            int len, int LW, int C, int D, T *sb)
{
    const T *lf = static_cast<const T *>(op.lf);
    const T *uf = static_cast<const T *>(op.uf);
    T s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    fwd<T, P, MM, false>(x, len, r0, lf, s);
    scan_states<T, P, true>(s, c, ell, LW, C, D, static_cast<const T *>(op.tf), sb);
    fwd<T, P, MM, true>(x, len, r0, lf, s);
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    bwd<T, P, MM, false>(x, len, r0, uf, s);
    scan_states<T, P, false>(s, c, ell, LW, C, D, static_cast<const T *>(op.tb), sb);
    bwd<T, P, MM, true>(x, len, r0, uf, s);
}

// Values of the line at rows r0 - P .. r0 + MM + P - 1 as seen from this
// chunk: xe[P + k] = x[k] for k < len, the neighbour chunks' values outside.
template <typename T, int P, int MM>
__device__ __forceinline__ void neighbours(const T (&x)[MM], T (&xe)[MM + 2 * P], int c, int ell,
                                           int len, int LW, int C, T *xb)
{
    // publish first and last P values of the chunk
    T first[P], last[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        first[i] = (i < len) ? x[i] : T(0);
        last[i] = T(0);
    }
#pragma unroll
    for (int k = 0; k < MM; ++k)
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (k == len - P + i) last[i] = x[k];
    T *me = xb + (size_t)(c * LW + ell) * 2 * P;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        me[i] = first[i];
        me[P + i] = last[i];
    }
    __syncthreads();
    T left[P], right[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        left[i] = (c > 0) ? xb[(size_t)((c - 1) * LW + ell) * 2 * P + P + i] : T(0);
        right[i] = (c + 1 < C) ? xb[(size_t)((c + 1) * LW + ell) * 2 * P + i] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < P; ++i) xe[i] = left[i];
#pragma unroll
    for (int k = 0; k < MM + P; ++k) {
        T v = (k < MM && k < len) ? x[k < MM ? k : 0] : T(0);
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (k == len + i) v = right[i];
        xe[P + k] = v;
    }
}

template <typename T, int P, int MM>
__device__ __forceinline__ void solve_refined(T (&x)[MM], const OpDev &op, int c, int ell, int r0,
                                              int len, int LW, int C, int D, T *sb, T *xb)
{
    if constexpr (sizeof(T) == 8) {
        chunk_solve<T, P, MM>(x, op, c, ell, r0, len, LW, C, D, sb);
    } else {
        T b[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) b[k] = x[k];
        chunk_solve<T, P, MM>(x, op, c, ell, r0, len, LW, C, D, sb);
        T xe[MM + 2 * P];
        neighbours<T, P, MM>(x, xe, c, ell, len, LW, C, xb);
        constexpr int W = 2 * P + 1;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            if (k < len) {
                const double *a = op.a64 + (size_t)(r0 + k) * W;
                double r = (double)b[k];
#pragma unroll
                for (int j = 0; j < W; ++j) r -= a[j] * (double)xe[k + j];
                b[k] = (T)r;
            }
        }
        chunk_solve<T, P, MM>(b, op, c, ell, r0, len, LW, C, D, sb);
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] += b[k];
    }
}

template <typename T, int P, int LW, int MM, bool DIRY>
__global__ __launch_bounds__(1024) void k_sweep(SweepParams prm)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const SweepJob job = prm.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int CPW = 64 / LW;
    const int ell = lane % LW;
    const int c = wave * CPW + lane / LW;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int line0 = blk * LW;
    const int line = line0 + ell;
    const int N = prm.N, C = prm.C, D = prm.D;
    const int r0 = c * prm.m;
    int len = N - r0;
    len = len < 0 ? 0 : (len > prm.m ? prm.m : len);
    if (line >= prm.nlines) len = 0;
    const int nl = min(LW, prm.nlines - line0);

    T *sb = reinterpret_cast<T *>(smem);         // scan states [C][LW][P]
    T *xb = sb + (size_t)C * LW * P;             // neighbour exchange [C][LW][2P]
    T *st = reinterpret_cast<T *>(smem);         // y staging [LW][N] (aliases both)

    T x[MM];
    if constexpr (DIRY) {
        const T *src = static_cast<const T *>(job.src) + (size_t)line0 * prm.ld;
        const int tot = nl * N;
        for (int e = tid; e < tot; e += blockDim.x) st[e] = src[e];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] = (k < len) ? st[ell * N + r0 + k] : T(0);
        __syncthreads();
    } else {
        const T *src = static_cast<const T *>(job.src);
#pragma unroll
        for (int k = 0; k < MM; ++k)
            x[k] = (k < len) ? src[(size_t)(r0 + k) * prm.ld + line] : T(0);
    }

    if (job.op0 >= 0)
        solve_refined<T, P, MM>(x, prm.ops[job.op0], c, ell, r0, len, LW, C, D, sb, xb);

    if (job.band >= 0) {
        // explicit Crank-Nicolson operator along the line, then the second solve
        T xe[MM + 2 * P];
        neighbours<T, P, MM>(x, xe, c, ell, len, LW, C, xb);
        constexpr int W = 2 * P + 1;
        const T *bnd = static_cast<const T *>(prm.bands[job.band]);
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            if (k < len) {
                const T *a = bnd + (size_t)(r0 + k) * W;
                T v = T(0);
#pragma unroll
                for (int j = 0; j < W; ++j) v += a[j] * xe[k + j];
                x[k] = v;
            }
        }
        solve_refined<T, P, MM>(x, prm.ops[job.op1], c, ell, r0, len, LW, C, D, sb, xb);
    }

    if constexpr (DIRY) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < len) st[ell * N + r0 + k] = x[k];
        __syncthreads();
        T *dst = static_cast<T *>(job.dst) + (size_t)line0 * prm.ld;
        const int tot = nl * N;
        for (int e = tid; e < tot; e += blockDim.x) dst[e] = st[e];
    } else {
        T *dst = static_cast<T *>(job.dst);
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < len) dst[(size_t)(r0 + k) * prm.ld + line] = x[k];
    }
}

using SweepFn = void (*)(SweepParams);

// instantiation helpers, one translation unit per (precision, degree)
template <typename T, int P, int LW, int MM> static SweepFn pick(bool diry)
{
    return diry ? k_sweep<T, P, LW, MM, true> : k_sweep<T, P, LW, MM, false>;
}

template <typename T, int P> static SweepFn pick_lw_mm(int lw, int mm, bool diry)
{
#define IGA_CASE(LW_, MM_) \
    if (lw == LW_ && mm == MM_) return pick<T, P, LW_, MM_>(diry);
    IGA_CASE(64, 16) IGA_CASE(64, 32) IGA_CASE(64, 48)
    IGA_CASE(16, 16) IGA_CASE(16, 32) IGA_CASE(16, 48)
    IGA_CASE(8, 16) IGA_CASE(8, 32) IGA_CASE(8, 48)
#undef IGA_CASE
    return nullptr;
}

SweepFn pick_sweep_f2(int lw, int mm, bool diry);
SweepFn pick_sweep_f3(int lw, int mm, bool diry);
SweepFn pick_sweep_d2(int lw, int mm, bool diry);
SweepFn pick_sweep_d3(int lw, int mm, bool diry);

}  // namespace iga
