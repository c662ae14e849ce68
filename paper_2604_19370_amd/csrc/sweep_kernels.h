// sweep_kernels.h -- batched banded line solves of the Kronecker-factored
// systems (Section 4: N_y independent solves of size N_x for an x substep,
// N_x of size N_y for a y substep).
//
// A workgroup owns W consecutive lines and stages them in LDS with coalesced
// loads (rows of W consecutive columns for x-lines, W whole contiguous rows
// for y-lines).  Each line is worked by WPL wavefronts; lane c of the line
// (c = part*64 + lane) holds rows [c*MM, c*MM + MM) in registers.  The line is
// padded to 64*WPL*MM rows with identity rows (no multipliers, unit pivot,
// zero data), which leaves the LU solve of the real rows unchanged and keeps
// the recurrences free of per-row predication.
//
// Forward and backward substitution are linear recurrences with a p-vector
// state, affine over a chunk: s_out = Phi_c s_in + psi_c(b).  Each lane runs
// its chunk from a zero state; the chunk maps (Phi_c, psi_c) are combined by a
// Hillis-Steele scan across the wavefront's lanes (shuffles), composing the
// precomputed per-chunk transfer matrices as it goes, then across the WPL
// wavefronts of the line (one LDS exchange); each lane re-runs its chunk from
// its exact incoming state.  The result is the banded LU solve of the line.
//
// Coefficients.  Interior rows of a factored operator on a uniform mesh agree
// to rounding (the LU of a banded Toeplitz matrix converges to a constant row
// within a few tens of rows); the plan keeps rows [0, K0) and [NK, N), one
// canonical row for [K0, NK) and an identity row for the padding, in LDS, so
// lanes on interior chunks all read the same address.
//
// FP32 plans: every solve is x0 = LU32^{-1} b, r = b - A64 x0 formed in double,
// x = x0 + LU32^{-1} r (one step of iterative refinement), and the state is
// advanced in increment form (the job adds the base field after the solve).
#pragma once
#include "iga_internal.h"

namespace iga {

constexpr int MAXJOBS = 4;
constexpr int MAXWPL = 8;        // wavefronts per line

// compressed coefficient rows (device, state precision unless noted)
struct OpTab {
    const void *rows;     // [nrows][RS] : L(r, r-1-j) j<P, 1/U(r,r), U(r,r+1+j)/U(r,r)
    const double *a64;    // [nrows][RS] : A(r, r-P .. r+P) in double
    const void *tf, *tb;  // [64*WPL][P*P] forward / backward transfer matrix of each chunk
    int K0, NK, nrows;    // row r -> table row min(min(r, K0) + max(0, r - NK + 1), nrows - 1)
};
struct BandTab {
    const void *rows;     // [nrows][RS] : band row r-P .. r+P (last row: zero, for padding)
    int K0, NK, nrows;
};

struct SweepParams {
    SweepJob jobs[MAXJOBS];
    OpTab ops[NOPS];
    BandTab bands[NBANDS];
    int N;        // line length
    int nlines;   // lines
    int ld;       // row stride of the field (Ny)
    int Ns;       // LDS stride between staged lines
    int W;        // lines per workgroup (power of two)
    int WPL;      // wavefronts per line (power of two)
    int njobs;    // jobs in use
};

template <int P> struct RowStride {
    static constexpr int RS = 2 * P + 2;
};

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// table row of line row r: rows below K0 and from NK on are stored, the
// interior shares row K0, padding rows (r >= N) map to the last table row
struct RowMap {
    int K0, NK1, ID;   // NK1 = NK - 1
};
__device__ __forceinline__ int row_index(int r, const RowMap &rm)
{
    return min(min(r, rm.K0) + max(0, r - rm.NK1), rm.ID);
}

template <typename T> __device__ __forceinline__ T shfl_up(T v, int d) { return __shfl_up(v, d, 64); }
template <typename T> __device__ __forceinline__ T shfl_down(T v, int d) { return __shfl_down(v, d, 64); }

// forward substitution over the chunk; s = state (y_{r-1}, y_{r-2}, ...)
template <typename T, int P, int MM, bool WRITE>
__device__ __forceinline__ void fwd(T (&x)[MM], int r0, const T *rows, const RowMap &rm,
                                    T (&s)[P])
{
    constexpr int RS = RowStride<P>::RS;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        const T *L = rows + row_index(r0 + k, rm) * RS;
        T y = x[k];
#pragma unroll
        for (int j = 0; j < P; ++j) y -= L[j] * s[j];
#pragma unroll
        for (int j = P - 1; j > 0; --j) s[j] = s[j - 1];
        s[0] = y;
        if (WRITE) x[k] = y;
    }
}

// backward substitution over the chunk; t = state (x_{r+1}, x_{r+2}, ...)
template <typename T, int P, int MM, bool WRITE>
__device__ __forceinline__ void bwd(T (&x)[MM], int r0, const T *rows, const RowMap &rm,
                                    T (&t)[P])
{
    constexpr int RS = RowStride<P>::RS;
#pragma unroll
    for (int k = MM - 1; k >= 0; --k) {
        const T *U = rows + row_index(r0 + k, rm) * RS + P;
        T v = x[k] * U[0];
#pragma unroll
        for (int j = 0; j < P; ++j) v -= U[1 + j] * t[j];
#pragma unroll
        for (int j = P - 1; j > 0; --j) t[j] = t[j - 1];
        t[0] = v;
        if (WRITE) x[k] = v;
    }
}

// Per-line context of a wavefront: which part of the line it works and the
// LDS slots shared by the line's wavefronts.
template <typename T> struct LineCtx {
    int lane, part, WPL;
    T *xscan;   // [2][WPL][P*P + P] wave totals of the two alternating scans
    T *xnb;     // [2][WPL][2P] first / last P values of each wavefront's rows
    int flip, nflip;
};

// Scan of the chunk maps along the line; on entry v is this chunk's
// particular end-state (zero incoming state), on exit the exact state
// entering this chunk from the left (FWD) or from the right.
template <typename T, int P, bool FWD>
__device__ __forceinline__ void line_scan(T (&v)[P], const T *__restrict__ tab, LineCtx<T> &ctx)
{
    constexpr int PP = P * P;
    const int lane = ctx.lane;
    T F[PP];
    const int c = ctx.part * 64 + lane;
#pragma unroll
    for (int i = 0; i < PP; ++i) F[i] = tab[c * PP + i];
    // inclusive scan within the wavefront
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int off = 1 << d;
        T o[P], oF[PP];
#pragma unroll
        for (int j = 0; j < P; ++j) o[j] = FWD ? shfl_up(v[j], off) : shfl_down(v[j], off);
#pragma unroll
        for (int i = 0; i < PP; ++i) oF[i] = FWD ? shfl_up(F[i], off) : shfl_down(F[i], off);
        const bool has = FWD ? lane >= off : lane + off < 64;
        T nF[PP], nv[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            nv[i] = v[i];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                nv[i] += F[i * P + j] * o[j];
                T s = T(0);
#pragma unroll
                for (int k = 0; k < P; ++k) s += F[i * P + k] * oF[k * P + j];
                nF[i * P + j] = s;
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i) v[i] = has ? nv[i] : v[i];
#pragma unroll
        for (int i = 0; i < PP; ++i) F[i] = has ? nF[i] : F[i];
    }
    // exclusive maps: shift by one lane (identity map at the wave's first lane)
    const int edge = FWD ? 0 : 63;
    T ev[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const T o = FWD ? shfl_up(v[j], 1) : shfl_down(v[j], 1);
        ev[j] = lane == edge ? T(0) : o;
    }
    if (ctx.WPL == 1) {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = ev[j];
        return;
    }
    T eF[PP];
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const T o = FWD ? shfl_up(F[i], 1) : shfl_down(F[i], 1);
        eF[i] = lane == edge ? ((i / P == i % P) ? T(1) : T(0)) : o;
    }
    // wave totals across the line's wavefronts (two alternating slot sets, so
    // one barrier per scan suffices)
    constexpr int SL = PP + P;
    T *slot = ctx.xscan + (size_t)ctx.flip * ctx.WPL * SL;
    ctx.flip ^= 1;
    const int last = FWD ? 63 : 0;
    if (lane == last) {
        T *me = slot + ctx.part * SL;
#pragma unroll
        for (int i = 0; i < PP; ++i) me[i] = F[i];
#pragma unroll
        for (int j = 0; j < P; ++j) me[PP + j] = v[j];
    }
    __syncthreads();
    T S[P];
#pragma unroll
    for (int j = 0; j < P; ++j) S[j] = T(0);
    const int q0 = FWD ? 0 : ctx.WPL - 1;
    const int nq = FWD ? ctx.part : ctx.WPL - 1 - ctx.part;
    for (int t = 0; t < nq; ++t) {
        const int q = FWD ? q0 + t : q0 - t;
        const T *o = slot + q * SL;
        T n[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            n[i] = o[PP + i];
#pragma unroll
            for (int j = 0; j < P; ++j) n[i] += o[i * P + j] * S[j];
        }
#pragma unroll
        for (int i = 0; i < P; ++i) S[i] = n[i];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        T s = ev[i];
#pragma unroll
        for (int j = 0; j < P; ++j) s += eF[i * P + j] * S[j];
        v[i] = s;
    }
}

template <typename T, int P, int MM>
__device__ __forceinline__ void chunk_solve(T (&x)[MM], const T *rows, const T *tf, const T *tb,
                                            const RowMap &rm, LineCtx<T> &ctx, int r0)
{
    T s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    fwd<T, P, MM, false>(x, r0, rows, rm, s);
    line_scan<T, P, true>(s, tf, ctx);
    fwd<T, P, MM, true>(x, r0, rows, rm, s);
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    bwd<T, P, MM, false>(x, r0, rows, rm, s);
    line_scan<T, P, false>(s, tb, ctx);
    bwd<T, P, MM, true>(x, r0, rows, rm, s);
}

// The P rows of the line just before (left) and just after (right) this
// lane's chunk.
template <typename T, int P, int MM>
__device__ __forceinline__ void neighbours(const T (&x)[MM], T (&left)[P], T (&right)[P],
                                           LineCtx<T> &ctx)
{
    const int lane = ctx.lane;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        left[i] = shfl_up(x[MM - P + i], 1);
        right[i] = shfl_down(x[i], 1);
    }
    if (ctx.WPL == 1) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            left[i] = lane > 0 ? left[i] : T(0);
            right[i] = lane < 63 ? right[i] : T(0);
        }
        return;
    }
    // across the line's wavefronts: lanes 0 and 63 publish their edge rows
    T *nb = ctx.xnb + (size_t)ctx.nflip * ctx.WPL * 2 * P;
    ctx.nflip ^= 1;
    T *me = nb + ctx.part * 2 * P;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < P; ++i) me[i] = x[i];
    }
    if (lane == 63) {
#pragma unroll
        for (int i = 0; i < P; ++i) me[P + i] = x[MM - P + i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const T l = ctx.part > 0 ? nb[(ctx.part - 1) * 2 * P + P + i] : T(0);
        const T r = ctx.part + 1 < ctx.WPL ? nb[(ctx.part + 1) * 2 * P + i] : T(0);
        left[i] = lane > 0 ? left[i] : l;
        right[i] = lane < 63 ? right[i] : r;
    }
}

// value of the line at chunk-relative row idx (compile-time), P <= MM
template <typename T, int P, int MM>
__device__ __forceinline__ T around(const T (&x)[MM], const T (&left)[P], const T (&right)[P],
                                    int idx)
{
    return idx < 0 ? left[idx + P] : (idx >= MM ? right[idx - MM] : x[idx]);
}

// One operator's tables as the kernel sees them (rows in LDS).
template <typename T> struct OpView {
    const T *rows;
    const double *a64;
    const T *tf, *tb;
    RowMap rm;
};

// x <- A^{-1} x; FP32 refines once with the residual b - A64 x0 in double
// (b = the value of x on entry).
template <typename T, int P, int MM>
__device__ __forceinline__ void solve_refined(T (&x)[MM], const OpView<T> &op, LineCtx<T> &ctx,
                                              int r0)
{
    if constexpr (sizeof(T) == 8) {
        chunk_solve<T, P, MM>(x, op.rows, op.tf, op.tb, op.rm, ctx, r0);
    } else {
        constexpr int RS = RowStride<P>::RS;
        T b[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) b[k] = x[k];
        chunk_solve<T, P, MM>(x, op.rows, op.tf, op.tb, op.rm, ctx, r0);
        T left[P], right[P];
        neighbours<T, P, MM>(x, left, right, ctx);
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const double *a = op.a64 + row_index(r0 + k, op.rm) * RS;
            double r = (double)b[k];
#pragma unroll
            for (int j = 0; j < 2 * P + 1; ++j)
                r -= a[j] * (double)around<T, P, MM>(x, left, right, k + j - P);
            b[k] = (T)r;
        }
        chunk_solve<T, P, MM>(b, op.rows, op.tf, op.tb, op.rm, ctx, r0);
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] += b[k];
    }
}

// copy `nwords` 32-bit words from global `g` straight into LDS `lds` with the
// whole workgroup (global_load_lds: no registers, every load in flight at
// once).  Instruction k of the copy moves words [64k, 64k + 64); lane i
// writes LDS word 64k + i.  The data are visible to the workgroup after the
// next barrier (the compiler waits for the transfers there).
__device__ __forceinline__ void lds_dma_words(void *lds, const void *g, int nwords)
{
    typedef __attribute__((address_space(1))) const void gvoid;
    typedef __attribute__((address_space(3))) void lvoid;
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const unsigned *src = static_cast<const unsigned *>(g);
    unsigned *dst = static_cast<unsigned *>(lds);
    for (int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); k * 64 < nwords; k += nw) {
        const int i = k * 64 + lane;
        if (i < nwords) __builtin_amdgcn_global_load_lds((gvoid *)(src + i), (lvoid *)(dst + k * 64), 4, 0, 0);
    }
}

// a table of n elements of type U, staged by DMA (sizes are whole words)
template <typename U> __device__ __forceinline__ void stage_table_dma(U *dst, const void *src, int n)
{
    static_assert(sizeof(U) % 4 == 0, "tables hold 32- or 64-bit elements");
    lds_dma_words(dst, src, (int)(n * sizeof(U) / 4));
}

// workgroup size bound: 16 wavefronts, or 8 where cubic double chunks of 12+
// rows need more than 128 registers
template <typename T, int P, int MM> constexpr int sweep_max_threads()
{
    return (sizeof(T) == 8 && P == 3 && MM >= 12) ? 512 : 1024;
}

// One workgroup's work: W lines starting at line blk*W, job `jobi`.
template <typename T, int P, int MM, bool DIRY>
__device__ __forceinline__ void sweep_body(const SweepParams &prm, const int blk, const int jobi)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RS = RowStride<P>::RS;
    constexpr int PP = P * P;
    constexpr bool F32 = sizeof(T) == 4;
    const SweepJob job = prm.jobs[jobi];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = prm.W, WPL = prm.WPL;
    const int wlog = __builtin_ctz(W);
    const int rstep = blockDim.x >> wlog;
    const int N = prm.N, Ns = prm.Ns, ld = prm.ld;
    const int line0 = blk * W;
    const int nl = min(W, prm.nlines - line0);
    const int lw = wave / WPL;          // line of this wavefront within the workgroup
    const int part = wave - lw * WPL;   // its part of the line
    const int C = 64 * WPL;             // chunks per line

    // LDS: staged lines, then the tables of this job and the line exchange slots
    T *st = reinterpret_cast<T *>(smem);
    // y-lines: the input block is copied by DMA while the tables are staged
    if constexpr (DIRY)
        lds_dma_words(st, static_cast<const T *>(job.src) + (size_t)line0 * ld, (int)(nl * N * sizeof(T) / 4));
    size_t off = ((size_t)W * Ns * sizeof(T) + 15) & ~(size_t)15;
    auto take = [&](size_t bytes) {
        unsigned char *p = smem + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    auto stage_op = [&](const OpTab &t, OpView<T> &v) {
        T *rows = reinterpret_cast<T *>(take((size_t)t.nrows * RS * sizeof(T)));
        stage_table_dma<T>(rows, t.rows, t.nrows * RS);
        v.rows = rows;
        v.a64 = nullptr;
        if (F32) {
            double *a = reinterpret_cast<double *>(take((size_t)t.nrows * RS * sizeof(double)));
            stage_table_dma<double>(a, t.a64, t.nrows * RS);
            v.a64 = a;
        }
        T *tf = reinterpret_cast<T *>(take((size_t)C * PP * sizeof(T)));
        T *tb = reinterpret_cast<T *>(take((size_t)C * PP * sizeof(T)));
        stage_table_dma<T>(tf, t.tf, C * PP);
        stage_table_dma<T>(tb, t.tb, C * PP);
        v.tf = tf;
        v.tb = tb;
        v.rm = RowMap{t.K0, t.NK - 1, t.nrows - 1};
    };
    OpView<T> v0, v1;
    const bool has0 = job.op0 >= 0, has1 = job.op1 >= 0, hasb = job.band >= 0;
    if (has0) stage_op(prm.ops[job.op0], v0);
    if (has1) stage_op(prm.ops[job.op1], v1);
    const T *brow = nullptr;
    RowMap brm{0, 0, 0};
    if (hasb) {
        const BandTab &t = prm.bands[job.band];
        T *rows = reinterpret_cast<T *>(take((size_t)t.nrows * RS * sizeof(T)));
        stage_table_dma<T>(rows, t.rows, t.nrows * RS);
        brow = rows;
        brm = RowMap{t.K0, t.NK - 1, t.nrows - 1};
    }
    LineCtx<T> ctx;
    ctx.lane = lane;
    ctx.part = part;
    ctx.WPL = WPL;
    ctx.flip = 0;
    ctx.nflip = 0;
    ctx.xscan = reinterpret_cast<T *>(take((size_t)W * 2 * WPL * (PP + P) * sizeof(T))) +
                (size_t)lw * 2 * WPL * (PP + P);
    ctx.xnb = reinterpret_cast<T *>(take((size_t)W * 2 * WPL * 2 * P * sizeof(T))) +
              (size_t)lw * 2 * WPL * 2 * P;

    // Stage W lines of a field (src layout) into st, and back.  y-lines: the
    // W rows are one contiguous block (Ns == N), copied straight into LDS by
    // DMA, every load in flight at once.  x-lines: rows of W consecutive
    // columns; loads are issued in batches of UNR per thread before their LDS
    // stores so that their latencies overlap.
    constexpr int UNR = 8;
    auto load_lines = [&](const T *src) {
        if constexpr (DIRY) {
            // one contiguous run in HBM and in LDS: copied by DMA
            lds_dma_words(st, src + (size_t)line0 * ld, (int)(nl * N * sizeof(T) / 4));
        } else {
            const int j = tid & (W - 1);
            const bool jok = j < nl;
            const int r00 = tid >> wlog;
            for (int b0 = 0; b0 < N; b0 += UNR * rstep) {
                T v[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int r = b0 + u * rstep + r00;
                    v[u] = (jok && r < N) ? src[(size_t)r * ld + line0 + j] : T(0);
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int r = b0 + u * rstep + r00;
                    if (jok && r < N) st[j * Ns + r] = v[u];
                }
            }
        }
    };
    auto store_lines = [&](T *dst) {
        if constexpr (DIRY) {
            T *d = dst + (size_t)line0 * ld;
            const int tot = nl * N;
            for (int e = tid; e < tot; e += blockDim.x) d[e] = st[e];
        } else {
            const int j = tid & (W - 1);
            if (j < nl)
                for (int r = tid >> wlog; r < N; r += rstep)
                    dst[(size_t)r * ld + line0 + j] = st[j * Ns + r];
        }
    };

    if constexpr (!DIRY) load_lines(static_cast<const T *>(job.src));
    __syncthreads();

    // this lane's chunk: rows [r0, r0 + MM) of line lw; rows >= N are padding
    const int r0 = (part * 64 + lane) * MM;
    const bool live = lw < nl;
    T *mine = st + lw * Ns + r0;   // valid for rows r0 + k < N
    T x[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) x[k] = (live && r0 + k < N) ? mine[k] : T(0);

    if (has0) solve_refined<T, P, MM>(x, v0, ctx, r0);
    if (job.base) {
        // increment form: the solve produced x - base; add the base state
        __syncthreads();
        load_lines(static_cast<const T *>(job.base));
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (live && r0 + k < N) x[k] += mine[k];
    }
    if (hasb) {
        // explicit Crank-Nicolson operator along the line, then the second solve
        T left[P], right[P];
        neighbours<T, P, MM>(x, left, right, ctx);
        T y[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const T *a = brow + row_index(r0 + k, brm) * RS;
            T v = T(0);
#pragma unroll
            for (int j = 0; j < 2 * P + 1; ++j) v += a[j] * around<T, P, MM>(x, left, right, k + j - P);
            y[k] = v;
        }
        if (has1) solve_refined<T, P, MM>(y, v1, ctx, r0);
        if (job.add_after) {
#pragma unroll
            for (int k = 0; k < MM; ++k) x[k] += y[k];
        } else {
#pragma unroll
            for (int k = 0; k < MM; ++k) x[k] = y[k];
        }
    }

    __syncthreads();
    if (live) {
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (r0 + k < N) mine[k] = x[k];
    }
    __syncthreads();
    store_lines(static_cast<T *>(job.dst));
}

template <typename T, int P, int MM, bool DIRY>
__global__ __launch_bounds__((sweep_max_threads<T, P, MM>())) void k_sweep(SweepParams prm)
{
    sweep_body<T, P, MM, DIRY>(prm, xcd_remap(blockIdx.x, gridDim.x), blockIdx.y);
}

// Batched launch over the members of an ensemble: workgroup b works block
// info[b].y of member info[b].x (x < 0: no work), job blockIdx.y if the
// member has that many jobs.
template <typename T, int P, int MM, bool DIRY>
__global__ __launch_bounds__((sweep_max_threads<T, P, MM>())) void k_sweep_batch(
    const SweepParams *__restrict__ prms, const int2 *__restrict__ info)
{
    const int2 bi = info[xcd_remap(blockIdx.x, gridDim.x)];
    if (bi.x < 0) return;
    const SweepParams &prm = prms[bi.x];
    if ((int)blockIdx.y >= prm.njobs) return;
    sweep_body<T, P, MM, DIRY>(prm, bi.y, blockIdx.y);
}

using SweepFn = void (*)(SweepParams);
using SweepBatchFn = void (*)(const SweepParams *, const int2 *);

#define IGA_SWEEP_MMS(X) X(4) X(8) X(12) X(17)

template <typename T, int P> static SweepFn pick_mm(int mm, bool diry)
{
#define IGA_CASE(MM_) \
    if (mm == MM_) return diry ? k_sweep<T, P, MM_, true> : k_sweep<T, P, MM_, false>;
    IGA_SWEEP_MMS(IGA_CASE)
#undef IGA_CASE
    return nullptr;
}

template <typename T, int P> static SweepBatchFn pick_mm_batch(int mm, bool diry)
{
#define IGA_CASE(MM_) \
    if (mm == MM_) return diry ? k_sweep_batch<T, P, MM_, true> : k_sweep_batch<T, P, MM_, false>;
    IGA_SWEEP_MMS(IGA_CASE)
#undef IGA_CASE
    return nullptr;
}

SweepFn pick_sweep_f1(int mm, bool diry);
SweepFn pick_sweep_d1(int mm, bool diry);
SweepBatchFn pick_sweep_batch_f1(int mm, bool diry);
SweepBatchFn pick_sweep_batch_d1(int mm, bool diry);
SweepFn pick_sweep_f2(int mm, bool diry);
SweepFn pick_sweep_f3(int mm, bool diry);
SweepFn pick_sweep_d2(int mm, bool diry);
SweepFn pick_sweep_d3(int mm, bool diry);
SweepBatchFn pick_sweep_batch_f2(int mm, bool diry);
SweepBatchFn pick_sweep_batch_f3(int mm, bool diry);
SweepBatchFn pick_sweep_batch_d2(int mm, bool diry);
SweepBatchFn pick_sweep_batch_d3(int mm, bool diry);

}  // namespace iga
