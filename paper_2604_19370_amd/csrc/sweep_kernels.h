// sweep_kernels.h -- batched banded line solves of the Kronecker-factored
// systems (Section 4: N_y independent solves of size N_x for an x substep,
// N_x of size N_y for a y substep), one wavefront per line.
//
// A workgroup of W wavefronts owns W consecutive lines.  It stages them in LDS
// with coalesced loads (rows of W consecutive columns for x-lines, W whole
// contiguous rows for y-lines), and wavefront w solves line w: lane c holds
// rows [c*m, c*m + m) of the line in registers (64 chunks per line).
//
// Forward and backward substitution are linear recurrences with a p-vector
// state, affine over a chunk: s_out = Phi_c s_in + psi_c(b).  Each lane runs
// its chunk from a zero state, the 64 chunk end-states are combined by a
// Hillis-Steele scan across the wavefront's lanes (shuffles, no barriers)
// whose matrix parts -- products of the rows' companion matrices, which do not
// depend on the data -- start from each chunk's precomputed transfer matrix and
// are composed along the scan, and each lane re-runs its chunk from its exact
// incoming state.  The result is the banded
// LU solve of the whole line.
//
// Every lane holds exactly mm rows: a line of N rows is padded to 64*mm rows
// with identity rows (no multipliers, unit pivot, zero data), which leaves the
// LU solve of the real rows unchanged and keeps the recurrences free of
// per-row predication.
//
// Coefficients.  Interior rows of a factored operator on a uniform mesh agree
// to rounding (the LU of a banded Toeplitz matrix converges to a constant row
// within a few tens of rows); the plan keeps rows [0, K0) and [NK, N) as they
// are and one canonical row for [K0, NK), in LDS, so lanes on interior chunks
// all read the same address.
//
// FP32 plans: every solve is x0 = LU32^{-1} b, r = b - A64 x0 formed in double,
// x = x0 + LU32^{-1} r (one step of iterative refinement), and the state is
// advanced in increment form (the job adds the base field after the solve).
#pragma once
#include "iga_internal.h"

namespace iga {

constexpr int MAXJOBS = 4;
constexpr int SCAN_LEVELS = 6;   // 64 chunks per line

// compressed coefficient rows (device, state precision unless noted)
struct OpTab {
    const void *rows;     // [nrows][RS] : L(r, r-1-j) j<P, 1/U(r,r), U(r,r+1+j)/U(r,r)
    const double *a64;    // [nrows][RS] : A(r, r-P .. r+P) in double
    const void *tf, *tb;  // [64][P*P] forward / backward transfer matrix of each chunk
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
    int m;        // rows per chunk
    int Ns;       // LDS stride between staged lines
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

// Scan of the chunk end-states across the 64 lanes: a Hillis-Steele scan of
// the affine chunk maps (Phi_c, psi_c), composing the matrices as it goes, so
// only each chunk's own transfer matrix is needed.  On exit v is the state
// entering this lane's chunk from the left (FWD) or from the right.
template <typename T, int P, bool FWD>
__device__ __forceinline__ void wave_scan(T (&v)[P], int lane, const T *__restrict__ tab)
{
    constexpr int PP = P * P;
    T F[PP];
#pragma unroll
    for (int i = 0; i < PP; ++i) F[i] = tab[lane * PP + i];
#pragma unroll
    for (int d = 0; d < SCAN_LEVELS; ++d) {
        const int off = 1 << d;
        T o[P], oF[PP];
#pragma unroll
        for (int j = 0; j < P; ++j) o[j] = FWD ? shfl_up(v[j], off) : shfl_down(v[j], off);
#pragma unroll
        for (int i = 0; i < PP; ++i) oF[i] = FWD ? shfl_up(F[i], off) : shfl_down(F[i], off);
        const bool has = FWD ? lane >= off : lane + off < 64;
        if (has) {
            T nF[PP];
#pragma unroll
            for (int i = 0; i < P; ++i) {
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    v[i] += F[i * P + j] * o[j];
                    T s = T(0);
#pragma unroll
                    for (int k = 0; k < P; ++k) s += F[i * P + k] * oF[k * P + j];
                    nF[i * P + j] = s;
                }
            }
#pragma unroll
            for (int i = 0; i < PP; ++i) F[i] = nF[i];
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const T o = FWD ? shfl_up(v[j], 1) : shfl_down(v[j], 1);
        v[j] = (FWD ? lane > 0 : lane < 63) ? o : T(0);
    }
}

template <typename T, int P, int MM>
__device__ __forceinline__ void chunk_solve(T (&x)[MM], const T *rows, const T *tf, const T *tb,
                                            const RowMap &rm, int lane, int r0)
{
    T s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    fwd<T, P, MM, false>(x, r0, rows, rm, s);
    wave_scan<T, P, true>(s, lane, tf);
    fwd<T, P, MM, true>(x, r0, rows, rm, s);
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    bwd<T, P, MM, false>(x, r0, rows, rm, s);
    wave_scan<T, P, false>(s, lane, tb);
    bwd<T, P, MM, true>(x, r0, rows, rm, s);
}

// Values of the line at rows r0-P .. r0+MM+P-1 as seen from this chunk:
// xe[P + k] = x[k], the neighbouring chunks' values beyond.
template <typename T, int P, int MM>
__device__ __forceinline__ void neighbours(const T (&x)[MM], T (&xe)[MM + 2 * P], int lane)
{
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const T left = shfl_up(x[MM - P + i], 1);
        const T right = shfl_down(x[i], 1);
        xe[i] = lane > 0 ? left : T(0);
        xe[P + MM + i] = lane < 63 ? right : T(0);
    }
#pragma unroll
    for (int k = 0; k < MM; ++k) xe[P + k] = x[k];
}

// One operator's tables as the kernel sees them (rows in LDS).
template <typename T> struct OpView {
    const T *rows;
    const double *a64;
    const T *tf, *tb;
    RowMap rm;
};

template <typename T, int P, int MM>
__device__ __forceinline__ void solve_refined(T (&x)[MM], const OpView<T> &op, int lane, int r0)
{
    if constexpr (sizeof(T) == 8) {
        chunk_solve<T, P, MM>(x, op.rows, op.tf, op.tb, op.rm, lane, r0);
    } else {
        constexpr int RS = RowStride<P>::RS;
        T b[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) b[k] = x[k];
        chunk_solve<T, P, MM>(x, op.rows, op.tf, op.tb, op.rm, lane, r0);
        T xe[MM + 2 * P];
        neighbours<T, P, MM>(x, xe, lane);
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const double *a = op.a64 + row_index(r0 + k, op.rm) * RS;
            double r = (double)b[k];
#pragma unroll
            for (int j = 0; j < 2 * P + 1; ++j) r -= a[j] * (double)xe[k + j];
            b[k] = (T)r;
        }
        chunk_solve<T, P, MM>(b, op.rows, op.tf, op.tb, op.rm, lane, r0);
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] += b[k];
    }
}

// copy `n` elements of type U from global to LDS with the whole workgroup
// (four loads in flight per thread)
template <typename U>
__device__ __forceinline__ void stage_table(U *dst, const void *src, int n)
{
    const U *s = static_cast<const U *>(src);
    for (int b0 = 0; b0 < n; b0 += 4 * blockDim.x) {
        U v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = b0 + u * blockDim.x + threadIdx.x;
            v[u] = i < n ? s[i] : U(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = b0 + u * blockDim.x + threadIdx.x;
            if (i < n) dst[i] = v[u];
        }
    }
}

template <int MM> struct SweepBounds {
    static constexpr int value = MM <= 17 ? 1024 : (MM <= 33 ? 512 : 256);
};

template <typename T, int P, int MM, bool DIRY>
__global__ __launch_bounds__(SweepBounds<MM>::value) void k_sweep(SweepParams prm)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RS = RowStride<P>::RS;
    constexpr int SCAN = 64 * P * P;                  // chunk transfer matrices per direction
    constexpr bool F32 = sizeof(T) == 4;
    const SweepJob job = prm.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = blockDim.x >> 6;            // lines per workgroup (power of two)
    const int wlog = __builtin_ctz(W);
    const int rstep = blockDim.x >> wlog;
    const int N = prm.N, Ns = prm.Ns, ld = prm.ld;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int line0 = blk * W;
    const int nl = min(W, prm.nlines - line0);

    // LDS: staged lines, then the tables of this job (coefficient rows, the
    // refinement operator rows, the chunk scan tables, the explicit band)
    T *st = reinterpret_cast<T *>(smem);
    size_t off = ((size_t)W * Ns * sizeof(T) + 15) & ~(size_t)15;
    auto take = [&](size_t bytes) {
        unsigned char *p = smem + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    auto stage_op = [&](const OpTab &t, OpView<T> &v) {
        T *rows = reinterpret_cast<T *>(take((size_t)t.nrows * RS * sizeof(T)));
        stage_table<T>(rows, t.rows, t.nrows * RS);
        v.rows = rows;
        v.a64 = nullptr;
        if (F32) {
            double *a = reinterpret_cast<double *>(take((size_t)t.nrows * RS * sizeof(double)));
            stage_table<double>(a, t.a64, t.nrows * RS);
            v.a64 = a;
        }
        T *tf = reinterpret_cast<T *>(take((size_t)SCAN * sizeof(T)));
        T *tb = reinterpret_cast<T *>(take((size_t)SCAN * sizeof(T)));
        stage_table<T>(tf, t.tf, SCAN);
        stage_table<T>(tb, t.tb, SCAN);
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
        stage_table<T>(rows, t.rows, t.nrows * RS);
        brow = rows;
        brm = RowMap{t.K0, t.NK - 1, t.nrows - 1};
    }

    // Stage W lines of a field (src layout) into st, and back.  Loads are
    // issued in batches of UNR per thread before their LDS stores so that
    // their latencies overlap.  y-lines: the W rows are one contiguous block,
    // copied flat (Ns == N).  x-lines: rows of W consecutive columns.
    constexpr int UNR = 8;
    auto load_lines = [&](const T *src) {
        if constexpr (DIRY) {
            const T *s = src + (size_t)line0 * ld;
            const int tot = nl * N;
            for (int b0 = 0; b0 < tot; b0 += UNR * blockDim.x) {
                T v[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int e = b0 + u * blockDim.x + tid;
                    v[u] = e < tot ? s[e] : T(0);
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int e = b0 + u * blockDim.x + tid;
                    if (e < tot) st[e] = v[u];
                }
            }
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

    load_lines(static_cast<const T *>(job.src));
    __syncthreads();

    // lane's chunk: rows [r0, r0 + MM) of line `wave`; rows >= N are padding
    const int r0 = lane * MM;
    const bool live = wave < nl;
    const T *mine = st + wave * Ns;
    T x[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) x[k] = (live && r0 + k < N) ? mine[r0 + k] : T(0);
    __syncthreads();

    if (has0) solve_refined<T, P, MM>(x, v0, lane, r0);
    if (job.base) {
        // increment form: the solve produced x - base; add the base state
        load_lines(static_cast<const T *>(job.base));
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (live && r0 + k < N) x[k] += mine[r0 + k];
        __syncthreads();
    }
    if (hasb) {
        // explicit Crank-Nicolson operator along the line, then the second solve
        T xe[MM + 2 * P];
        neighbours<T, P, MM>(x, xe, lane);
        T y[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const T *a = brow + row_index(r0 + k, brm) * RS;
            T v = T(0);
#pragma unroll
            for (int j = 0; j < 2 * P + 1; ++j) v += a[j] * xe[k + j];
            y[k] = v;
        }
        if (has1) solve_refined<T, P, MM>(y, v1, lane, r0);
        if (job.add_after) {
#pragma unroll
            for (int k = 0; k < MM; ++k) x[k] += y[k];
        } else {
#pragma unroll
            for (int k = 0; k < MM; ++k) x[k] = y[k];
        }
    }

#pragma unroll
    for (int k = 0; k < MM; ++k)
        if (live && r0 + k < N) st[wave * Ns + r0 + k] = x[k];
    __syncthreads();
    store_lines(static_cast<T *>(job.dst));
}

using SweepFn = void (*)(SweepParams);

#define IGA_SWEEP_MMS(X) X(4) X(8) X(12) X(17) X(33) X(48) X(65)

template <typename T, int P> static SweepFn pick_mm(int mm, bool diry)
{
#define IGA_CASE(MM_) \
    if (mm == MM_) return diry ? k_sweep<T, P, MM_, true> : k_sweep<T, P, MM_, false>;
    IGA_SWEEP_MMS(IGA_CASE)
#undef IGA_CASE
    return nullptr;
}

SweepFn pick_sweep_f2(int mm, bool diry);
SweepFn pick_sweep_f3(int mm, bool diry);
SweepFn pick_sweep_d2(int mm, bool diry);
SweepFn pick_sweep_d3(int mm, bool diry);

}  // namespace iga
