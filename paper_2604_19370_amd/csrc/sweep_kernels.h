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
// depend on the data -- come precomputed per (level, lane), and each lane
// re-runs its chunk from its exact incoming state.  The result is the banded
// LU solve of the whole line.
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
    const void *tf, *tb;  // [6][64][P*P] chunk scan tables
    int K0, NK, nrows;
};
struct BandTab {
    const void *rows;     // [nrows][RS] : band row r-P .. r+P
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

__device__ __forceinline__ int row_index(int r, int K0, int NK)
{
    return r < K0 ? r : (r >= NK ? K0 + 1 + (r - NK) : K0);
}

template <typename T> __device__ __forceinline__ T shfl_up(T v, int d) { return __shfl_up(v, d, 64); }
template <typename T> __device__ __forceinline__ T shfl_down(T v, int d) { return __shfl_down(v, d, 64); }

// forward substitution over the chunk; s = state (y_{r-1}, y_{r-2}, ...)
template <typename T, int P, int MM, bool WRITE>
__device__ __forceinline__ void fwd(T (&x)[MM], int len, int r0, const T *rows, int K0, int NK,
                                    T (&s)[P])
{
    constexpr int RS = RowStride<P>::RS;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        if (k < len) {
            const T *L = rows + row_index(r0 + k, K0, NK) * RS;
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

// backward substitution over the chunk; t = state (x_{r+1}, x_{r+2}, ...)
template <typename T, int P, int MM, bool WRITE>
__device__ __forceinline__ void bwd(T (&x)[MM], int len, int r0, const T *rows, int K0, int NK,
                                    T (&t)[P])
{
    constexpr int RS = RowStride<P>::RS;
#pragma unroll
    for (int k = MM - 1; k >= 0; --k) {
        if (k < len) {
            const T *U = rows + row_index(r0 + k, K0, NK) * RS + P;
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

// Scan of the chunk end-states across the 64 lanes; on exit v is the state
// entering this lane's chunk from the left (FWD) or from the right.
template <typename T, int P, bool FWD>
__device__ __forceinline__ void wave_scan(T (&v)[P], int lane, const T *__restrict__ tab)
{
    constexpr int PP = P * P;
#pragma unroll
    for (int d = 0; d < SCAN_LEVELS; ++d) {
        const int off = 1 << d;
        T o[P];
#pragma unroll
        for (int j = 0; j < P; ++j) o[j] = FWD ? shfl_up(v[j], off) : shfl_down(v[j], off);
        const bool has = FWD ? lane >= off : lane + off < 64;
        const T *Mt = tab + (d * 64 + lane) * PP;
        T Mv[PP];
#pragma unroll
        for (int i = 0; i < PP; ++i) Mv[i] = Mt[i];
        if (has) {
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
                for (int j = 0; j < P; ++j) v[i] += Mv[i * P + j] * o[j];
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const T o = FWD ? shfl_up(v[j], 1) : shfl_down(v[j], 1);
        v[j] = (FWD ? lane > 0 : lane < 63) ? o : T(0);
    }
}

template <typename T, int P, int MM>
__device__ __forceinline__ void chunk_solve(T (&x)[MM], const OpTab &op, const T *rows, int lane,
                                            int r0, int len)
{
    T s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    fwd<T, P, MM, false>(x, len, r0, rows, op.K0, op.NK, s);
    wave_scan<T, P, true>(s, lane, static_cast<const T *>(op.tf));
    fwd<T, P, MM, true>(x, len, r0, rows, op.K0, op.NK, s);
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    bwd<T, P, MM, false>(x, len, r0, rows, op.K0, op.NK, s);
    wave_scan<T, P, false>(s, lane, static_cast<const T *>(op.tb));
    bwd<T, P, MM, true>(x, len, r0, rows, op.K0, op.NK, s);
}

// Values of the line at rows r0-P .. r0+MM+P-1 as seen from this chunk:
// xe[P + k] = x[k] for k < len, the neighbouring chunks' values beyond.
template <typename T, int P, int MM>
__device__ __forceinline__ void neighbours(const T (&x)[MM], T (&xe)[MM + 2 * P], int len)
{
    T first[P], last[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        first[i] = x[i];
        last[i] = T(0);
    }
#pragma unroll
    for (int k = 0; k < MM; ++k)
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (k == len - P + i) last[i] = x[k];
    T left[P], right[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        left[i] = shfl_up(last[i], 1);    // lane 0 receives its own: rows < 0 have no coefficients
        right[i] = shfl_down(first[i], 1);
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < P; ++i) xe[i] = lane > 0 ? left[i] : T(0);
#pragma unroll
    for (int k = 0; k < MM + P; ++k) {
        T v = (k < MM) ? x[k < MM ? k : 0] : T(0);
        if (k >= len) v = T(0);
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (k == len + i && lane < 63) v = right[i];
        xe[P + k] = v;
    }
}

template <typename T, int P, int MM>
__device__ __forceinline__ void solve_refined(T (&x)[MM], const OpTab &op, const T *rows,
                                              const double *a64, int lane, int r0, int len)
{
    if constexpr (sizeof(T) == 8) {
        chunk_solve<T, P, MM>(x, op, rows, lane, r0, len);
    } else {
        constexpr int RS = RowStride<P>::RS;
        T b[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) b[k] = x[k];
        chunk_solve<T, P, MM>(x, op, rows, lane, r0, len);
        T xe[MM + 2 * P];
        neighbours<T, P, MM>(x, xe, len);
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            if (k < len) {
                const double *a = a64 + row_index(r0 + k, op.K0, op.NK) * RS;
                double r = (double)b[k];
#pragma unroll
                for (int j = 0; j < 2 * P + 1; ++j) r -= a[j] * (double)xe[k + j];
                b[k] = (T)r;
            }
        }
        chunk_solve<T, P, MM>(b, op, rows, lane, r0, len);
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] += b[k];
    }
}

// copy `n` elements of type U from global to LDS with the whole workgroup
template <typename U>
__device__ __forceinline__ void stage_table(U *dst, const void *src, int n)
{
    const U *s = static_cast<const U *>(src);
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = s[i];
}

template <int MM> struct SweepBounds {
    static constexpr int value = MM <= 17 ? 1024 : (MM <= 33 ? 512 : 256);
};

template <typename T, int P, int MM, bool DIRY>
__global__ __launch_bounds__(SweepBounds<MM>::value) void k_sweep(SweepParams prm)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RS = RowStride<P>::RS;
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

    // LDS: staged lines, then the coefficient tables of this job
    T *st = reinterpret_cast<T *>(smem);
    size_t off = ((size_t)W * Ns * sizeof(T) + 15) & ~(size_t)15;
    const OpTab *op0 = job.op0 >= 0 ? &prm.ops[job.op0] : nullptr;
    const OpTab *op1 = job.op1 >= 0 ? &prm.ops[job.op1] : nullptr;
    const BandTab *bd = job.band >= 0 ? &prm.bands[job.band] : nullptr;
    T *r0t = nullptr, *r1t = nullptr, *rbt = nullptr;
    double *a0t = nullptr, *a1t = nullptr;
    constexpr bool F32 = sizeof(T) == 4;
    if (op0) {
        r0t = reinterpret_cast<T *>(smem + off);
        off += ((size_t)op0->nrows * RS * sizeof(T) + 15) & ~(size_t)15;
        stage_table<T>(r0t, op0->rows, op0->nrows * RS);
        if (F32) {
            a0t = reinterpret_cast<double *>(smem + off);
            off += (size_t)op0->nrows * RS * sizeof(double);
            stage_table<double>(a0t, op0->a64, op0->nrows * RS);
        }
    }
    if (op1) {
        r1t = reinterpret_cast<T *>(smem + off);
        off += ((size_t)op1->nrows * RS * sizeof(T) + 15) & ~(size_t)15;
        stage_table<T>(r1t, op1->rows, op1->nrows * RS);
        if (F32) {
            a1t = reinterpret_cast<double *>(smem + off);
            off += (size_t)op1->nrows * RS * sizeof(double);
            stage_table<double>(a1t, op1->a64, op1->nrows * RS);
        }
    }
    if (bd) {
        rbt = reinterpret_cast<T *>(smem + off);
        off += ((size_t)bd->nrows * RS * sizeof(T) + 15) & ~(size_t)15;
        stage_table<T>(rbt, bd->rows, bd->nrows * RS);
    }

    // stage W lines of a field (src layout) into st, and back
    auto load_lines = [&](const T *src) {
        if constexpr (DIRY) {
            for (int i = 0; i < nl; ++i) {
                const T *s = src + (size_t)(line0 + i) * ld;
                for (int r = tid; r < N; r += blockDim.x) st[i * Ns + r] = s[r];
            }
        } else {
            const int j = tid & (W - 1);
            for (int r = tid >> wlog; r < N; r += rstep)
                if (j < nl) st[j * Ns + r] = src[(size_t)r * ld + line0 + j];
        }
    };
    auto store_lines = [&](T *dst) {
        if constexpr (DIRY) {
            for (int i = 0; i < nl; ++i) {
                T *d = dst + (size_t)(line0 + i) * ld;
                for (int r = tid; r < N; r += blockDim.x) d[r] = st[i * Ns + r];
            }
        } else {
            const int j = tid & (W - 1);
            for (int r = tid >> wlog; r < N; r += rstep)
                if (j < nl) dst[(size_t)r * ld + line0 + j] = st[j * Ns + r];
        }
    };

    load_lines(static_cast<const T *>(job.src));
    __syncthreads();

    const int m = prm.m;
    const int r0 = lane * m;
    int len = N - r0;
    len = len < 0 ? 0 : (len > m ? m : len);
    if (wave >= nl) len = 0;
    T x[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) x[k] = (k < len) ? st[wave * Ns + r0 + k] : T(0);
    __syncthreads();

    if (op0) solve_refined<T, P, MM>(x, *op0, r0t, a0t, lane, r0, len);
    if (job.base) {
        // increment form: the solve produced x - base; add the base state
        load_lines(static_cast<const T *>(job.base));
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MM; ++k)
            if (k < len) x[k] += st[wave * Ns + r0 + k];
        __syncthreads();
    }
    if (bd) {
        // explicit Crank-Nicolson operator along the line, then the second solve
        T xe[MM + 2 * P];
        neighbours<T, P, MM>(x, xe, len);
        T y[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            y[k] = T(0);
            if (k < len) {
                const T *a = rbt + row_index(r0 + k, bd->K0, bd->NK) * RS;
                T v = T(0);
#pragma unroll
                for (int j = 0; j < 2 * P + 1; ++j) v += a[j] * xe[k + j];
                y[k] = v;
            }
        }
        if (op1) solve_refined<T, P, MM>(y, *op1, r1t, a1t, lane, r0, len);
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
        if (k < len) st[wave * Ns + r0 + k] = x[k];
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
