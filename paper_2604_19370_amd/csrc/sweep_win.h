// sweep_win.h -- windowed batched banded line solves (truncated partition).
//
// Section 4's directional solves are independent banded LU solves per line.
// Here a workgroup owns W lines, each worked by WPL wavefronts; lane c of a
// line holds rows [c*MM, c*MM + MM) in registers, and the line is kept in LDS
// in two buffers (one in the compact form, WSweepParams) with H zero rows
// before and after it.  Forward substitution
// is a linear recurrence whose state contracts geometrically for these
// mass-dominated operators (the L and U factors of a banded Toeplitz-like
// matrix); restarting it from a zero state H rows before the chunk reproduces
// the exact state to below the plan's tolerance, H computed by the plan from
// the factors (products of the companion matrices).  So each lane:
//   forward:  runs its H warm-up rows (input values read from LDS), then its
//             own rows; publishes y to LDS;
//   backward: runs H warm-up rows of y after its chunk, then its own rows.
// No scan and no cross-lane arithmetic: lanes only meet in LDS, at barriers.
// Rows outside [0, N) are identity rows with zero data, so the line ends are
// exact.  FP32 plans refine once: x0 = LU32^{-1} b, r = b - A64 x0 in double,
// x = x0 + LU32^{-1} r (as in the exact kernels).  The correction solve runs
// a shorter warm-up Hc <= H: its result is a small correction, needed to a
// few bits only, and the first solve's truncation error is part of the
// residual it corrects.
//
// Coefficients come from strip tables in LDS (see WinGeom): each lane reads
// window row j of its table at base + j*RS, base fixed per lane, so the
// own-row loop uses compile-time offsets and no per-row index arithmetic.
#pragma once
#include "sweep_kernels.h"

namespace iga {

struct WinOpTab {
    const void *rows;     // [nrows][RS] factor windows (state precision)
    const double *a64;    // [anrows][RS] operator rows A(r, r-P .. r+P) (FP32 plans)
};
struct WinBandTab {
    const void *rows;     // [anrows][RS] band rows r-P .. r+P (state precision)
};

struct WSweepParams {
    SweepJob jobs[MAXJOBS];
    WinOpTab ops[NOPS];
    WinBandTab bands[NBANDS];
    WinGeom g;
    int N;        // line length
    int nlines;   // lines
    int ld;       // row stride of the field (Ny)
    int Lb;       // LDS stride of one line buffer: H + 64*WPL*MM + H (+1 if even)
    int W;        // lines per workgroup (power of two)
    int WPL;      // wavefronts per line
    int njobs;
    int compact;  // one line buffer per line (not two), and a second operator's
                  // tables staged over the first's once its solve is done
};

template <typename T, int P, int MM> struct WinLane {
    int r0;       // first row of the chunk
    int wb;       // base row of the factor window (row r0 - H)
    int ab;       // base row of the mm-row windows (row r0)
};

// forward substitution: Hr <= H warm-up rows from `in` (line buffer, row r at
// in[r]), then the lane's own rows in x; the factor window starts H rows
// before the chunk
template <typename T, int P, int MM>
__device__ __forceinline__ void wfwd(T (&x)[MM], const T *__restrict__ in, const T *__restrict__ tab,
                                     const WinLane<T, P, MM> &ln, int H, int Hr)
{
    constexpr int RS = RowStride<P>::RS;
    T s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = T(0);
    const T *d = in + ln.r0 - Hr;
    const T *c = tab + ((size_t)ln.wb + H - Hr) * RS;
    for (int j0 = 0; j0 < Hr; j0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T *L = c + (j0 + u) * RS;
            T y = d[j0 + u];
#pragma unroll
            for (int j = P - 1; j >= 0; --j) y -= L[j] * s[j];
#pragma unroll
            for (int j = P - 1; j > 0; --j) s[j] = s[j - 1];
            s[0] = y;
        }
    }
    const T *co = tab + ((size_t)ln.wb + H) * RS;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        const T *L = co + k * RS;
        T y = x[k];
#pragma unroll
        for (int j = P - 1; j >= 0; --j) y -= L[j] * s[j];
#pragma unroll
        for (int j = P - 1; j > 0; --j) s[j] = s[j - 1];
        s[0] = y;
        x[k] = y;
    }
}

// backward substitution: Hr <= H warm-up rows of y after the chunk from
// `in`, then the own rows
template <typename T, int P, int MM>
__device__ __forceinline__ void wbwd(T (&x)[MM], const T *__restrict__ in, const T *__restrict__ tab,
                                     const WinLane<T, P, MM> &ln, int H, int Hr)
{
    constexpr int RS = RowStride<P>::RS;
    T t[P];
#pragma unroll
    for (int j = 0; j < P; ++j) t[j] = T(0);
    const T *d = in + ln.r0 + MM;
    const T *c = tab + ((size_t)ln.wb + H + MM) * RS + P;
    for (int j0 = Hr - 4; j0 >= 0; j0 -= 4) {
#pragma unroll
        for (int u = 3; u >= 0; --u) {
            const T *U = c + (j0 + u) * RS;
            T v = d[j0 + u] * U[0];
#pragma unroll
            for (int j = P - 1; j >= 0; --j) v -= U[1 + j] * t[j];
#pragma unroll
            for (int j = P - 1; j > 0; --j) t[j] = t[j - 1];
            t[0] = v;
        }
    }
    const T *co = tab + ((size_t)ln.wb + H) * RS + P;
#pragma unroll
    for (int k = MM - 1; k >= 0; --k) {
        const T *U = co + k * RS;
        T v = x[k] * U[0];
#pragma unroll
        for (int j = P - 1; j >= 0; --j) v -= U[1 + j] * t[j];
#pragma unroll
        for (int j = P - 1; j > 0; --j) t[j] = t[j - 1];
        t[0] = v;
        x[k] = v;
    }
}

template <typename T, int MM>
__device__ __forceinline__ void publish(T *buf, const T (&x)[MM], int r0)
{
#pragma unroll
    for (int k = 0; k < MM; ++k) buf[r0 + k] = x[k];
}

// One factored solve, x <- A^{-1} x.  `in` holds x's values for every lane
// of the line (published, followed by a barrier); `tmp` is not being read.
// On return `tmp` holds y and is still being read by other lanes.
// With a single buffer (one: in == tmp) a barrier first lets every lane
// finish reading its warm-up rows before y overwrites them.
template <typename T, int P, int MM>
__device__ __forceinline__ void wsolve(T (&x)[MM], const T *in, T *tmp, const T *tab,
                                       const WinLane<T, P, MM> &ln, int H, int Hr, bool one)
{
    wfwd<T, P, MM>(x, in, tab, ln, H, Hr);
    if (one) __syncthreads();
    publish<T, MM>(tmp, x, ln.r0);
    __syncthreads();
    wbwd<T, P, MM>(x, tmp, tab, ln, H, Hr);
}

// x <- A^{-1} x with one FP64-residual refinement for FP32 plans.  Entry:
// `bin` holds x (published), `bout` not being read.  Exit: both buffers may
// still be read by other lanes (the caller synchronises before reuse).
// one (bin == bout, a single buffer): each publish waits for the readers of
// what it overwrites.
template <typename T, int P, int MM>
__device__ __forceinline__ void wsolve_refined(T (&x)[MM], T *bin, T *bout, const T *tab,
                                               const double *a64, const WinLane<T, P, MM> &ln,
                                               int H, int Hc, bool one)
{
    if constexpr (sizeof(T) == 8) {
        wsolve<T, P, MM>(x, bin, bout, tab, ln, H, H, one);
    } else {
        constexpr int RS = RowStride<P>::RS;
        T b[MM];
#pragma unroll
        for (int k = 0; k < MM; ++k) b[k] = x[k];
        wsolve<T, P, MM>(x, bin, bout, tab, ln, H, H, one);   // bin read (warm-up), bout = y
        // x0 -> bin: bin's last readers passed the barrier inside wsolve
        if (one) __syncthreads();
        publish<T, MM>(bin, x, ln.r0);
        __syncthreads();
        // residual b - A64 x0 in double (neighbour rows from bin), over a
        // sliding window of the 2P+1 rows r0 + k - P .. r0 + k + P, each
        // converted when it enters (not all MM + 2P at once: registers)
        const double *a = a64 + (size_t)ln.ab * RS;
        double w[2 * P + 1];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            w[i + 1] = (double)bin[ln.r0 - P + i];
            w[P + 1 + i] = (double)x[i];
        }
#pragma unroll
        for (int k = 0; k < MM; ++k) {
#pragma unroll
            for (int q = 0; q < 2 * P; ++q) w[q] = w[q + 1];
            T xn = k + P < MM ? x[k + P] : bin[ln.r0 + k + P];
            asm volatile("" : "+v"(xn));   // converted here, not hoisted
            w[2 * P] = (double)xn;
            double r = (double)b[k];
#pragma unroll
            for (int j = 0; j < 2 * P + 1; ++j) r -= a[k * RS + j] * w[j];
            b[k] = (T)r;
        }
        // r -> bout: bout's last readers (backward warm-up) passed the barrier above
        if (one) __syncthreads();
        publish<T, MM>(bout, b, ln.r0);
        __syncthreads();
        // correction: bin (x0) was last read by the residual, before that barrier
        wsolve<T, P, MM>(b, bout, bin, tab, ln, H, Hc, one);
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] += b[k];
    }
}

// One workgroup's work: W lines starting at line blk*W, job `jobi`.  NB:
// values of a line a thread loads at once (MM: all of them, see below).
// ONE: the compact form (WSweepParams::compact), chosen at compile time
// (as a run-time flag it made the compiler spill the chunk registers)
template <typename T, int P, int MM, bool DIRY, int NB, bool ONE>
__device__ __forceinline__ void wsweep_body(const WSweepParams &prm, const int blk, const int jobi)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RS = RowStride<P>::RS;
    constexpr bool F32 = sizeof(T) == 4;
    const SweepJob job = prm.jobs[jobi];
    const WinGeom &g = prm.g;
    const int H = g.H, Hc = g.Hc;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = prm.W, WPL = prm.WPL;
    const int wlog = __builtin_ctz(W);
    const int rstep = blockDim.x >> wlog;
    const int N = prm.N, Lb = prm.Lb, ld = prm.ld;
    const int line0 = blk * W;
    const int nl = min(W, prm.nlines - line0);
    const int lw = wave / WPL;
    const int part = wave - lw * WPL;

    // Stage W lines of a field into buffer `buf` (row r of line l at
    // buf[l*Lb + H + r]) and back.  A thread moves at most MM values of a
    // line (64*WPL*MM >= N), NB at a time, each batch's loads issued before
    // its stores: a staging costs MM/NB memory latencies.  Where the whole
    // chunk fits in flight (NB == MM), the input lines load while the tables
    // are staged, and the increment form's base state loads in one latency
    // after the solve (held through it, its registers cost occupancy more
    // than the latency costs).  y-lines: the WPL wavefronts of a line copy its contiguous run
    // of N values, 64 consecutive values per wavefront and instruction.
    // x-lines: rows of W consecutive columns; a workgroup slot past the last
    // line copies a live column into its own (unused) buffer.  Results use
    // write-back stores: x-line rows are W columns wide and L2 merges the
    // partial lines of neighbouring workgroups (streamed, they reached memory
    // unmerged); for y-lines streaming made no measurable difference.
    constexpr bool WHOLE = NB >= MM;
    const int jcol = tid & (W - 1), r00 = tid >> wlog;
    const int ystep = 64 * WPL;
#define IGA_YI0 const int yi0 = part * 64 + (threadIdx.x & 63);
    auto fetch_lines = [&](const T *src, T *v, int k0) {
        if constexpr (DIRY) {
            IGA_YI0
            const T *s = src + (size_t)(line0 + min(lw, nl - 1)) * ld;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int i = (k0 + k) * ystep + yi0;
                v[k] = (k0 + k < MM && i < N) ? s[i] : T(0);
            }
        } else {
            const T *s = src + line0 + min(jcol, nl - 1);
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int r = (k0 + k) * rstep + r00;
                v[k] = (k0 + k < MM && r < N) ? s[(size_t)r * ld] : T(0);
            }
        }
    };
    auto put_lines = [&](const T *v, T *buf, int k0) {
        if constexpr (DIRY) {
            IGA_YI0
            T *d = buf + (size_t)lw * Lb + H;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int i = (k0 + k) * ystep + yi0;
                if (k0 + k < MM && i < N) d[i] = v[k];
            }
        } else {
            T *d = buf + (size_t)jcol * Lb + H;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int r = (k0 + k) * rstep + r00;
                if (k0 + k < MM && r < N) d[r] = v[k];
            }
        }
    };
    auto load_lines = [&](const T *src, T *buf) {
#pragma unroll 1
        for (int k0 = 0; k0 < MM; k0 += NB) {
            T v[NB];
            fetch_lines(src, v, k0);
            put_lines(v, buf, k0);
        }
    };
    auto store_lines = [&](T *dst, const T *buf) {
#pragma unroll 1
        for (int k0 = 0; k0 < MM; k0 += NB) {
            T v[NB];
            if constexpr (DIRY) {
                if (lw < nl) {
                    IGA_YI0
                    const T *b = buf + (size_t)lw * Lb + H;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const int i = (k0 + k) * ystep + yi0;
                        v[k] = (k0 + k < MM && i < N) ? b[i] : T(0);
                    }
                    T *d = dst + (size_t)(line0 + lw) * ld;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const int i = (k0 + k) * ystep + yi0;
                        if (k0 + k < MM && i < N) d[i] = v[k];
                    }
                }
            } else {
                if (jcol < nl) {
                    const T *b = buf + (size_t)jcol * Lb + H;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const int r = (k0 + k) * rstep + r00;
                        v[k] = (k0 + k < MM && r < N) ? b[r] : T(0);
                    }
                    T *d = dst + line0 + jcol;
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        const int r = (k0 + k) * rstep + r00;
                        if (k0 + k < MM && r < N) d[(size_t)r * ld] = v[k];
                    }
                }
            }
        }
    };

#undef IGA_YI0
    T lv[NB];
    if (WHOLE) fetch_lines(static_cast<const T *>(job.src), lv, 0);

    // LDS: two line buffers [W][Lb] (row r of line l at H + l*Lb + r), or
    // one in the compact form, then the tables of this job
    constexpr bool one = ONE;
    const int nbuf = one ? 1 : 2;
    T *bufA = reinterpret_cast<T *>(smem);
    T *bufB = one ? bufA : bufA + (size_t)W * Lb;
    size_t off = ((size_t)nbuf * W * Lb * sizeof(T) + 15) & ~(size_t)15;
    auto take = [&](size_t bytes) {
        unsigned char *p = smem + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    const T *tab0 = nullptr, *tab1 = nullptr, *btab = nullptr;
    const double *a640 = nullptr, *a641 = nullptr;
    auto stage_op = [&](const WinOpTab &t, const T *&rows, const double *&a) {
        T *r = reinterpret_cast<T *>(take((size_t)g.nrows * RS * sizeof(T)));
        stage_table_dma<T>(r, t.rows, g.nrows * RS);
        rows = r;
        if (F32) {
            double *d = reinterpret_cast<double *>(take((size_t)g.anrows * RS * sizeof(double)));
            stage_table_dma<double>(d, t.a64, g.anrows * RS);
            a = d;
        }
    };
    const bool has0 = job.op0 >= 0, has1 = job.op1 >= 0, hasb = job.band >= 0;
    int *flag = reinterpret_cast<int *>(take(16));   // workgroup-wide "input not all zero"
    int *wnz = reinterpret_cast<int *>(take(64));    // the same per wavefront
    // A zero-skip job whose lines are all zero has nothing to do: the result
    // (zero, or the base it is added to) is already in dst.  With the whole
    // chunk in registers this is known before any table is staged.
    if (WHOLE && job.zero_skip) {
        bool nz = false;
#pragma unroll
        for (int k = 0; k < NB; ++k) nz = nz || lv[k] != T(0);
        const bool wz = __any(nz);
        if (lane == 0) wnz[wave] = wz ? 1 : 0;
        __syncthreads();
        int any = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) any |= wnz[w];
        if (!any) return;   // the same value for every thread of the workgroup
    }
    if (tid == 0) *flag = 0;
    // compact: a second operator reuses the first one's table space, staged
    // there once the first solve is done (both have the direction's window
    // geometry, so the same size)
    const size_t off_op0 = off;
    if (has0) stage_op(prm.ops[job.op0], tab0, a640);
    if (has1 && !(one && has0)) stage_op(prm.ops[job.op1], tab1, a641);
    if (hasb) {
        T *r = reinterpret_cast<T *>(take((size_t)g.anrows * RS * sizeof(T)));
        stage_table_dma<T>(r, prm.bands[job.band].rows, g.anrows * RS);
        btab = r;
    }
    // zero the pads of every line buffer: [0, H) and [H + N, Lb)
    for (int i = tid; i < nbuf * W * H; i += blockDim.x) {
        const int l = i / H, r = i - l * H;
        bufA[(size_t)l * Lb + r] = T(0);
    }
    const int tailn = Lb - H - N;
    for (int i = tid; i < nbuf * W * tailn; i += blockDim.x) {
        const int l = i / tailn, r = i - l * tailn;
        bufA[(size_t)l * Lb + H + N + r] = T(0);
    }

    // this lane's chunk and table windows
    const int c = part * 64 + lane;
    WinLane<T, P, MM> ln;
    ln.r0 = c * MM;
    if (c < g.nhead) {
        ln.wb = g.off_head + c * MM;
        ln.ab = g.aoff_head + c * MM;
    } else if (c >= g.tail1) {
        ln.wb = g.off_id;
        ln.ab = g.aoff_id;
    } else if (c >= g.tail0) {
        ln.wb = g.off_tail + (c - g.tail0) * MM;
        ln.ab = g.aoff_tail + (c - g.tail0) * MM;
    } else {
        ln.wb = g.off_canon;
        ln.ab = g.aoff_canon;
    }
    // slots beyond nl (the last workgroup) compute on their own, unused buffers
    T *A = bufA + (size_t)lw * Lb + H;
    T *B = bufB + (size_t)lw * Lb + H;
    const bool live = lw < nl;

    if (WHOLE)
        put_lines(lv, bufA, 0);
    else
        load_lines(static_cast<const T *>(job.src), bufA);
    __syncthreads();
    T x[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) x[k] = live ? A[ln.r0 + k] : T(0);
    if (!WHOLE && job.zero_skip) {
        // all-zero input lines: the result (zero, or the base it is added to)
        // is already in dst
        bool nz = false;
#pragma unroll
        for (int k = 0; k < MM; ++k) nz = nz || x[k] != T(0);
        if (__any(nz) && lane == 0) *flag = 1;
        __syncthreads();
        if (!*flag) return;   // the same value for every thread of the workgroup
    }
    // A: input published; B: free
    if (has0) {
        wsolve_refined<T, P, MM>(x, A, B, tab0, a640, ln, H, Hc, one);
        __syncthreads();
    }
    if (job.base) {
        // increment form: the solve produced x - base; add the base state
        // (one buffer without a solve: the lanes' reads of the input first)
        if (one && !has0) __syncthreads();
        if (WHOLE) {
            fetch_lines(static_cast<const T *>(job.base), lv, 0);
            put_lines(lv, bufB, 0);
        } else {
            load_lines(static_cast<const T *>(job.base), bufB);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MM; ++k) x[k] += live ? B[ln.r0 + k] : T(0);
        __syncthreads();
    }
    if (hasb) {
        // explicit Crank-Nicolson operator along the line, then the second solve
        if (one && has0 && has1) {
            // the first operator's tables were last read before the barrier
            // that ended its solve; the barrier below makes these visible
            off = off_op0;
            stage_op(prm.ops[job.op1], tab1, a641);
        }
        publish<T, MM>(A, x, ln.r0);
        __syncthreads();
        T xd[MM + 2 * P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            xd[i] = A[ln.r0 - P + i];
            xd[MM + P + i] = A[ln.r0 + MM + i];
        }
#pragma unroll
        for (int k = 0; k < MM; ++k) xd[P + k] = x[k];
        T y[MM];
        const T *bt = btab + (size_t)ln.ab * RS;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            T v = T(0);
#pragma unroll
            for (int j = 0; j < 2 * P + 1; ++j) v += bt[k * RS + j] * xd[k + j];
            y[k] = v;
        }
        // y -> B (free since the last barrier; one buffer: once every lane
        // has read its neighbours' rows of x), then solve with A as scratch
        if (one) __syncthreads();
        publish<T, MM>(B, y, ln.r0);
        __syncthreads();
        if (has1) {
            wsolve_refined<T, P, MM>(y, B, A, tab1, a641, ln, H, Hc, one);
            __syncthreads();
        }
        if (job.add_after) {
#pragma unroll
            for (int k = 0; k < MM; ++k) x[k] += y[k];
        } else {
#pragma unroll
            for (int k = 0; k < MM; ++k) x[k] = y[k];
        }
    }
    if (live) publish<T, MM>(A, x, ln.r0);
    __syncthreads();
    store_lines(static_cast<T *>(job.dst), bufA);
}

// workgroup size bound: 16 wavefronts, or 8 for large windows, which need
// more than 128 registers per lane
template <typename T, int P, int MM> constexpr int wsweep_max_threads()
{
    return (MM >= 25 || (sizeof(T) == 8 && MM >= 17)) ? 512 : 1024;
}

// Values in flight per thread when lines are staged: the whole chunk where
// the registers hold it without spilling (checked per variant against the
// compiler's resource report), else batches of four.  The batched-launch
// form carries more state and gets the smaller budget.
template <typename T, int P, int MM, bool BATCH> constexpr int wsweep_nb()
{
    if (wsweep_max_threads<T, P, MM>() == 512) return MM;   // 256 registers
    const int bytes = MM * (int)sizeof(T);
    const int fits = BATCH ? 36 : (P <= 2 ? 68 : 36);
    return bytes <= fits ? MM : 4;
}

template <typename T, int P, int MM, bool DIRY, bool ONE>
__global__ __launch_bounds__((wsweep_max_threads<T, P, MM>())) void k_wsweep(WSweepParams prm)
{
    wsweep_body<T, P, MM, DIRY, wsweep_nb<T, P, MM, false>(), ONE>(prm, xcd_remap(blockIdx.x, gridDim.x),
                                                                   blockIdx.y);
}

template <typename T, int P, int MM, bool DIRY, bool ONE>
__global__ __launch_bounds__((wsweep_max_threads<T, P, MM>())) void k_wsweep_batch(
    const WSweepParams *__restrict__ prms, const int2 *__restrict__ info)
{
    const int2 bi = info[xcd_remap(blockIdx.x, gridDim.x)];
    if (bi.x < 0) return;
    const WSweepParams &prm = prms[bi.x];
    if ((int)blockIdx.y >= prm.njobs) return;
    wsweep_body<T, P, MM, DIRY, wsweep_nb<T, P, MM, true>(), ONE>(prm, bi.y, blockIdx.y);
}

using WSweepFn = void (*)(WSweepParams);
using WSweepBatchFn = void (*)(const WSweepParams *, const int2 *);

#define IGA_WSWEEP_MMS(X) X(9) X(13) X(17) X(25) X(33)

template <typename T, int P> static WSweepFn pick_wmm(int mm, bool diry, bool one)
{
#define IGA_CASE(MM_)                                                                          \
    if (mm == MM_)                                                                             \
        return diry ? (one ? k_wsweep<T, P, MM_, true, true> : k_wsweep<T, P, MM_, true, false>) \
                    : (one ? k_wsweep<T, P, MM_, false, true> : k_wsweep<T, P, MM_, false, false>);
    IGA_WSWEEP_MMS(IGA_CASE)
#undef IGA_CASE
    return nullptr;
}

template <typename T, int P> static WSweepBatchFn pick_wmm_batch(int mm, bool diry, bool one)
{
#define IGA_CASE(MM_)                                                                     \
    if (mm == MM_)                                                                        \
        return diry ? (one ? k_wsweep_batch<T, P, MM_, true, true>                        \
                           : k_wsweep_batch<T, P, MM_, true, false>)                      \
                    : (one ? k_wsweep_batch<T, P, MM_, false, true>                       \
                           : k_wsweep_batch<T, P, MM_, false, false>);
    IGA_WSWEEP_MMS(IGA_CASE)
#undef IGA_CASE
    return nullptr;
}

WSweepFn pick_wsweep_f1(int mm, bool diry, bool one);
WSweepFn pick_wsweep_d1(int mm, bool diry, bool one);
WSweepBatchFn pick_wsweep_batch_f1(int mm, bool diry, bool one);
WSweepBatchFn pick_wsweep_batch_d1(int mm, bool diry, bool one);
WSweepFn pick_wsweep_f2(int mm, bool diry, bool one);
WSweepFn pick_wsweep_f3(int mm, bool diry, bool one);
WSweepFn pick_wsweep_d2(int mm, bool diry, bool one);
WSweepFn pick_wsweep_d3(int mm, bool diry, bool one);
WSweepBatchFn pick_wsweep_batch_f2(int mm, bool diry, bool one);
WSweepBatchFn pick_wsweep_batch_f3(int mm, bool diry, bool one);
WSweepBatchFn pick_wsweep_batch_d2(int mm, bool diry, bool one);
WSweepBatchFn pick_wsweep_batch_d3(int mm, bool diry, bool one);

}  // namespace iga
