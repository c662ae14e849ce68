// sample.hip -- diagnostics on a state, outside the time step:
//  - the spline value sum_ij C_ij B_i(x) B_j(y) at a tensor grid of points
//    (to compare fields at sample points, e.g. a 256^2 grid);
//  - the number of quadrature points whose ignition decision
//    [T > T_ig and fuel > thr] lies within (dT, dF) of its thresholds, the
//    points where two correct evaluations in different precisions may decide
//    differently.
// Both evaluate the basis in double with the Cox-de Boor recurrence on the
// plan's uniform open knot vector (Section 3.1), one thread per output.
#include "iga_internal.h"

namespace iga {

struct SampleAxis {
    int nel, p;
    double h, L;
};

// Knot k of the uniform open knot vector (p + 1 repeated end knots).
__device__ __forceinline__ double knot(const SampleAxis &a, int k)
{
    const int e = min(max(k - a.p, 0), a.nel);
    return e == a.nel ? a.L : e * a.h;
}

// Element containing x (clamped to the domain) and the p + 1 basis
// functions that are nonzero there, B_{e}, ..., B_{e+p}.
__device__ __forceinline__ int basis_at(const SampleAxis &a, double x, double (&N)[4])
{
    x = fmin(fmax(x, 0.0), a.L);
    int e = (int)floor(x / a.h);
    e = min(max(e, 0), a.nel - 1);
    const int s = e + a.p;   // knot span [t_s, t_{s+1})
    double left[4], right[4];
    N[0] = 1.0;
    for (int j = 1; j <= a.p; ++j) {
        left[j] = x - knot(a, s + 1 - j);
        right[j] = knot(a, s + j) - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            const double t = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * t;
            saved = left[j - r] * t;
        }
        N[j] = saved;
    }
    return e;
}

template <typename T>
__global__ void k_sample(const T *__restrict__ C, int Ny, SampleAxis ax, SampleAxis ay,
                         const double *__restrict__ xs, int nx, const double *__restrict__ ys,
                         int ny, double *__restrict__ out)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)nx * ny) return;
    const int a = (int)(k / ny), b = (int)(k % ny);
    double bx[4], by[4];
    const int ex = basis_at(ax, xs[a], bx);
    const int ey = basis_at(ay, ys[b], by);
    double s = 0.0;
    for (int i = 0; i <= ax.p; ++i) {
        double r = 0.0;
        for (int j = 0; j <= ay.p; ++j) r += (double)C[(size_t)(ex + i) * Ny + ey + j] * by[j];
        s += r * bx[i];
    }
    out[k] = s;
}

struct AmbParams {
    SampleAxis ax, ay;
    int Ny, nq;
    double g[4];   // Gauss nodes on [0, 1]
    double t_ig, thr, dT, dF;
};

__global__ void k_zero_count(unsigned long long *c) { *c = 0ull; }

template <typename T>
__global__ void k_ambiguous(const T *__restrict__ S, const T *__restrict__ F, AmbParams a,
                            unsigned long long *__restrict__ count)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nel = (long long)a.ax.nel * a.ay.nel;
    unsigned n = 0;
    if (k < nel) {
        const int ex = (int)(k / a.ay.nel), ey = (int)(k % a.ay.nel);
        for (int qx = 0; qx < a.nq; ++qx) {
            double bx[4], by[4];
            const int cx = basis_at(a.ax, (ex + a.g[qx]) * a.ax.h, bx);
            for (int qy = 0; qy < a.nq; ++qy) {
                const int cy = basis_at(a.ay, (ey + a.g[qy]) * a.ay.h, by);
                double s = 0.0, f = 0.0;
                for (int i = 0; i <= a.ax.p; ++i)
                    for (int j = 0; j <= a.ay.p; ++j) {
                        const size_t idx = (size_t)(cx + i) * a.Ny + cy + j;
                        s += (double)S[idx] * bx[i] * by[j];
                        f += (double)F[idx] * bx[i] * by[j];
                    }
                const bool near_t = fabs(s - a.t_ig) <= a.dT && f > a.thr - a.dF;
                const bool near_f = fabs(f - a.thr) <= a.dF && s > a.t_ig - a.dT;
                n += (near_t || near_f) ? 1u : 0u;
            }
        }
    }
    // one atomic per wavefront
    for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off, 64);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, (unsigned long long)n);
}

static SampleAxis axis_of(const DirHost &D, int p) { return SampleAxis{D.n, p, D.h, D.L}; }

}  // namespace iga

using namespace iga;

extern "C" iga_status iga_sample_points(const iga_plan *plan, const void *field, const double *xs,
                                        int32_t nx, const double *ys, int32_t ny, double *out,
                                        void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(field, "field"))) return st;
    if (!xs || !ys || !out) return fail(IGA_EINVAL, "xs, ys and out must not be NULL");
    if (nx < 0 || ny < 0) return fail(IGA_EINVAL, "point counts must be >= 0");
    const long long n = (long long)nx * ny;
    if (n == 0) return IGA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SampleAxis ax = axis_of(plan->X, plan->P), ay = axis_of(plan->Y, plan->P);
    const int blocks = (int)((n + 255) / 256);
    if (plan->fp32)
        hipLaunchKernelGGL(k_sample<float>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const float *>(field), plan->Ny, ax, ay, xs, nx, ys, ny, out);
    else
        hipLaunchKernelGGL(k_sample<double>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const double *>(field), plan->Ny, ax, ay, xs, nx, ys, ny, out);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

extern "C" iga_status iga_count_ambiguous(const iga_plan *plan, const void *T, const void *fuel,
                                          double dT, double dF, int64_t *count, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel"))) return st;
    if (!count || (reinterpret_cast<uintptr_t>(count) & 7))
        return fail(IGA_EINVAL, "count must be an 8-byte aligned device pointer");
    if (!(dT >= 0) || !(dF >= 0)) return fail(IGA_EINVAL, "dT and dF must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    AmbParams a;
    a.ax = axis_of(plan->X, plan->P);
    a.ay = axis_of(plan->Y, plan->P);
    a.Ny = plan->Ny;
    a.nq = plan->P + 1;
    for (int q = 0; q < 4; ++q)
        a.g[q] = q < a.nq ? (plan->X.xq[q] - plan->X.knots[plan->P]) / plan->X.h : 0.0;
    a.t_ig = plan->d.c.t_ig;
    a.thr = plan->d.c.fuel_thr;
    a.dT = dT;
    a.dF = dF;
    unsigned long long *c = reinterpret_cast<unsigned long long *>(count);
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, c);
    const long long nel = (long long)plan->d.nel_x * plan->d.nel_y;
    const int blocks = (int)((nel + 255) / 256);
    if (plan->fp32)
        hipLaunchKernelGGL(k_ambiguous<float>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const float *>(T), static_cast<const float *>(fuel), a, c);
    else
        hipLaunchKernelGGL(k_ambiguous<double>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const double *>(T), static_cast<const double *>(fuel), a, c);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}
