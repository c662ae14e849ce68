// factor.hip -- banded LU of the 1D operators, in double, on the device.  The
// factors are read back once to build the line-solve tables (plan.cpp).
//
// Section 4: every directional substep solves (M + gamma K + delta G) along
// independent lines; the operators are banded with half-bandwidth p, so a
// banded LU without pivoting (the matrices are symmetric positive definite
// mass/stiffness combinations plus a small skew advection part) gives
// O(p^2 N) solves.
#include "iga_internal.h"

namespace iga {

// One thread per operator.  Doolittle elimination with a sliding window of
// the p+1 active rows kept in registers: win[i][k - (row_i) + P] holds
// A(k + i, .) for the current pivot row k.
template <int P>
__global__ void k_band_lu(const double *const *bands, double *const *lf, double *const *uf,
                          const int *Ns, int nops)
{
    const int op = blockIdx.x * blockDim.x + threadIdx.x;
    if (op >= nops) return;
    constexpr int W = 2 * P + 1;
    const int N = Ns[op];
    const double *A = bands[op];
    double *L = lf[op], *U = uf[op];
    double win[P + 1][W];
#pragma unroll
    for (int i = 0; i <= P; ++i)
#pragma unroll
        for (int c = 0; c < W; ++c) win[i][c] = (i < N) ? A[(size_t)i * W + c] : 0.0;
    // rows r < P have no multipliers for columns r-1-j < 0
    for (int r = 0; r < P && r < N; ++r)
        for (int j = 0; j < P; ++j) L[(size_t)r * P + j] = 0.0;
    for (int k = 0; k < N; ++k) {
        const double piv = win[0][P];
        const double inv = 1.0 / piv;
        U[(size_t)k * (P + 1)] = inv;
#pragma unroll
        for (int c = 1; c <= P; ++c)
            U[(size_t)k * (P + 1) + c] = (k + c < N) ? win[0][P + c] * inv : 0.0;
#pragma unroll
        for (int i = 1; i <= P; ++i) {
            if (k + i < N) {
                const double l = win[i][P - i] * inv;
                L[(size_t)(k + i) * P + (i - 1)] = l;
#pragma unroll
                for (int c = 1; c <= P; ++c) win[i][P - i + c] -= l * win[0][P + c];
            }
        }
        // slide the window
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int c = 0; c < W; ++c) win[i][c] = win[i + 1][c];
        const int nr = k + P + 1;
#pragma unroll
        for (int c = 0; c < W; ++c) win[P][c] = (nr < N) ? A[(size_t)nr * W + c] : 0.0;
    }
}

iga_status launch_factor(iga_plan *pl, hipStream_t s)
{
    const double *bands[NOPS];
    double *lf[NOPS], *uf[NOPS];
    int Ns[NOPS];
    for (int op = 0; op < NOPS; ++op) {
        bands[op] = pl->op_a64[op].as<double>();
        lf[op] = pl->op_lf64[op].as<double>();
        uf[op] = pl->op_uf64[op].as<double>();
        Ns[op] = (op == OP_AX || op == OP_MX) ? pl->Nx : pl->Ny;
    }
    DevBuf meta;
    const size_t mbytes = sizeof(bands) + sizeof(lf) + sizeof(uf) + sizeof(Ns);
    IGA_HIP(meta.alloc(mbytes));
    char host[sizeof(bands) + sizeof(lf) + sizeof(uf) + sizeof(Ns)];
    std::memcpy(host, bands, sizeof(bands));
    std::memcpy(host + sizeof(bands), lf, sizeof(lf));
    std::memcpy(host + sizeof(bands) + sizeof(lf), uf, sizeof(uf));
    std::memcpy(host + sizeof(bands) + sizeof(lf) + sizeof(uf), Ns, sizeof(Ns));
    IGA_HIP(hipMemcpyAsync(meta.ptr, host, mbytes, hipMemcpyHostToDevice, s));
    char *mp = meta.as<char>();
    auto d_bands = reinterpret_cast<const double *const *>(mp);
    auto d_lf = reinterpret_cast<double *const *>(mp + sizeof(bands));
    auto d_uf = reinterpret_cast<double *const *>(mp + sizeof(bands) + sizeof(lf));
    auto d_N = reinterpret_cast<const int *>(mp + sizeof(bands) + sizeof(lf) + sizeof(uf));
    if (pl->P == 1)
        hipLaunchKernelGGL(k_band_lu<1>, dim3(1), dim3(64), 0, s, d_bands, d_lf, d_uf, d_N, (int)NOPS);
    else if (pl->P == 2)
        hipLaunchKernelGGL(k_band_lu<2>, dim3(1), dim3(64), 0, s, d_bands, d_lf, d_uf, d_N, (int)NOPS);
    else if (pl->P == 3)
        hipLaunchKernelGGL(k_band_lu<3>, dim3(1), dim3(64), 0, s, d_bands, d_lf, d_uf, d_N, (int)NOPS);
    else
        return fail(IGA_EUNSUPPORTED, "degree not compiled");
    IGA_HIP(hipGetLastError());
    // the metadata buffer is freed at scope exit and the factors are read
    // back for the line-solve tables: wait for the kernel
    IGA_HIP(hipStreamSynchronize(s));
    return build_solve_tables(pl);
}

}  // namespace iga
