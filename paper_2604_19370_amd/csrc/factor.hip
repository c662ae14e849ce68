// factor.hip -- banded LU of the 1D operators and the chunk-transfer tables
// of the line solves, in double, on the device.
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

// Chunk transfer matrices.  Forward substitution y_r = b_r - sum_j L(r, r-1-j)
// y_{r-1-j} carries the state s = (y_r, ..., y_{r-P+1}); over the rows of one
// chunk it is affine, s_out = Phi s_in + psi(b), with Phi the product of the
// companion matrices of the rows.  Backward substitution carries
// t = (x_r, ..., x_{r+P-1}) and gives t_out = Psi t_in + phi(y).  Level d of
// the scan tables composes 2^d consecutive chunks.  One thread per operator.
template <int P>
__global__ void k_chunk_tables(const double *lf, const double *uf, int N, int m, int C, int D,
                               double *tf, double *tb)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    constexpr int PP = P * P;
    for (int c = 0; c < C; ++c) {
        double F[P][P], B[P][P];
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < P; ++j) F[i][j] = B[i][j] = (i == j) ? 1.0 : 0.0;
        const int r0 = c * m;
        const int r1 = min(N, r0 + m);
        for (int r = r0; r < r1; ++r) {  // F <- C_r F
            double row0[P];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k) s -= lf[(size_t)r * P + k] * F[k][j];
                row0[j] = s;
            }
#pragma unroll
            for (int i = P - 1; i >= 1; --i)
#pragma unroll
                for (int j = 0; j < P; ++j) F[i][j] = F[i - 1][j];
#pragma unroll
            for (int j = 0; j < P; ++j) F[0][j] = row0[j];
        }
        for (int r = r1 - 1; r >= r0; --r) {  // B <- D_r B
            double row0[P];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k) s -= uf[(size_t)r * (P + 1) + 1 + k] * B[k][j];
                row0[j] = s;
            }
#pragma unroll
            for (int i = P - 1; i >= 1; --i)
#pragma unroll
                for (int j = 0; j < P; ++j) B[i][j] = B[i - 1][j];
#pragma unroll
            for (int j = 0; j < P; ++j) B[0][j] = row0[j];
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < P; ++j) {
                tf[(size_t)c * PP + i * P + j] = F[i][j];
                tb[(size_t)c * PP + i * P + j] = B[i][j];
            }
    }
    for (int d = 1; d < D; ++d) {
        const int off = 1 << (d - 1);
        const double *pf = tf + (size_t)(d - 1) * C * PP;
        const double *pb = tb + (size_t)(d - 1) * C * PP;
        double *nf = tf + (size_t)d * C * PP;
        double *nb = tb + (size_t)d * C * PP;
        for (int c = 0; c < C; ++c) {
            for (int i = 0; i < P; ++i)
                for (int j = 0; j < P; ++j) {
                    double sf = 0.0, sb = 0.0;
                    if (c >= off) {
                        for (int k = 0; k < P; ++k)
                            sf += pf[(size_t)c * PP + i * P + k] * pf[(size_t)(c - off) * PP + k * P + j];
                    } else {
                        sf = pf[(size_t)c * PP + i * P + j];
                    }
                    if (c + off < C) {
                        for (int k = 0; k < P; ++k)
                            sb += pb[(size_t)c * PP + i * P + k] * pb[(size_t)(c + off) * PP + k * P + j];
                    } else {
                        sb = pb[(size_t)c * PP + i * P + j];
                    }
                    nf[(size_t)c * PP + i * P + j] = sf;
                    nb[(size_t)c * PP + i * P + j] = sb;
                }
        }
    }
}

__global__ void k_d2f(const double *src, float *dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

static iga_status d2f(const DevBuf &src, DevBuf &dst, hipStream_t s)
{
    size_t n = src.bytes / 8;
    if (dst.bytes != n * 4) IGA_HIP(dst.alloc(n * 4));
    if (!n) return IGA_OK;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_d2f, dim3(blocks), dim3(256), 0, s, src.as<double>(), dst.as<float>(), n);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

iga_status launch_chunk_tables(iga_plan *pl, int op, hipStream_t s)
{
    const int dir = (op == OP_AX || op == OP_MX) ? 0 : 1;
    const Schedule &sc = pl->sched[dir];
    const int N = dir ? pl->Ny : pl->Nx, P = pl->P;
    const int D = sc.levels > 0 ? sc.levels : 1;
    size_t bytes = (size_t)D * sc.chunks * P * P * 8;
    if (pl->op_tf64[op].bytes != bytes) {
        IGA_HIP(pl->op_tf64[op].alloc(bytes));
        IGA_HIP(pl->op_tb64[op].alloc(bytes));
    }
    auto lf = pl->op_lf64[op].as<double>();
    auto uf = pl->op_uf64[op].as<double>();
    auto tf = pl->op_tf64[op].as<double>();
    auto tb = pl->op_tb64[op].as<double>();
    if (P == 2)
        hipLaunchKernelGGL(k_chunk_tables<2>, dim3(1), dim3(64), 0, s, lf, uf, N, sc.m, sc.chunks, D, tf, tb);
    else if (P == 3)
        hipLaunchKernelGGL(k_chunk_tables<3>, dim3(1), dim3(64), 0, s, lf, uf, N, sc.m, sc.chunks, D, tf, tb);
    else
        return fail(IGA_EUNSUPPORTED, "degree not compiled");
    IGA_HIP(hipGetLastError());
    if (pl->fp32) {
        iga_status st;
        if ((st = d2f(pl->op_tf64[op], pl->op_tf32[op], s))) return st;
        if ((st = d2f(pl->op_tb64[op], pl->op_tb32[op], s))) return st;
    }
    return IGA_OK;
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
    if (pl->P == 2)
        hipLaunchKernelGGL(k_band_lu<2>, dim3(1), dim3(64), 0, s, d_bands, d_lf, d_uf, d_N, (int)NOPS);
    else if (pl->P == 3)
        hipLaunchKernelGGL(k_band_lu<3>, dim3(1), dim3(64), 0, s, d_bands, d_lf, d_uf, d_N, (int)NOPS);
    else
        return fail(IGA_EUNSUPPORTED, "degree not compiled");
    IGA_HIP(hipGetLastError());
    iga_status st;
    for (int op = 0; op < NOPS; ++op)
        if ((st = launch_chunk_tables(pl, op, s))) return st;
    if (pl->fp32) {
        for (int op = 0; op < NOPS; ++op) {
            if ((st = d2f(pl->op_lf64[op], pl->op_lf32[op], s))) return st;
            if ((st = d2f(pl->op_uf64[op], pl->op_uf32[op], s))) return st;
        }
    }
    // the metadata buffer is freed at scope exit: make sure the kernel is done
    IGA_HIP(hipStreamSynchronize(s));
    return IGA_OK;
}

}  // namespace iga
