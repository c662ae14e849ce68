// assemble.hip -- Gauss-quadrature right-hand side of one substep.
//
// Weak forms eq. (varPR_wildfire) and eq. (varCN), with F of the generic
// equation at the start of Section 3 evaluated explicitly from the state S
// entering the substep:
//   R_ij = sum_e sum_q w|J| [ S v - alpha (C_diff d_eS d_ev + C_adv bbar_e d_eS v
//                                           - [e=x] C_react S v)
//                             + beta (f v - C_nld S^3 grad S . grad v) ]
//   f = -C_adv (b - bbar).grad S + C_forcing - C_rad S^4
//       + [S > T_ig and fuel > thr] C_ign S exp(-T_act/S)
// and, for the first substep of a step, the fuel right-hand side of the
// compute_rhs listing (Section 7): fuel v (1 - tau rate [ign] S exp(-T_act/S)).
//
// Schedule: one wavefront owns a strip of 64 element columns (lane = element
// column ey, the strip's first p lanes are halo) and marches along x over a
// tile of element rows.  Per step it loads one new coefficient row of S and
// fuel (coalesced), contracts it in y with the lane's own basis table (the
// y half of the sum factorisation, reused by the p+1 elements that share the
// row), finishes the x half with the element row's basis table held in scalar
// registers, evaluates the pointwise terms at the (p+1)^2 points, and
// accumulates the x half of the test-function contraction into rolling
// per-row accumulators.  When a dof row is complete its y contraction is
// gathered from the p neighbouring lanes and stored.  Every dof is summed by
// exactly one lane in a fixed order: no atomics, deterministic.
#include "iga_internal.h"

namespace iga {

template <typename T> struct AsmParams {
    const T *S, *F;
    T *R, *RF;
    const T *bx, *by;   // [e][2][Q][Q]: (values, derivatives)[a][q]
    const T *wx, *wy;   // (b_y(x) - bbar_y) at x-points, (b_x(y) - bbar_x) at y-points
    T w[16];            // w_qx w_qy |J| per point (uniform mesh)
    T alpha, beta, c_adv, c_diff, react_e, bbar_e, c_nld, c_ign, t_ig, fthr, t_act, c_forc,
        c_rad, fuel_dt_rate;
    int nel_x, nel_y, Nx, Ny, rows, nstrips, ntiles;
};

template <typename T> __device__ __forceinline__ T shfl(T v, int src)
{
    return __shfl(v, src, 64);
}

template <typename T> __device__ __forceinline__ T arrhenius(T S, T t_act)
{
    return S * exp(-t_act / S);
}

template <typename T, int P, bool FUEL, int EDIR>
__global__ __launch_bounds__(256) void k_assemble(AsmParams<T> a)
{
    constexpr int Q = P + 1;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (gw >= a.nstrips * a.ntiles) return;
    const int strip = gw % a.nstrips, tile = gw / a.nstrips;
    const int J0 = strip * (64 - P);
    const int ey = J0 - P + lane;
    const bool eyok = ey >= 0 && ey < a.nel_y;
    const int Ny = a.Ny;

    T byv[Q][Q], byd[Q][Q], wyr[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            byv[b][q] = eyok ? a.by[(((size_t)ey * 2 + 0) * Q + b) * Q + q] : T(0);
            byd[b][q] = eyok ? a.by[(((size_t)ey * 2 + 1) * Q + b) * Q + q] : T(0);
        }
#pragma unroll
    for (int q = 0; q < Q; ++q) wyr[q] = eyok ? a.wy[(size_t)ey * Q + q] : T(0);

    // y half of the sum factorisation for coefficient row `row`
    auto load_row = [&](int row, T(&v)[Q], T(&d)[Q], T(&f)[Q]) {
        T c0 = 0, c1 = 0, f0 = 0, f1 = 0;
        if (row >= 0 && row < a.Nx) {
            const int colA = J0 - P + lane, colB = colA + 64;
            const size_t base = (size_t)row * Ny;
            if (colA >= 0 && colA < Ny) {
                c0 = a.S[base + colA];
                f0 = a.F[base + colA];
            }
            if (lane < P && colB < Ny) {
                c1 = a.S[base + colB];
                f1 = a.F[base + colB];
            }
        }
        T cb[Q], fb[Q];
        cb[0] = c0;
        fb[0] = f0;
#pragma unroll
        for (int b = 1; b < Q; ++b) {
            const int src = lane + b;
            const T u0 = shfl(c0, src & 63), u1 = shfl(c1, (src - 64) & 63);
            const T g0 = shfl(f0, src & 63), g1 = shfl(f1, (src - 64) & 63);
            cb[b] = src < 64 ? u0 : u1;
            fb[b] = src < 64 ? g0 : g1;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T sv = 0, sd = 0, sf = 0;
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                sv += cb[b] * byv[b][q];
                sd += cb[b] * byd[b][q];
                sf += fb[b] * byv[b][q];
            }
            v[q] = sv;
            d[q] = sd;
            f[q] = sf;
        }
    };

    const int X0 = tile * a.rows;
    const int X1 = min(X0 + a.rows, a.Nx);
    T tv[Q][Q], td[Q][Q], tf[Q][Q];
    T acc0[Q][Q], acc1[Q][Q], accf[Q][Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int q = 0; q < Q; ++q) acc0[i][q] = acc1[i][q] = accf[i][q] = T(0);
#pragma unroll
    for (int s = 0; s < P; ++s) load_row(X0 - P + s, tv[s], td[s], tf[s]);

    for (int ex = X0 - P; ex < X1; ++ex) {
        load_row(ex + P, tv[P], td[P], tf[P]);
        if (ex >= 0 && ex < a.nel_x) {
            const T *bxe = a.bx + (size_t)ex * 2 * Q * Q;
            T bxv[Q][Q], bxd[Q][Q], wxr[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    bxv[i][q] = bxe[i * Q + q];
                    bxd[i][q] = bxe[Q * Q + i * Q + q];
                }
#pragma unroll
            for (int q = 0; q < Q; ++q) wxr[q] = a.wx[(size_t)ex * Q + q];
#pragma unroll
            for (int qx = 0; qx < Q; ++qx) {
#pragma unroll
                for (int qy = 0; qy < Q; ++qy) {
                    T S = 0, Sx = 0, Sy = 0, F = 0;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        S += bxv[i][qx] * tv[i][qy];
                        Sx += bxd[i][qx] * tv[i][qy];
                        Sy += bxv[i][qx] * td[i][qy];
                        F += bxv[i][qx] * tf[i][qy];
                    }
                    const T W = a.w[qx * Q + qy];
                    const T S2 = S * S;
                    const T g = a.c_nld * S2 * S;
                    T f = a.c_forc - a.c_rad * S2 * S2 - a.c_adv * (wyr[qy] * Sx + wxr[qx] * Sy);
                    T arr = T(0);
                    if (S > a.t_ig && F > a.fthr) arr = arrhenius(S, a.t_act);
                    f += a.c_ign * arr;
                    const T dSe = EDIR ? Sy : Sx;
                    const T a0 = W * (S + a.alpha * (a.react_e * S - a.c_adv * a.bbar_e * dSe) + a.beta * f);
                    const T ax = W * ((EDIR ? T(0) : -a.alpha * a.c_diff) - a.beta * g) * Sx;
                    const T ay = W * ((EDIR ? -a.alpha * a.c_diff : T(0)) - a.beta * g) * Sy;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        acc0[i][qy] += a0 * bxv[i][qx] + ax * bxd[i][qx];
                        acc1[i][qy] += ay * bxv[i][qx];
                    }
                    if (FUEL) {
                        const T af = W * F * (T(1) - a.fuel_dt_rate * arr);
#pragma unroll
                        for (int i = 0; i < Q; ++i) accf[i][qy] += af * bxv[i][qx];
                    }
                }
            }
        }
        if (ex >= X0) {
            // dof row ex is complete: y half of the test contraction
            T pb[Q], pf[Q];
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    s0 += acc0[0][q] * byv[b][q] + acc1[0][q] * byd[b][q];
                    if (FUEL) s1 += accf[0][q] * byv[b][q];
                }
                pb[b] = s0;
                pf[b] = s1;
            }
            T r = pb[0], rf = pf[0];
#pragma unroll
            for (int b = 1; b < Q; ++b) {
                r += shfl(pb[b], (lane - b) & 63);
                if (FUEL) rf += shfl(pf[b], (lane - b) & 63);
            }
            const int col = J0 - P + lane;
            if (lane >= P && col < Ny) {
                a.R[(size_t)ex * Ny + col] = r;
                if (FUEL) a.RF[(size_t)ex * Ny + col] = rf;
            }
        }
        // roll the windows
#pragma unroll
        for (int s = 0; s < P; ++s)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                tv[s][q] = tv[s + 1][q];
                td[s][q] = td[s + 1][q];
                tf[s][q] = tf[s + 1][q];
                acc0[s][q] = acc0[s + 1][q];
                acc1[s][q] = acc1[s + 1][q];
                accf[s][q] = accf[s + 1][q];
            }
#pragma unroll
        for (int q = 0; q < Q; ++q) acc0[P][q] = acc1[P][q] = accf[P][q] = T(0);
    }
}

template <typename T>
static iga_status launch_t(const iga_plan *pl, int substep, const void *S, const void *F, void *R,
                           void *RF, hipStream_t s)
{
    const iga_plan_desc &d = pl->d;
    const int P = pl->P, Q = P + 1;
    AsmParams<T> a;
    std::memset(&a, 0, sizeof a);
    a.S = static_cast<const T *>(S);
    a.F = static_cast<const T *>(F);
    a.R = static_cast<T *>(R);
    a.RF = static_cast<T *>(RF);
    a.bx = pl->asm_bx.as<T>();
    a.by = pl->asm_by.as<T>();
    a.wx = pl->asm_wx.as<T>();
    a.wy = pl->asm_wy.as<T>();
    for (int qx = 0; qx < Q; ++qx)
        for (int qy = 0; qy < Q; ++qy) a.w[qx * Q + qy] = (T)(pl->X.wq[qx] * pl->Y.wq[qy]);
    int edir;
    double alpha, beta;
    if (d.scheme == IGA_PR) {
        edir = substep == 0 ? 1 : 0;
        alpha = beta = 0.5 * d.dt;
    } else {
        edir = 0;
        alpha = 0.25 * d.dt;
        beta = 0.5 * d.dt;
    }
    a.alpha = (T)alpha;
    a.beta = (T)beta;
    a.c_adv = (T)d.c.c_adv;
    a.c_diff = (T)d.c.c_diff;
    a.react_e = (T)(edir ? 0.0 : d.c.c_react);
    a.bbar_e = (T)(edir ? d.wind.bbar_y : d.wind.bbar_x);
    a.c_nld = (T)d.c.c_nld;
    a.c_ign = (T)d.c.c_ign;
    a.t_ig = (T)d.c.t_ig;
    a.fthr = (T)d.c.fuel_thr;
    a.t_act = (T)d.c.t_act;
    a.c_forc = (T)d.c.c_forcing;
    a.c_rad = (T)d.c.c_rad;
    a.fuel_dt_rate = (T)(d.dt * d.c.fuel_rate);
    a.nel_x = d.nel_x;
    a.nel_y = d.nel_y;
    a.Nx = pl->Nx;
    a.Ny = pl->Ny;
    a.rows = pl->asm_rows;
    a.nstrips = (pl->Ny + (64 - P) - 1) / (64 - P);
    a.ntiles = (pl->Nx + a.rows - 1) / a.rows;
    const int waves = a.nstrips * a.ntiles;
    const int blocks = (waves + 3) / 4;
    const bool fuel = RF != nullptr;
#define IGA_ASM(P_, FU_, E_)                                                                   \
    hipLaunchKernelGGL((k_assemble<T, P_, FU_, E_>), dim3(blocks), dim3(256), 0, s, a)
    if (P == 2) {
        if (fuel) { if (edir) IGA_ASM(2, true, 1); else IGA_ASM(2, true, 0); }
        else { if (edir) IGA_ASM(2, false, 1); else IGA_ASM(2, false, 0); }
    } else if (P == 3) {
        if (fuel) { if (edir) IGA_ASM(3, true, 1); else IGA_ASM(3, true, 0); }
        else { if (edir) IGA_ASM(3, false, 1); else IGA_ASM(3, false, 0); }
    } else {
        return fail(IGA_EUNSUPPORTED, "degree not compiled");
    }
#undef IGA_ASM
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

iga_status launch_assemble(const iga_plan *pl, int substep, const void *S, const void *F, void *R,
                           void *RF, hipStream_t s)
{
    return pl->fp32 ? launch_t<float>(pl, substep, S, F, R, RF, s)
                    : launch_t<double>(pl, substep, S, F, R, RF, s);
}

// ---------------------------------------------------------------------------
// non-finite detector (iga_run with check_every > 0)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_nonfinite(const T *a, const T *b, size_t n, int *flag)
{
    int bad = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        bad |= (!isfinite(a[i]) || !isfinite(b[i])) ? 1 : 0;
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

iga_status launch_nonfinite(const iga_plan *pl, const void *T_, const void *F, int *flag,
                            hipStream_t s)
{
    const size_t n = pl->ndof;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
    if (pl->fp32)
        hipLaunchKernelGGL(k_nonfinite<float>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const float *>(T_), static_cast<const float *>(F), n, flag);
    else
        hipLaunchKernelGGL(k_nonfinite<double>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const double *>(T_), static_cast<const double *>(F), n, flag);
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

}  // namespace iga
