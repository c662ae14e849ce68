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
// FP32 plans assemble the same quantities in increment form, R - A_impl S
// (A_impl the substep's implicit Kronecker operator), so that the float
// right-hand side carries only the O(tau) change of the state.
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
    // integrand  a0 v + ax v_x + ay v_y  with
    //   a0 = cs S - cx S_x - cy S_y + beta f,  ax = -(dx + beta g) S_x,  ay = -(dy + beta g) S_y
    T cs, cx, cy, dx, dy, beta;
    T c_adv, c_nld, c_ign, t_ig, fthr, t_act, c_forc, c_rad;
    T cf, fuel_dt_rate;   // fuel: a0f = F (cf - tau rate arr)
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

template <typename T, int P, bool FUEL>
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
    const int colA = J0 - P + lane, colB = colA + 64;
    const bool okA = colA >= 0 && colA < Ny, okB = lane < P && colB < Ny;

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

    // raw coefficients of row `row` for columns colA (and colB for the halo)
    auto fetch = [&](int row, T &c0, T &c1, T &f0, T &f1) {
        c0 = c1 = f0 = f1 = T(0);
        if (row >= 0 && row < a.Nx) {
            const size_t base = (size_t)row * Ny;
            if (okA) {
                c0 = a.S[base + colA];
                f0 = a.F[base + colA];
            }
            if (okB) {
                c1 = a.S[base + colB];
                f1 = a.F[base + colB];
            }
        }
    };
    // y half of the sum factorisation of one fetched row
    auto ytransform = [&](T c0, T c1, T f0, T f1, T(&v)[Q], T(&d)[Q], T(&f)[Q]) {
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
    for (int s = 0; s < P; ++s) {
        T c0, c1, f0, f1;
        fetch(X0 - P + s, c0, c1, f0, f1);
        ytransform(c0, c1, f0, f1, tv[s], td[s], tf[s]);
    }
    // coefficient rows are fetched two element rows ahead, the element row's
    // x basis table one row ahead, so neither load latency is exposed
    T nc0, nc1, nf0, nf1, mc0, mc1, mf0, mf1;
    fetch(X0, nc0, nc1, nf0, nf1);
    fetch(X0 + 1, mc0, mc1, mf0, mf1);
    auto xtab = [&](int ex, T(&v)[Q][Q], T(&dv)[Q][Q], T(&w)[Q]) {
        const int e = ex < 0 ? 0 : (ex >= a.nel_x ? a.nel_x - 1 : ex);
        const T *bxe = a.bx + (size_t)e * 2 * Q * Q;
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                v[i][q] = bxe[i * Q + q];
                dv[i][q] = bxe[Q * Q + i * Q + q];
            }
#pragma unroll
        for (int q = 0; q < Q; ++q) w[q] = a.wx[(size_t)e * Q + q];
    };
    T bxv[Q][Q], bxd[Q][Q], wxr[Q];
    xtab(X0 - P, bxv, bxd, wxr);

    for (int ex = X0 - P; ex < X1; ++ex) {
        const T c0 = nc0, c1 = nc1, f0 = nf0, f1 = nf1;
        nc0 = mc0; nc1 = mc1; nf0 = mf0; nf1 = mf1;
        fetch(ex + P + 2, mc0, mc1, mf0, mf1);
        T nbxv[Q][Q], nbxd[Q][Q], nwxr[Q];
        xtab(ex + 1, nbxv, nbxd, nwxr);
        ytransform(c0, c1, f0, f1, tv[P], td[P], tf[P]);
        if (ex >= 0 && ex < a.nel_x) {
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
                    const T a0 = W * (a.cs * S - a.cx * Sx - a.cy * Sy + a.beta * f);
                    const T bg = a.beta * g;
                    const T ax = -W * (a.dx + bg) * Sx;
                    const T ay = -W * (a.dy + bg) * Sy;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        acc0[i][qy] += a0 * bxv[i][qx] + ax * bxd[i][qx];
                        acc1[i][qy] += ay * bxv[i][qx];
                    }
                    if (FUEL) {
                        const T af = W * F * (a.cf - a.fuel_dt_rate * arr);
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
            if (lane >= P && colA < Ny) {
                a.R[(size_t)ex * Ny + colA] = r;
                if (FUEL) a.RF[(size_t)ex * Ny + colA] = rf;
            }
        }
        // roll the windows
#pragma unroll
        for (int i = 0; i < Q; ++i) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                bxv[i][q] = nbxv[i][q];
                bxd[i][q] = nbxd[i][q];
            }
            wxr[i] = nwxr[i];
        }
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
    // weights of the explicit (kx_e, ky_e) and implicit (kx_i, ky_i) parts of
    // the linear operator in this substep, and of F (beta)
    double kx_e = 0, ky_e = 0, kx_i = 0, ky_i = 0, beta;
    if (d.scheme == IGA_PR) {
        // substep 0: x implicit, L2 (y) explicit; substep 1: y implicit, L1 (x) explicit
        const double h = 0.5 * d.dt;
        if (substep == 0) { ky_e = h; kx_i = h; }
        else { kx_e = h; ky_i = h; }
        beta = h;
    } else {
        // S1 / S3: Crank-Nicolson on L1 over tau/2 (explicit and implicit halves)
        kx_e = kx_i = 0.25 * d.dt;
        beta = 0.5 * d.dt;
    }
    const double react = d.c.c_react;
    double cs, kx, ky;
    if (pl->delta) {
        // increment form: R - (implicit operator) S
        kx = kx_e + kx_i;
        ky = ky_e + ky_i;
        cs = kx * react;
        a.cf = T(0);
    } else {
        kx = kx_e;
        ky = ky_e;
        cs = 1.0 + kx * react;
        a.cf = T(1);
    }
    a.cs = (T)cs;
    a.cx = (T)(kx * d.c.c_adv * d.wind.bbar_x);
    a.cy = (T)(ky * d.c.c_adv * d.wind.bbar_y);
    a.dx = (T)(kx * d.c.c_diff);
    a.dy = (T)(ky * d.c.c_diff);
    a.beta = (T)beta;
    a.c_adv = (T)d.c.c_adv;
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
#define IGA_ASM(P_, FU_) \
    hipLaunchKernelGGL((k_assemble<T, P_, FU_>), dim3(blocks), dim3(256), 0, s, a)
    if (P == 2) {
        if (fuel) IGA_ASM(2, true);
        else IGA_ASM(2, false);
    } else if (P == 3) {
        if (fuel) IGA_ASM(3, true);
        else IGA_ASM(3, false);
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
