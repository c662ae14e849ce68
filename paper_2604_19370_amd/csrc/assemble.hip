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
// A forced step adds to f a source sampled at the quadrature points (the
// forcing of the manufactured-solution study, Section 6.1); that is a
// separate compile-time variant, the unforced kernels do not test for it.
// FP32 plans assemble the same quantities in increment form, R - A_impl S
// (A_impl the substep's implicit Kronecker operator), so that the float
// right-hand side carries only the O(tau) change of the state.
//
// Schedule: one wavefront owns a strip of 64 element columns (lane = element
// column ey, the strip's first p lanes are halo) and marches along x over a
// tile of element rows.  Per step it takes one new coefficient row of S and
// fuel (loaded p+1 rows ahead, coalesced), contracts it in y with the lane's
// own basis table (the y half of the sum factorisation, reused by the p+1
// elements that share the row; neighbouring columns arrive by DPP rotates),
// finishes the x half with the element row's basis table (one for the
// whole wavefront: held in registers across steps, or read from LDS),
// evaluates the pointwise terms at the (p+1)^2 points and
// accumulates the x half of the test-function contraction into per-row
// accumulators.  When a dof row is complete its y contraction is gathered from
// the p neighbouring lanes and stored.  In the stacked variant a workgroup's
// four wavefronts take four consecutive tiles of one strip; the p dof rows
// where two of its tiles meet are summed in two parts (the upper tile's
// elements, then the lower one's) that meet in LDS, so only the first tile
// re-evaluates the p elements above it (in the unstacked variant every tile
// does).  Every dof is summed by one lane, or two parts by two fixed lanes,
// in a fixed order: no atomics, deterministic.  The right-hand sides are
// stored non-temporally (streamed out of L2): the sweep that reads them next
// runs on every XCD.
//
// The marching loop is unrolled by p+1, so the rolling windows (coefficient
// rows, accumulators, pending loads) are renamed, not copied.  The x
// quadrature weight is folded into the pointwise coefficients, the y weight
// into the completed row.  The ignition indicator needs S > T_ig somewhere in
// the element; S is a convex combination of the element's coefficients
// (B-splines are non-negative and sum to one), so where no coefficient of any
// element of the wavefront's row exceeds T_ig (less a rounding margin) the
// Arrhenius term is zero and the fuel terms that only it feeds are skipped.
// In increment form (FP32 plans) an element whose coefficients all equal the
// ambient fixed point (where c_react T + c_forcing - c_rad T^4 = 0) has no
// gradient and no net source, so it contributes nothing; where that holds for
// every element of the wavefront's row, the row's pointwise terms and test
// contractions are skipped too.
#include <cmath>
#include <limits>

#include "dpp.h"
#include "iga_internal.h"

namespace iga {

template <typename T> struct AsmParams {
    const T *S, *F;
    T *R, *RF;
    const T *bx, *by;   // [e][2][Q][Q]: (values, derivatives)[a][q]
    const T *wx, *wy;   // (b_y(x) - bbar_y) at x-points, (b_x(y) - bbar_x) at y-points
    T wxq[4], wyq[4];   // Gauss weight * h/2 per point and direction (uniform mesh)
    // integrand  a0 v + ax v_x + ay v_y, weighted by wxq[qx] here:
    //   a0 = cs S + (-cx - beta c_adv wy) S_x + (-cy - beta c_adv wx) S_y
    //        + beta (c_forc - c_rad S^4 + c_ign arr)
    //   ax = -(dx + beta c_nld S^3) S_x,  ay = -(dy + beta c_nld S^3) S_y
    // fuel: af = F (cf - tau rate arr)
    T cs_w[4], frc_w[4], rad_w[4], nld_w[4], dx_w[4], dy_w[4], ign_w[4], cf_w[4], rate_w[4];
    T cx, cy, bca;      // bca = beta c_adv
    T t_ig, t_skip, fthr, t_act;
    // increment form: an element whose coefficients all equal t_fix (the
    // ambient fixed point) contributes nothing, and is skipped when amb != 0
    T t_fix;
    int amb;
    int fuel_all;       // fuel right-hand side nonzero without ignition (direct form)
    int nel_x, nel_y, Nx, Ny, rows, nstrips, ntiles, ngroups;   // rows: dof rows per tile
    int stack;   // tiles of a workgroup share halos (else each evaluates its own);
                 // the kernels are compiled for one or the other
    // source samples src[(ex*Q + qx) * nel_y*Q + ey*Q + qy] (forced variant),
    // weighted by src_w[qx] = beta * x weight
    const T *src;
    T src_w[4];
};

template <int N> struct Ic {
    static constexpr int value = N;
};

// read-only device data seen through the constant address space (loads the
// compiler may issue as scalar loads where the address is uniform)
template <typename T> using CT = const __attribute__((address_space(4))) T;
template <typename T> __device__ __forceinline__ CT<T> *as_const(const T *p)
{
    return (CT<T> *)p;
}

// The work of one wavefront: dof rows [X0, X1) of strip `strip` (and the
// elements of those rows).
//   halo: also evaluate the p elements above the tile, so that its first p
//         dof rows are complete (the first tile of a workgroup);
//   hold: those p rows get the contributions of the tile's own elements only
//         and go to hd[2][P][64] (T, fuel) for the workgroup to finish;
//   tail: march p more steps without elements, and put the contributions of
//         the tile's last elements to the p rows below it into tl[2][P][64].
template <typename T, int P, bool FUEL, bool SRC = false>
__device__ __forceinline__ void assemble_body(const AsmParams<T> &a, const int strip, const int X0,
                                              const int X1, const bool halo, const bool hold, const bool tail,
                                              T *__restrict__ hd, T *__restrict__ tl,
                                              const T *__restrict__ ltab)
{
    constexpr int Q = P + 1;
    const int lane = threadIdx.x & 63;
    const int J0 = strip * (64 - P);
    const int ey = J0 - P + lane;
    const bool eyok = ey >= 0 && ey < a.nel_y;
    const int Ny = a.Ny;
    const int colA = J0 - P + lane, colB = colA + 64;
    const bool okA = colA >= 0 && colA < Ny, okB = lane < P && colB < Ny;

    T byv[Q][Q], byd[Q][Q], kxw[Q][Q];
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            byv[b][q] = eyok ? a.by[(((size_t)ey * 2 + 0) * Q + b) * Q + q] : T(0);
            byd[b][q] = eyok ? a.by[(((size_t)ey * 2 + 1) * Q + b) * Q + q] : T(0);
        }
    T wyl[Q];   // the lane's wind values, turned into kxw once the rows are requested
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) wyl[qy] = eyok ? a.wy[(size_t)ey * Q + qy] : T(0);

    // Marching-loop form.  The hardware counts vector loads in issue order,
    // so a step that waits for any vector load also waits for every row
    // fetched before it.  The march is split: a main loop over the steps
    // whose row fetch lies inside the tile issues no other vector loads
    // than those rows, each Q steps ahead of its use and with no branch
    // around it, so that a step waits only for the row it consumes.  There
    // the element row's basis tables are held across steps and reloaded
    // where they change, at the mesh ends (p <= 2), or read from LDS at
    // every step (LTAB, p = 3, whose kernels are at the register limit),
    // and the wind values come by scalar loads.  The tile's last steps use
    // a conditional fetch and load the tables at every step.  FP64 cubic
    // kernels spill more with the split loop and keep the single one (PIPE
    // false: every step as the tile's last ones).
    constexpr bool PIPE = !(sizeof(T) == 8 && P >= 3);
    constexpr bool LTAB = PIPE && P >= 3;   // tables from ltab (LDS, one slot per distinct table)
    // raw coefficients of row `row` for columns colA (and colB for the halo).
    // Every lane loads, from its column clamped into the mesh (lanes without
    // a halo column repeat their own); columns outside the mesh are zeroed
    // where the values are consumed, so no lane mask surrounds the loads.
    // Rows from min(X1, nel_x) + p on only feed elements that are not
    // evaluated: they are not loaded (the registers keep what they held).
    const int rlim = min(X1, a.nel_x) + P;
    const unsigned offA = (unsigned)min(max(colA, 0), Ny - 1) * (unsigned)sizeof(T);
    const unsigned offB = okB ? (unsigned)colB * (unsigned)sizeof(T) : offA;
    auto load_row = [&](int row, T &c0, T &c1, T &f0, T &f1) {
        const size_t rb = (size_t)row * Ny * sizeof(T);
        const char *sr = reinterpret_cast<const char *>(a.S) + rb;
        const char *fr = reinterpret_cast<const char *>(a.F) + rb;
        c0 = *reinterpret_cast<const T *>(sr + offA);
        f0 = *reinterpret_cast<const T *>(fr + offA);
        c1 = *reinterpret_cast<const T *>(sr + offB);
        f1 = *reinterpret_cast<const T *>(fr + offB);
    };
    // mode Ic<0>: conditional.  Ic<1> (the main loop): the row lies below
    // rlim, loaded without a branch.  Ic<2> (the window set-up): rows
    // past rlim clamped to rlim - 1 (rows below 0 to 0; both only feed
    // elements that are not evaluated) and loaded without a branch, so that
    // the main loop starts with every load accounted for.
    auto fetch = [&](int row, T &c0, T &c1, T &f0, T &f1, auto inrange) {
        constexpr int mode = decltype(inrange)::value;
        if constexpr (PIPE && mode == 1) load_row(max(row, 0), c0, c1, f0, f1);
        else if constexpr (PIPE && mode == 2) load_row(min(max(row, 0), rlim - 1), c0, c1, f0, f1);
        else if (row < rlim) load_row(max(row, 0), c0, c1, f0, f1);
    };
    // The fuel enters only the ignition and fuel terms, which FP32
    // (increment-form) plans evaluate in the rare wavefronts near T_ig: there
    // (LAZYF) the ring keeps the row's raw fuel coefficients and their y
    // contraction is formed only where it is used, in the same order.
    constexpr bool LAZYF = sizeof(T) == 4 && P <= 2;
    auto ytrans_fuel = [&](const T(&fb)[Q], int q) {
        T sf = 0;
#pragma unroll
        for (int b = 0; b < Q; ++b) sf += fb[b] * byv[b][q];
        return sf;
    };
    // y half of the sum factorisation of one fetched row, the largest
    // coefficient of the row within the lane's element, and whether all of
    // them equal the ambient fixed point
    auto ytransform = [&](T c0, T c1, T f0, T f1, T(&v)[Q], T(&d)[Q], T(&f)[Q], T &mx, bool &am) {
        c0 = okA ? c0 : T(0);
        f0 = okA ? f0 : T(0);
        c1 = okB ? c1 : T(0);
        f1 = okB ? f1 : T(0);
        T cb[Q], fb[Q];
        cb[0] = c0;
        fb[0] = f0;
        cb[1] = lane_ahead<1>(c0, c1, lane);
        fb[1] = lane_ahead<1>(f0, f1, lane);
        if constexpr (Q > 2) {
            cb[2] = lane_ahead<2>(c0, c1, lane);
            fb[2] = lane_ahead<2>(f0, f1, lane);
        }
        if constexpr (Q > 3) {
            cb[3] = lane_ahead<3>(c0, c1, lane);
            fb[3] = lane_ahead<3>(f0, f1, lane);
        }
        // (compare and select, not fmax: the inputs need no canonicalising,
        // and a NaN coefficient leaves a NaN right-hand side either way)
        mx = cb[0];
        am = cb[0] == a.t_fix;
#pragma unroll
        for (int b = 1; b < Q; ++b) {
            mx = cb[b] > mx ? cb[b] : mx;
            am = am & (cb[b] == a.t_fix);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T sv = 0, sd = 0;
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                sv += cb[b] * byv[b][q];
                sd += cb[b] * byd[b][q];
            }
            v[q] = sv;
            d[q] = sd;
        }
        if constexpr (LAZYF) {
#pragma unroll
            for (int b = 0; b < Q; ++b) f[b] = fb[b];
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) f[q] = ytrans_fuel(fb, q);
        }
    };

    const int E0 = halo ? X0 - P : X0;       // first element row marched
    const int K = X1 - E0 + (tail ? P : 0);   // marching steps
    // rings indexed by (step + i) mod Q
    T tv[Q][Q], td[Q][Q], tf[Q][Q], rmx[Q];   // tf: raw fuel coefficients under LAZYF
    bool ram[Q];
    T acc0[Q][Q], acc1[Q][Q], accf[Q][Q];
    T pc0[Q] = {}, pc1[Q] = {}, pf0[Q] = {}, pf1[Q] = {};
    // live[s]: the dof row in slot s has received the contribution of an
    // evaluated element (wavefront-uniform); a row without one is exactly zero
    bool live[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        live[i] = false;
#pragma unroll
        for (int q = 0; q < Q; ++q) acc0[i][q] = acc1[i][q] = accf[i][q] = T(0);
    }
    // window rows E0 .. E0+P-1 (slots 0 .. P-1) and the pending rows (step
    // k consumes row E0 + P + k from slot k mod Q), all requested before the
    // window rows are transformed, so that their latencies overlap
    T wc0[P], wc1[P], wf0[P], wf1[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
        wc0[s] = wc1[s] = wf0[s] = wf1[s] = T(0);
        fetch(E0 + s, wc0[s], wc1[s], wf0[s], wf1[s], Ic<2>{});
    }
#pragma unroll
    for (int s = 0; s < Q; ++s) fetch(E0 + P + s, pc0[s], pc1[s], pf0[s], pf1[s], Ic<2>{});
#pragma unroll
    for (int s = 0; s < P; ++s)
        ytransform(wc0[s], wc1[s], wf0[s], wf1[s], tv[s], td[s], tf[s], rmx[s], ram[s]);
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
        const T k = -a.cx - a.bca * wyl[qy];
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) kxw[qx][qy] = k * a.wxq[qx];
    }

    const T t_skip = a.t_skip;
    T bxv[Q][Q], bxd[Q][Q];   // basis tables of element row e2_held
    int e2_held = -1;
    auto step = [&](auto phase, int k, auto inrange) {
        constexpr int ph = decltype(phase)::value;
        constexpr int snew = (ph + P) % Q;   // slot of the new coefficient row / dof row ex+P
        const int ex = E0 + k;
        ytransform(pc0[ph], pc1[ph], pf0[ph], pf1[ph], tv[snew], td[snew], tf[snew], rmx[snew],
                   ram[snew]);
        fetch(ex + P + Q, pc0[ph], pc1[ph], pf0[ph], pf1[ph], inrange);
        // an element whose coefficients all sit at the ambient fixed point
        // has no gradient, no net source and no ignition: in increment form
        // it contributes exactly nothing (the skip is wavefront-uniform)
        bool eam = ram[0];
#pragma unroll
        for (int s = 1; s < Q; ++s) eam = eam & ram[s];
        const bool quiet = !SRC && a.amb && __all(!eyok || eam);
        if (ex >= 0 && ex < a.nel_x && ex < X1 && !quiet) {
            const int e2 = (ex >= P && ex < a.nel_x - P) ? P : ex;   // interior tables coincide
            // the main loop holds the tables (reloaded where they change) or
            // reads them from LDS; elsewhere they are loaded at every step
            constexpr bool MAIN = PIPE && decltype(inrange)::value == 1;
            constexpr bool HOLD = MAIN && !LTAB;
            if constexpr (LTAB) {
                // slots: the p head tables, the interior one, the p tail tables
                const int slot = e2 <= P ? e2 : P + 1 + e2 - (a.nel_x - P);
                const T *bxe = ltab + slot * 2 * Q * Q;
#pragma unroll
                for (int i = 0; i < Q; ++i)
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        bxv[i][q] = bxe[i * Q + q];
                        bxd[i][q] = bxe[Q * Q + i * Q + q];
                    }
            } else if (!HOLD || e2 != e2_held) {
                const T *bxe = a.bx + (size_t)e2 * 2 * Q * Q;
#pragma unroll
                for (int i = 0; i < Q; ++i)
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        bxv[i][q] = bxe[i * Q + q];
                        bxd[i][q] = bxe[Q * Q + i * Q + q];
                    }
                e2_held = HOLD ? e2 : -1;
                // HOLD: wait here, on this rare path, for every vector load,
                // so that after the branch the tables are known to have
                // arrived on both paths and the common path waits only for
                // the coefficient row it consumes
                if constexpr (HOLD) __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
            }
            T kyw[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                T w;
                if constexpr (MAIN) w = as_const(a.wx)[(size_t)ex * Q + q];
                else w = a.wx[(size_t)ex * Q + q];
                kyw[q] = (-a.cy - a.bca * w) * a.wxq[q];
            }
            T emx = rmx[0];
#pragma unroll
            for (int s = 1; s < Q; ++s) emx = rmx[s] > emx ? rmx[s] : emx;
            const bool hot = FUEL ? (a.fuel_all || __any(emx > t_skip)) : __any(emx > t_skip);
            // linear, loss, forcing, wind and T^3-diffusion terms; the first
            // contribution to the fresh dof row (slot snew) is assigned
#pragma unroll
            for (int qx = 0; qx < Q; ++qx) {
#pragma unroll
                for (int qy = 0; qy < Q; ++qy) {
                    T S = 0, Sx = 0, Sy = 0;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int si = (ph + i) % Q;
                        S += bxv[i][qx] * tv[si][qy];
                        Sx += bxd[i][qx] * tv[si][qy];
                        Sy += bxv[i][qx] * td[si][qy];
                    }
                    // chains ordered so that no instruction reads two scalar operands
                    const T S2 = S * S;
                    const T g = a.nld_w[qx] * (S2 * S);
                    T a0 = kyw[qx] * Sy + a.frc_w[qx];
                    a0 += a.rad_w[qx] * (S2 * S2);
                    a0 += a.cs_w[qx] * S;
                    a0 += kxw[qx][qy] * Sx;
                    if constexpr (SRC) {
                        if (eyok)
                            a0 += a.src_w[qx] * a.src[((size_t)ex * Q + qx) * ((size_t)a.nel_y * Q) +
                                                     (size_t)ey * Q + qy];
                    }
                    const T ax = (g + a.dx_w[qx]) * Sx;
                    const T ay = (g + a.dy_w[qx]) * Sy;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int si = (ph + i) % Q;
                        if (i == P && qx == 0) {
                            acc0[si][qy] = a0 * bxv[i][qx] + ax * bxd[i][qx];
                            acc1[si][qy] = ay * bxv[i][qx];
                        } else {
                            acc0[si][qy] += a0 * bxv[i][qx] + ax * bxd[i][qx];
                            acc1[si][qy] += ay * bxv[i][qx];
                        }
                    }
                }
            }
            if (hot) {
                // ignition source and fuel terms (S and fuel re-evaluated).
                // Points by y, then x: each accumulator still receives its
                // contributions in the order of qx.
#pragma unroll
                for (int qy = 0; qy < Q; ++qy) {
                    T tfe[Q];   // the fuel rows' y contraction at qy, by ring slot
#pragma unroll
                    for (int si = 0; si < Q; ++si) tfe[si] = LAZYF ? ytrans_fuel(tf[si], qy) : tf[si][qy];
#pragma unroll
                    for (int qx = 0; qx < Q; ++qx) {
                        T S = 0, F = 0;
#pragma unroll
                        for (int i = 0; i < Q; ++i) {
                            const int si = (ph + i) % Q;
                            S += bxv[i][qx] * tv[si][qy];
                            F += bxv[i][qx] * tfe[si];
                        }
                        T arr = T(0);
                        if (S > a.t_ig && F > a.fthr) arr = S * exp(-a.t_act / S);
                        const T a0 = a.ign_w[qx] * arr;
                        const T af = F * (a.cf_w[qx] - a.rate_w[qx] * arr);
#pragma unroll
                        for (int i = 0; i < Q; ++i) {
                            const int si = (ph + i) % Q;
                            acc0[si][qy] += a0 * bxv[i][qx];
                            if (FUEL) accf[si][qy] += af * bxv[i][qx];
                        }
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < Q; ++s) live[s] = true;
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) acc0[snew][q] = acc1[snew][q] = T(0);
            live[snew] = false;
        }
        if (ex >= X0) {
            // dof row ex (slot ph) is complete: y weights, y half of the test
            // contraction, gather from the p lanes to the left.  A row that no
            // evaluated element reached stores zero (what the contraction of
            // its zero accumulators gives, +0, without evaluating it).
            constexpr int sd = ph;
            T r = T(0), rf = T(0);
            if (live[sd]) {
                T pb[Q], pf[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    acc0[sd][q] *= a.wyq[q];
                    acc1[sd][q] *= a.wyq[q];
                    if (FUEL) accf[sd][q] *= a.wyq[q];
                }
#pragma unroll
                for (int b = 0; b < Q; ++b) {
                    T s0 = 0, s1 = 0;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        s0 += acc0[sd][q] * byv[b][q] + acc1[sd][q] * byd[b][q];
                        if (FUEL) s1 += accf[sd][q] * byv[b][q];
                    }
                    pb[b] = s0;
                    pf[b] = s1;
                }
                r = pb[0] + lane_behind<1>(pb[1]);
                if (FUEL) rf = pf[0] + lane_behind<1>(pf[1]);
                if constexpr (Q > 2) {
                    r += lane_behind<2>(pb[2]);
                    if (FUEL) rf += lane_behind<2>(pf[2]);
                }
                if constexpr (Q > 3) {
                    r += lane_behind<3>(pb[3]);
                    if (FUEL) rf += lane_behind<3>(pf[3]);
                }
            }
            const int hi = ex - X0, ti = ex - X1;
            if (hold && hi < P) {
                hd[hi * 64 + lane] = r;
                if (FUEL) hd[(P + hi) * 64 + lane] = rf;
            } else if (ti >= 0) {
                tl[ti * 64 + lane] = r;
                if (FUEL) tl[(P + ti) * 64 + lane] = rf;
            } else if (lane >= P && colA < Ny) {
                __builtin_nontemporal_store(r, &a.R[(size_t)ex * Ny + colA]);
                if (FUEL) __builtin_nontemporal_store(rf, &a.RF[(size_t)ex * Ny + colA]);
            }
        }
        if (FUEL) {
#pragma unroll
            for (int q = 0; q < Q; ++q) accf[ph][q] = T(0);
        }
    };

    int k = 0;
    // steps whose row fetch lies below rlim: branch-free loads; then the
    // tile's last steps (about Q + p), whose fetches are conditional
    const int Kf = PIPE ? min(K, rlim - E0 - P - Q) : 0;
    for (; k + Q <= Kf; k += Q) {
        step(Ic<0>{}, k, Ic<1>{});
        step(Ic<1>{}, k + 1, Ic<1>{});
        if constexpr (Q > 2) step(Ic<2>{}, k + 2, Ic<1>{});
        if constexpr (Q > 3) step(Ic<3>{}, k + 3, Ic<1>{});
    }
    for (; k + Q <= K; k += Q) {
        step(Ic<0>{}, k, Ic<0>{});
        step(Ic<1>{}, k + 1, Ic<0>{});
        if constexpr (Q > 2) step(Ic<2>{}, k + 2, Ic<0>{});
        if constexpr (Q > 3) step(Ic<3>{}, k + 3, Ic<0>{});
    }
    // fewer than Q steps remain
    if (k < K) step(Ic<0>{}, k, Ic<0>{});
    if constexpr (Q > 2) {
        if (k + 1 < K) step(Ic<1>{}, k + 1, Ic<0>{});
    }
    if constexpr (Q > 3) {
        if (k + 2 < K) step(Ic<2>{}, k + 2, Ic<0>{});
    }
}

// The work of workgroup `grp`: four wavefronts on four consecutive tiles of
// dof rows of one strip.  Stacked (a.stack): only the first evaluates the p
// elements above its tile (the halo); each later wavefront leaves its first
// p dof rows with its own elements' contributions in LDS, its predecessor
// adds the contributions of its last elements to the same rows, and after
// the barrier the later wavefront stores predecessor + own, in that order
// (deterministic, no atomics).  The first tile is p rows shorter than the
// others, so that the four wavefronts march the same number of elements; a
// group covers 4 rows - p dof rows, and a tile shorter than p rows evaluates
// its own halo.  Unstacked: the four wavefronts take neighbouring strips of
// one tile row, every tile evaluates its own halo and no wavefront waits for
// another (better where few wavefronts fit per SIMD).
template <typename T, int P, bool FUEL, bool SRC, bool STK>
__device__ __forceinline__ void assemble_group(const AsmParams<T> &a, const int grp)
{
    constexpr int G = 4;   // wavefronts per workgroup
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // FP32 cubic kernels read the element rows' basis tables from LDS: the
    // 2p + 1 distinct ones (p head, the interior, p tail), copied once per
    // workgroup
    constexpr bool LTAB = sizeof(T) == 4 && P >= 3;   // as in assemble_body
    constexpr int TAB = 2 * (P + 1) * (P + 1);
    __shared__ T ltab[LTAB ? (2 * P + 1) * TAB : 1];
    if constexpr (LTAB) {
        for (int i = threadIdx.x; i < (2 * P + 1) * TAB; i += blockDim.x) {
            const int slot = i / TAB;
            const int e = slot <= P ? slot : a.nel_x - P + (slot - P - 1);
            ltab[i] = a.bx[(size_t)e * TAB + i % TAB];
        }
        __syncthreads();
    }
    if constexpr (!STK) {
        // independent wavefronts: four neighbouring strips of one tile row
        const int gw = grp * G + w;
        if (gw >= a.nstrips * a.ntiles) return;
        const int X0 = (gw / a.nstrips) * a.rows;
        assemble_body<T, P, FUEL, SRC>(a, gw % a.nstrips, X0, min(X0 + a.rows, a.Nx), X0 > 0, false,
                                       false, nullptr, nullptr, ltab);
    } else {
        __shared__ T part[2][G][2 * P * 64];   // [head, tail][wavefront][(T, fuel) x row x lane]
        const int strip = grp % a.nstrips;
        const int base = (grp / a.nstrips) * (G * a.rows - P);
        // dof rows of the tile of wavefront ww (the first is p rows shorter)
        auto first = [&](int ww) { return min(base + (ww == 0 ? 0 : ww * a.rows - P), a.Nx); };
        auto last = [&](int ww) { return min(base + (ww + 1) * a.rows - P, a.Nx); };
        auto holds = [&](int ww) { return ww > 0 && ww < G && first(ww) > 0 && last(ww) - first(ww) >= P; };
        const int X0 = first(w), X1 = last(w);
        const bool live = X1 > X0;
        const bool hold = holds(w);
        const bool halo = live && X0 > 0 && !hold;
        const bool tail = live && holds(w + 1);
        if (live)
            assemble_body<T, P, FUEL, SRC>(a, strip, X0, X1, halo, hold, tail, part[0][w], part[1][w], ltab);
        __syncthreads();
        if (hold) {
            const int lane = threadIdx.x & 63;
            const int colA = strip * (64 - P) - P + lane;
            if (lane >= P && colA < a.Ny) {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const size_t o = (size_t)(X0 + i) * a.Ny + colA;
                    __builtin_nontemporal_store(part[1][w - 1][i * 64 + lane] + part[0][w][i * 64 + lane], &a.R[o]);
                    if (FUEL)
                        __builtin_nontemporal_store(part[1][w - 1][(P + i) * 64 + lane] + part[0][w][(P + i) * 64 + lane], &a.RF[o]);
                }
            }
        }
    }
}

// Occupancy target: float cubic kernels sit a few registers above the 256
// that allow two wavefronts per SIMD; asking for two costs a couple of
// spilled registers and doubles the wavefronts in flight.  Elsewhere the
// compiler's own allocation stands.
template <typename T, int P> struct AsmWaves {
    static constexpr int value = (sizeof(T) == 4 && P == 3) ? 2 : 1;
};

template <typename T, int P, bool FUEL, bool SRC, bool STK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AsmWaves<T, P>::value)))
void k_assemble(AsmParams<T> a)
{
    assemble_group<T, P, FUEL, SRC, STK>(a, blockIdx.x);
}

// Batched launch over the members of an ensemble: workgroup b does workgroup
// info[b].y of member info[b].x (x < 0: no work).
template <typename T, int P, bool FUEL, bool STK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AsmWaves<T, P>::value)))
void k_assemble_batch(const AsmParams<T> *__restrict__ prms, const int2 *__restrict__ info)
{
    const int2 wi = info[blockIdx.x];
    if (wi.x < 0) return;   // the whole workgroup
    assemble_group<T, P, FUEL, false, STK>(prms[wi.x], wi.y);
}

// The ambient fixed point: the temperature c > 0 at which the source of a
// constant field vanishes, c_react c + c_forcing - c_rad c^4 = 0 (the
// ambient temperature of the generic equation at the start of Section 3;
// 300 K with the default coefficients).  Newton from the radiative root.
static bool ambient_fixed_point(const iga_coeffs &c, double &out)
{
    auto g = [&](double t) { return c.c_react * t + c.c_forcing - c.c_rad * t * t * t * t; };
    double t;
    if (c.c_rad > 0 && c.c_forcing > 0) t = std::pow(c.c_forcing / c.c_rad, 0.25);
    else if (c.c_rad == 0 && c.c_react != 0) t = -c.c_forcing / c.c_react;
    else return false;
    for (int it = 0; it < 60 && std::isfinite(t) && t > 0; ++it) {
        const double d = c.c_react - 4.0 * c.c_rad * t * t * t;
        if (d == 0) return false;
        const double step = g(t) / d;
        t -= step;
        if (std::fabs(step) <= 1e-15 * std::fabs(t)) break;
    }
    if (!std::isfinite(t) || !(t > 0)) return false;
    out = t;
    return true;
}

template <typename T>
static void make_params(const iga_plan *pl, int substep, const void *S, const void *F, void *R,
                        void *RF, AsmParams<T> &a, const void *src = nullptr)
{
    const iga_plan_desc &d = pl->d;
    const int P = pl->P, Q = P + 1;
    std::memset(&a, 0, sizeof a);
    a.S = static_cast<const T *>(S);
    a.F = static_cast<const T *>(F);
    a.R = static_cast<T *>(R);
    a.RF = static_cast<T *>(RF);
    a.bx = pl->asm_bx.as<T>();
    a.by = pl->asm_by.as<T>();
    a.wx = pl->asm_wx.as<T>();
    a.wy = pl->asm_wy.as<T>();
    // weights of the explicit (kx_e, ky_e) and implicit (kx_i, ky_i) parts of
    // the linear operator in this substep, and of F (beta)
    double kx_e = 0, ky_e = 0, kx_i = 0, ky_i = 0, beta;
    if (d.scheme == IGA_PR) {
        // substep 0: x implicit, L2 (y) explicit; substep 1: y implicit, L1 (x) explicit
        const double h = 0.5 * d.dt;
        if (substep == 0) { ky_e = h; kx_i = h; }
        else { kx_e = h; ky_i = h; }
        beta = h;
    } else if (d.scheme == IGA_EXPLICIT) {
        // eq. (linear): every term at T^n with weight tau; implicit part M (x) M
        kx_e = ky_e = d.dt;
        beta = d.dt;
    } else {
        // S1 / S3: Crank-Nicolson on L1 over tau/2 (explicit and implicit halves)
        kx_e = kx_i = 0.25 * d.dt;
        beta = 0.5 * d.dt;
    }
    const double react = d.c.c_react;
    double cs, kx, ky, cf;
    if (pl->delta) {
        // increment form: R - (implicit operator) S
        kx = kx_e + kx_i;
        ky = ky_e + ky_i;
        cs = kx * react;
        cf = 0.0;
    } else {
        kx = kx_e;
        ky = ky_e;
        cs = 1.0 + kx * react;
        cf = 1.0;
    }
    const double dx = kx * d.c.c_diff, dy = ky * d.c.c_diff;
    for (int q = 0; q < Q; ++q) {
        const double w = pl->X.wq[q];
        a.wxq[q] = (T)w;
        a.wyq[q] = (T)pl->Y.wq[q];
        a.cs_w[q] = (T)(cs * w);
        a.frc_w[q] = (T)(beta * d.c.c_forcing * w);
        a.rad_w[q] = (T)(-beta * d.c.c_rad * w);
        a.nld_w[q] = (T)(-beta * d.c.c_nld * w);
        a.dx_w[q] = (T)(-dx * w);
        a.dy_w[q] = (T)(-dy * w);
        a.ign_w[q] = (T)(beta * d.c.c_ign * w);
        a.cf_w[q] = (T)(cf * w);
        a.rate_w[q] = (T)(d.dt * d.c.fuel_rate * w);
        a.src_w[q] = (T)(beta * w);
    }
    a.src = static_cast<const T *>(src);
    a.cx = (T)(kx * d.c.c_adv * d.wind.bbar_x);
    a.cy = (T)(ky * d.c.c_adv * d.wind.bbar_y);
    a.bca = (T)(beta * d.c.c_adv);
    a.t_ig = (T)d.c.t_ig;
    // S exceeds the largest coefficient of its element by at most a few
    // roundings of the basis contraction; skip only well below T_ig
    a.t_skip = (T)(d.c.t_ig - 1e-4 * std::fabs(d.c.t_ig));
    a.fthr = (T)d.c.fuel_thr;
    a.t_act = (T)d.c.t_act;
    // Increment form, no sampled source: elements whose coefficients all equal
    // the fixed point in the state's precision are skipped, provided the
    // source left at that rounded value, over a step, is far below the
    // state's resolution there (and the point is below the ignition cut).
    a.amb = 0;
    a.t_fix = T(0);
    double tfix;
    if (pl->delta && !src && ambient_fixed_point(d.c, tfix)) {
        const T tf = (T)tfix;
        const double t = (double)tf;
        const double gres = d.c.c_react * t + d.c.c_forcing - d.c.c_rad * t * t * t * t;
        const double ulp = std::ldexp(t, -std::numeric_limits<T>::digits);
        if (std::fabs(gres) * d.dt <= 1e-3 * ulp && tf < a.t_skip) {
            a.amb = 1;
            a.t_fix = tf;
        }
    }
    a.fuel_all = cf != 0.0;
    a.nel_x = d.nel_x;
    a.nel_y = d.nel_y;
    a.Nx = pl->Nx;
    a.Ny = pl->Ny;
    a.rows = pl->asm_rows;
    a.nstrips = (pl->Ny + (64 - P) - 1) / (64 - P);
    a.stack = pl->asm_stack;
    a.ntiles = (pl->Nx + a.rows - 1) / a.rows;
    a.ngroups = (pl->Nx + 4 * a.rows - P - 1) / (4 * a.rows - P);
}

// workgroups of one assembly launch: four tiles of one strip each (stacked),
// or four wavefronts on neighbouring strips of a tile row
template <typename T> static int asm_groups(const AsmParams<T> &a)
{
    return a.stack ? a.nstrips * a.ngroups : (a.nstrips * a.ntiles + 3) / 4;
}

template <typename T>
static iga_status launch_t(const iga_plan *pl, int substep, const void *S, const void *F, void *R,
                           void *RF, const void *src, hipStream_t s)
{
    AsmParams<T> a;
    make_params<T>(pl, substep, S, F, R, RF, a, src);
    const int P = pl->P;
    const int blocks = asm_groups(a);
    const bool fuel = RF != nullptr;
#define IGA_ASM_S(P_, FU_, SR_)                                                                     \
    do {                                                                                            \
        if (a.stack)                                                                                \
            hipLaunchKernelGGL((k_assemble<T, P_, FU_, SR_, true>), dim3(blocks), dim3(256), 0, s, a); \
        else                                                                                        \
            hipLaunchKernelGGL((k_assemble<T, P_, FU_, SR_, false>), dim3(blocks), dim3(256), 0, s, a); \
    } while (0)
#define IGA_ASM(P_, FU_)              \
    do {                              \
        if (src)                      \
            IGA_ASM_S(P_, FU_, true); \
        else                          \
            IGA_ASM_S(P_, FU_, false); \
    } while (0)
    if (P == 1) {
        if (fuel) IGA_ASM(1, true);
        else IGA_ASM(1, false);
    } else if (P == 2) {
        if (fuel) IGA_ASM(2, true);
        else IGA_ASM(2, false);
    } else if (P == 3) {
        if (fuel) IGA_ASM(3, true);
        else IGA_ASM(3, false);
    } else {
        return fail(IGA_EUNSUPPORTED, "degree not compiled");
    }
#undef IGA_ASM
#undef IGA_ASM_S
    IGA_HIP(hipGetLastError());
    return IGA_OK;
}

iga_status launch_assemble(const iga_plan *pl, int substep, const void *S, const void *F, void *R,
                           void *RF, hipStream_t s, const void *src)
{
    return pl->fp32 ? launch_t<float>(pl, substep, S, F, R, RF, src, s)
                    : launch_t<double>(pl, substep, S, F, R, RF, src, s);
}

template <typename T>
static iga_status batch_t(const std::vector<iga_plan *> &pls, const std::vector<AsmArgs> &args,
                          BatchLaunch &out)
{
    const int P = pls[0]->P;
    const bool fuel = args[0].RF != nullptr;
    std::vector<AsmParams<T>> prms(pls.size());
    std::vector<int2> info;
    for (size_t m = 0; m < pls.size(); ++m) {
        if (pls[m]->P != P || pls[m]->fp32 != pls[0]->fp32 || (args[m].RF != nullptr) != fuel ||
            pls[m]->asm_stack != pls[0]->asm_stack)
            return fail(IGA_EINVAL,
                        "assembly batch: members differ in degree, precision, fuel or tile stacking");
        make_params<T>(pls[m], args[m].substep, args[m].T, args[m].fuel, args[m].R, args[m].RF,
                       prms[m]);
        const int groups = asm_groups(prms[m]);
        for (int g = 0; g < groups; ++g) info.push_back(int2{(int)m, g});
    }
    const void *fn = nullptr;
    const bool stk = pls[0]->asm_stack != 0;
#define IGA_ASMB(P_, FU_)                                                                    \
    fn = stk ? reinterpret_cast<const void *>(k_assemble_batch<T, P_, FU_, true>)           \
             : reinterpret_cast<const void *>(k_assemble_batch<T, P_, FU_, false>)
    if (P == 1) {
        if (fuel) IGA_ASMB(1, true);
        else IGA_ASMB(1, false);
    } else if (P == 2) {
        if (fuel) IGA_ASMB(2, true);
        else IGA_ASMB(2, false);
    } else if (P == 3) {
        if (fuel) IGA_ASMB(3, true);
        else IGA_ASMB(3, false);
    } else {
        return fail(IGA_EUNSUPPORTED, "degree not compiled");
    }
#undef IGA_ASMB
    out.fn = fn;
    out.nblk = (int)info.size();
    out.njobs = 1;
    out.block = 256;
    out.lds = 0;
    IGA_HIP(out.prm.alloc(prms.size() * sizeof(AsmParams<T>)));
    IGA_HIP(out.info.alloc(info.size() * sizeof(int2)));
    IGA_HIP(hipMemcpy(out.prm.ptr, prms.data(), prms.size() * sizeof(AsmParams<T>),
                      hipMemcpyHostToDevice));
    IGA_HIP(hipMemcpy(out.info.ptr, info.data(), info.size() * sizeof(int2), hipMemcpyHostToDevice));
    return IGA_OK;
}

iga_status build_assemble_batch(const std::vector<iga_plan *> &pls, const std::vector<AsmArgs> &args,
                                BatchLaunch &out)
{
    if (pls.empty() || args.size() != pls.size()) return fail(IGA_EINVAL, "assembly batch: members");
    return pls[0]->fp32 ? batch_t<float>(pls, args, out) : batch_t<double>(pls, args, out);
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
