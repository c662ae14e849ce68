// plan.cpp -- host side of a plan: knot vectors, Gauss rules, B-spline basis
// tables at the quadrature points, the 1D matrices M, K, G of Section 3.1 and
// the directional operators of the two schemes, and their upload.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "iga_internal.h"

namespace iga {

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1, 1] by Newton's method on P_n, started from the
// asymptotic node estimates cos(pi (i + 3/4) / (n + 1/2)).
// ---------------------------------------------------------------------------
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;   // P_0, P_1
            if (n == 0) p1 = 1.0;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            // P_n = p1, P_{n-1} = p0; P_n' = n (z P_n - P_{n-1}) / (z^2 - 1)
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Values and first derivatives of the p+1 B-splines N_{s-p} .. N_s that are
// non-zero in knot span [t_s, t_{s+1}), by the triangular recurrence of
// de Boor: ndu[r][j] (r <= j) are the degree-j values, ndu[j][r] (r < j) the
// knot differences they divide by.
static void basis_ders(const std::vector<double> &t, int s, int p, double x, double *val,
                       double *der)
{
    double left[4], right[4], ndu[4][4];
    ndu[0][0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            ndu[j][r] = right[r + 1] + left[j - r];
            double temp = ndu[r][j - 1] / ndu[j][r];
            ndu[r][j] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        ndu[j][j] = saved;
    }
    for (int r = 0; r <= p; ++r) {
        val[r] = ndu[r][p];
        double d = 0.0;
        if (r >= 1) d += ndu[r - 1][p - 1] / ndu[p][r - 1];
        if (r <= p - 1) d -= ndu[r][p - 1] / ndu[p][r];
        der[r] = p * d;
    }
}

static void build_dir(DirHost &D, int n, int p, double L)
{
    D.n = n;
    D.N = n + p;
    D.L = L;
    D.h = L / n;
    D.knots.assign(n + 2 * p + 1, 0.0);
    for (int k = 0; k < n + 2 * p + 1; ++k) {
        int e = std::min(std::max(k - p, 0), n);
        D.knots[k] = (e == n) ? L : L * e / n;
    }
    std::vector<double> gx, gw;
    gauss_legendre(p + 1, gx, gw);
    const int nq = p + 1, W = 2 * p + 1;
    D.bv.assign((size_t)n * nq * nq, 0.0);
    D.bd.assign((size_t)n * nq * nq, 0.0);
    D.xq.assign((size_t)n * nq, 0.0);
    D.wq.assign(nq, 0.0);
    for (int q = 0; q < nq; ++q) D.wq[q] = gw[q] * 0.5 * D.h;
    D.M.assign((size_t)D.N * W, 0.0);
    D.K.assign((size_t)D.N * W, 0.0);
    D.G.assign((size_t)D.N * W, 0.0);
    for (int e = 0; e < n; ++e) {
        double a = D.knots[p + e], b = D.knots[p + e + 1];
        for (int q = 0; q < nq; ++q) {
            double x = a + 0.5 * (gx[q] + 1.0) * (b - a);
            D.xq[(size_t)e * nq + q] = x;
            double v[4], dv[4];
            basis_ders(D.knots, p + e, p, x, v, dv);
            for (int r = 0; r <= p; ++r) {
                D.bv[((size_t)e * nq + r) * nq + q] = v[r];
                D.bd[((size_t)e * nq + r) * nq + q] = dv[r];
            }
            // element contributions to M, K, G (row = test function)
            for (int r = 0; r <= p; ++r)
                for (int c = 0; c <= p; ++c) {
                    size_t idx = (size_t)(e + r) * W + (c - r + p);
                    D.M[idx] += D.wq[q] * v[r] * v[c];
                    D.K[idx] += D.wq[q] * dv[r] * dv[c];
                    D.G[idx] += D.wq[q] * v[r] * dv[c];
                }
        }
    }
}

// gamma and the reaction share of the implicit operator along dir
// (eq. varPR_wildfire: tau/2 both directions; eq. varCN: tau/4 along x and
// tau/2 along y; the linear reaction belongs to L1, the x operator).
static void op_params(const iga_plan *pl, int dir, double &g, double &react)
{
    if (pl->d.scheme == IGA_PR) g = 0.5 * pl->d.dt;
    else g = dir == 0 ? 0.25 * pl->d.dt : 0.5 * pl->d.dt;
    react = dir == 0 ? pl->d.c.c_react : 0.0;
}

iga_status build_plan_host(iga_plan *pl)
{
    const iga_plan_desc &d = pl->d;
    pl->P = d.p;
    build_dir(pl->X, d.nel_x, d.p, d.len_x);
    build_dir(pl->Y, d.nel_y, d.p, d.len_y);
    pl->Nx = pl->X.N;
    pl->Ny = pl->Y.N;
    pl->ndof = (size_t)pl->Nx * pl->Ny;
    pl->fp32 = d.precision == IGA_FP32_REFINE;
    pl->wsize = pl->fp32 ? 4 : 8;
    for (int dir = 0; dir < 2; ++dir) {
        const DirHost &D = dir ? pl->Y : pl->X;
        double g, react;
        op_params(pl, dir, g, react);
        double bbar = dir ? d.wind.bbar_y : d.wind.bbar_x;
        size_t n = D.M.size();
        std::vector<double> A(n), M(D.M), B(n);
        for (size_t k = 0; k < n; ++k) {
            double lin = d.c.c_diff * D.K[k] + d.c.c_adv * bbar * D.G[k];
            A[k] = (1.0 - g * react) * D.M[k] + g * lin;
            B[k] = (1.0 + g * react) * D.M[k] - g * lin;
        }
        pl->op_band[dir ? OP_AY : OP_AX] = A;
        pl->op_band[dir ? OP_MY : OP_MX] = M;
        pl->cn_band[dir ? BAND_BY : BAND_BX] = B;
    }
    return IGA_OK;
}

template <typename T> static std::vector<T> cast_vec(const std::vector<double> &v)
{
    return std::vector<T>(v.begin(), v.end());
}

static iga_status upload(DevBuf &b, const void *src, size_t bytes)
{
    IGA_HIP(b.alloc(bytes));
    IGA_HIP(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice));
    return IGA_OK;
}

template <typename T> static iga_status upload_vec(DevBuf &b, const std::vector<double> &v)
{
    std::vector<T> c = cast_vec<T>(v);
    return upload(b, c.data(), c.size() * sizeof(T));
}

// Assembly tables of one direction: per element e, [0][a][q] values and
// [1][a][q] derivatives of the element's p+1 functions at its p+1 points.
static std::vector<double> asm_table(const DirHost &D, int p)
{
    int nq = p + 1;
    std::vector<double> t((size_t)D.n * 2 * nq * nq);
    for (int e = 0; e < D.n; ++e)
        for (int a = 0; a < nq; ++a)
            for (int q = 0; q < nq; ++q) {
                t[(((size_t)e * 2 + 0) * nq + a) * nq + q] = D.bv[((size_t)e * nq + a) * nq + q];
                t[(((size_t)e * 2 + 1) * nq + a) * nq + q] = D.bd[((size_t)e * nq + a) * nq + q];
            }
    return t;
}

iga_status upload_plan(iga_plan *pl)
{
    const int p = pl->P, nq = p + 1;
    const iga_plan_desc &d = pl->d;
    iga_status st;
    for (int op = 0; op < NOPS; ++op) {
        if ((st = upload_vec<double>(pl->op_a64[op], pl->op_band[op]))) return st;
    }
    for (int b = 0; b < NBANDS; ++b) {
        st = pl->fp32 ? upload_vec<float>(pl->cn_dev[b], pl->cn_band[b])
                      : upload_vec<double>(pl->cn_dev[b], pl->cn_band[b]);
        if (st) return st;
    }
    std::vector<double> tx = asm_table(pl->X, p), ty = asm_table(pl->Y, p);
    // explicit wind remainders: (by(x) - bbar_y) at x-points, (bx(y) - bbar_x) at y-points
    std::vector<double> wx((size_t)pl->X.n * nq), wy((size_t)pl->Y.n * nq);
    const bool sc = d.wind.kind == IGA_WIND_SINCOS;
    for (int e = 0; e < pl->X.n; ++e)
        for (int q = 0; q < nq; ++q) {
            double x = pl->X.xq[(size_t)e * nq + q];
            double by = d.wind.by + (sc ? d.wind.ay * std::cos(2.0 * M_PI * x / d.len_x) : 0.0);
            wx[(size_t)e * nq + q] = by - d.wind.bbar_y;
        }
    for (int e = 0; e < pl->Y.n; ++e)
        for (int q = 0; q < nq; ++q) {
            double y = pl->Y.xq[(size_t)e * nq + q];
            double bx = d.wind.bx + (sc ? d.wind.ax * std::sin(2.0 * M_PI * y / d.len_y) : 0.0);
            wy[(size_t)e * nq + q] = bx - d.wind.bbar_x;
        }
    if (pl->fp32) {
        if ((st = upload_vec<float>(pl->asm_bx, tx))) return st;
        if ((st = upload_vec<float>(pl->asm_by, ty))) return st;
        if ((st = upload_vec<float>(pl->asm_wx, wx))) return st;
        if ((st = upload_vec<float>(pl->asm_wy, wy))) return st;
    } else {
        if ((st = upload_vec<double>(pl->asm_bx, tx))) return st;
        if ((st = upload_vec<double>(pl->asm_by, ty))) return st;
        if ((st = upload_vec<double>(pl->asm_wx, wx))) return st;
        if ((st = upload_vec<double>(pl->asm_wy, wy))) return st;
    }
    IGA_HIP(pl->scratch_r.alloc(pl->ndof * pl->wsize));
    IGA_HIP(pl->scratch_rf.alloc(pl->ndof * pl->wsize));
    IGA_HIP(pl->flag.alloc(64));
    for (int dir = 0; dir < 2; ++dir) {
        int N = dir ? pl->Ny : pl->Nx;
        int lines = dir ? pl->Nx : pl->Ny;
        (void)lines;
        for (int op = 0; op < NOPS; ++op) {
            if ((op == OP_AX || op == OP_MX) != (dir == 0)) continue;
            IGA_HIP(pl->op_lf64[op].alloc((size_t)N * p * 8));
            IGA_HIP(pl->op_uf64[op].alloc((size_t)N * (p + 1) * 8));
            if (pl->fp32) {
                IGA_HIP(pl->op_lf32[op].alloc((size_t)N * p * 4));
                IGA_HIP(pl->op_uf32[op].alloc((size_t)N * (p + 1) * 4));
            }
        }
    }
    return IGA_OK;
}

// ---------------------------------------------------------------------------
// line-solve schedules
// ---------------------------------------------------------------------------
static bool fill_schedule(const iga_plan *pl, int dir, int lw, int waves, int mm, Schedule &sc)
{
    const int N = dir ? pl->Ny : pl->Nx, p = pl->P;
    if (!sweep_compiled(p, lw, mm)) return false;
    if ((waves * 64) % lw) return false;
    int C = waves * 64 / lw;
    int m = (N + C - 1) / C;
    if (m < p) m = p;
    // the last non-empty chunk must hold at least p rows (neighbour exchange)
    while (m <= mm) {
        int used = (N + m - 1) / m;
        int last = N - (used - 1) * m;
        if (last >= p) break;
        ++m;
    }
    if (m > mm) return false;
    sc.lw = lw;
    sc.waves = waves;
    sc.mm = mm;
    sc.m = m;
    sc.chunks = C;
    int lev = 0;
    while ((1 << lev) < C) ++lev;
    sc.levels = lev;
    if (sweep_lds_bytes(pl, dir, sc) > 160 * 1024) return false;
    return true;
}

iga_status choose_schedule(iga_plan *pl, int dir, int lw, int waves)
{
    static const int mms[] = {16, 32, 48};
    Schedule best;
    bool found = false;
    if (lw > 0) {
        for (int mm : mms)
            if (fill_schedule(pl, dir, lw, waves, mm, best)) { found = true; break; }
        if (!found)
            return fail(IGA_EUNSUPPORTED, "line-solve schedule lw=" + std::to_string(lw) +
                                              " waves=" + std::to_string(waves) +
                                              " does not fit this line length / precision");
        pl->sched[dir] = best;
        return sweep_prepare(pl, dir);
    }
    // default heuristic: widest line group that fits, with 16 waves, the
    // smallest register capacity; narrower for long lines.
    const int N = dir ? pl->Ny : pl->Nx;
    const int nlines = dir ? pl->Nx : pl->Ny;
    static const int lws_long[] = {16, 8, 64};
    static const int lws_short[] = {64, 16, 8};
    const int *lws = (nlines >= 256 && N >= 256) ? lws_long : lws_short;
    for (int i = 0; i < 3 && !found; ++i)
        for (int w : {16, 8, 4}) {
            if (found) break;
            for (int mm : mms)
                if (fill_schedule(pl, dir, lws[i], w, mm, best)) { found = true; break; }
        }
    if (!found) return fail(IGA_EUNSUPPORTED, "no compiled line-solve schedule fits lines of " +
                                                  std::to_string(N) + " dofs");
    pl->sched[dir] = best;
    return sweep_prepare(pl, dir);
}

OpDev op_dev(const iga_plan *pl, int op)
{
    OpDev o;
    if (pl->fp32) {
        o.lf = pl->op_lf32[op].ptr;
        o.uf = pl->op_uf32[op].ptr;
        o.tf = pl->op_tf32[op].ptr;
        o.tb = pl->op_tb32[op].ptr;
    } else {
        o.lf = pl->op_lf64[op].ptr;
        o.uf = pl->op_uf64[op].ptr;
        o.tf = pl->op_tf64[op].ptr;
        o.tb = pl->op_tb64[op].ptr;
    }
    o.a64 = pl->op_a64[op].as<double>();
    return o;
}

}  // namespace iga
