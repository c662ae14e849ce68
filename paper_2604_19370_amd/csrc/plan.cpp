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
    // Basis functions are evaluated in element-local coordinates: on a uniform
    // knot vector the knots seen from element e are exact multiples of h, so
    // every interior element gets bitwise the same tables (and the interior
    // rows of M, K, G are exactly Toeplitz) with no cancellation at large x.
    std::vector<double> tl(n + 2 * p + 1);
    for (int e = 0; e < n; ++e) {
        for (int k = 0; k < n + 2 * p + 1; ++k)
            tl[k] = (double)(std::min(std::max(k - p, 0), n) - e) * D.h;
        for (int q = 0; q < nq; ++q) {
            const double xl = 0.5 * (gx[q] + 1.0) * D.h;
            D.xq[(size_t)e * nq + q] = D.knots[p + e] + xl;
            double v[4], dv[4];
            basis_ders(tl, p + e, p, xl, v, dv);
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
// tau/2 along y; the linear reaction belongs to L1, the x operator).  The
// explicit scheme inverts the mass matrices only (gamma = 0).
static void op_params(const iga_plan *pl, int dir, double &g, double &react)
{
    if (pl->d.scheme == IGA_PR) g = 0.5 * pl->d.dt;
    else if (pl->d.scheme == IGA_EXPLICIT) g = 0.0;
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
    pl->delta = pl->fp32;
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
            // explicit Crank-Nicolson counterpart B = (1 + g react) M - g (...);
            // in increment form the line solve applies B - A = 2 g (react M - (...))
            B[k] = pl->delta ? 2.0 * g * (react * D.M[k] - lin)
                             : (1.0 + g * react) * D.M[k] - g * lin;
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

static iga_status upload_state(const iga_plan *pl, DevBuf &b, const std::vector<double> &v)
{
    return pl->fp32 ? upload_vec<float>(b, v) : upload_vec<double>(b, v);
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
    for (int op = 0; op < NOPS; ++op)
        if ((st = upload_vec<double>(pl->op_a64[op], pl->op_band[op]))) return st;
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
    if ((st = upload_state(pl, pl->asm_bx, tx))) return st;
    if ((st = upload_state(pl, pl->asm_by, ty))) return st;
    if ((st = upload_state(pl, pl->asm_wx, wx))) return st;
    if ((st = upload_state(pl, pl->asm_wy, wy))) return st;
    IGA_HIP(pl->scratch_r.alloc(pl->ndof * pl->wsize));
    IGA_HIP(pl->scratch_rf.alloc(pl->ndof * pl->wsize));
    if (pl->fp32) {
        // out-of-place x solves (column waves)
        IGA_HIP(pl->scratch_r2.alloc(pl->ndof * pl->wsize));
        IGA_HIP(pl->scratch_rf2.alloc(pl->ndof * pl->wsize));
    }
    IGA_HIP(pl->flag.alloc(64));
    for (int op = 0; op < NOPS; ++op) {
        const int N = op_dir(op) ? pl->Ny : pl->Nx;
        IGA_HIP(pl->op_lf64[op].alloc((size_t)N * p * 8));
        IGA_HIP(pl->op_uf64[op].alloc((size_t)N * (p + 1) * 8));
    }
    return IGA_OK;
}

// ---------------------------------------------------------------------------
// line-solve tables: compressed coefficient rows and chunk scan tables
// ---------------------------------------------------------------------------
// Rows of `f` (stride RS, N rows) that agree with the middle row to `rtol`
// form the interior [K0, NK).
static void interior_range(const std::vector<double> &f, int N, int RS, double rtol, int &K0,
                           int &NK)
{
    const int mid = N / 2;
    auto same = [&](int r) {
        for (int i = 0; i < RS; ++i) {
            const double a = f[(size_t)r * RS + i], b = f[(size_t)mid * RS + i];
            if (std::fabs(a - b) > rtol * std::fabs(b)) return false;
        }
        return true;
    };
    K0 = 0;
    for (int r = mid - 1; r >= 0; --r)
        if (!same(r)) { K0 = r + 1; break; }
    NK = N;
    for (int r = mid + 1; r < N; ++r)
        if (!same(r)) { NK = r; break; }
}

static std::vector<double> compress_rows(const std::vector<double> &f, int N, int RS, int K0, int NK)
{
    std::vector<double> out;
    out.reserve((size_t)(K0 + 1 + N - NK) * RS);
    for (int r = 0; r < K0; ++r) out.insert(out.end(), f.begin() + (size_t)r * RS, f.begin() + (size_t)(r + 1) * RS);
    const int c = std::min(K0, N - 1);
    out.insert(out.end(), f.begin() + (size_t)c * RS, f.begin() + (size_t)(c + 1) * RS);
    for (int r = NK; r < N; ++r) out.insert(out.end(), f.begin() + (size_t)r * RS, f.begin() + (size_t)(r + 1) * RS);
    return out;
}

// table row of line row r (the kernels' mapping): rows below K0 and from NK
// on are stored, the interior shares row K0, padding rows map to the last row
static inline int row_of(int r, int K0, int NK, int nrows)
{
    return std::min(std::min(r, K0) + std::max(0, r - NK + 1), nrows - 1);
}

// Forward / backward chunk transfer matrices for the 64 chunks of length m
// (products of the companion matrices of forward and backward substitution,
// from the compressed rows the kernels use; rows past N are the identity
// padding rows).  The line-solve kernels compose them along their scan.
static void scan_tables(OpHost &o, int N, int P, int m, int C)
{
    const int RS = 2 * P + 2, PP = P * P;
    std::vector<double> F((size_t)C * PP), B((size_t)C * PP);
    for (int c = 0; c < C; ++c) {
        std::vector<double> f(PP, 0.0), b(PP, 0.0);
        for (int i = 0; i < P; ++i) f[i * P + i] = b[i * P + i] = 1.0;
        const int r0 = c * m, r1 = r0 + m;
        (void)N;
        for (int r = r0; r < r1; ++r) {           // f <- C_r f
            const double *L = &o.rows[(size_t)row_of(r, o.K0, o.NK, o.nrows) * RS];
            std::vector<double> nf(PP, 0.0);
            for (int j = 0; j < P; ++j) {
                double s = 0.0;
                for (int k = 0; k < P; ++k) s -= L[k] * f[k * P + j];
                nf[j] = s;
            }
            for (int i = 1; i < P; ++i)
                for (int j = 0; j < P; ++j) nf[i * P + j] = f[(i - 1) * P + j];
            f.swap(nf);
        }
        for (int r = r1 - 1; r >= r0; --r) {      // b <- D_r b
            const double *U = &o.rows[(size_t)row_of(r, o.K0, o.NK, o.nrows) * RS + P];
            std::vector<double> nb(PP, 0.0);
            for (int j = 0; j < P; ++j) {
                double s = 0.0;
                for (int k = 0; k < P; ++k) s -= U[1 + k] * b[k * P + j];
                nb[j] = s;
            }
            for (int i = 1; i < P; ++i)
                for (int j = 0; j < P; ++j) nb[i * P + j] = b[(i - 1) * P + j];
            b.swap(nb);
        }
        std::copy(f.begin(), f.end(), F.begin() + (size_t)c * PP);
        std::copy(b.begin(), b.end(), B.begin() + (size_t)c * PP);
    }
    o.tf = F;
    o.tb = B;
}

// chunk transfer matrices of the current schedule of direction dir
iga_status build_scan_tables(iga_plan *pl, int dir)
{
    const Schedule &sc = pl->sched[dir];
    const int N = dir ? pl->Ny : pl->Nx;
    iga_status st;
    for (int op = 0; op < NOPS; ++op) {
        if (op_dir(op) != dir) continue;
        OpHost &o = pl->op_host[op];
        if (o.rows.empty()) continue;   // not factored yet
        scan_tables(o, N, pl->P, sc.mm, 64 * sc.wpl);
        if ((st = upload_state(pl, pl->op_tf[op], o.tf))) return st;
        if ((st = upload_state(pl, pl->op_tb[op], o.tb))) return st;
    }
    return IGA_OK;
}

// ---------------------------------------------------------------------------
// windowed solves: warm-up length and strip tables
// ---------------------------------------------------------------------------
// Forward substitution carries the state (y_r, .., y_{r-P+1}) through the
// companion matrices C_r of the L rows; backward substitution carries
// (x_r, .., x_{r+P-1}) through those of the scaled U rows.  Restarting either
// from a zero state h rows early perturbs the result by the product of h
// such matrices applied to the true state.  The warm-up is the smallest h
// whose products from every start (head rows, the canonical interior, tail
// rows) have infinity norm <= tol; 0 if none up to hmax.
static int compute_warmup(const OpHost &o, int N, int P, double tol, int hmax)
{
    const int RS = 2 * P + 2;
    auto row = [&](int r) { return &o.rows[(size_t)row_of(r, o.K0, o.NK, o.nrows) * RS]; };
    auto worst = [&](bool fwd) {
        std::vector<int> starts;
        for (int s = 0; s < std::min(N, o.K0 + hmax + 2); ++s) starts.push_back(s);
        for (int s = std::max(0, o.NK - hmax - 2); s < N; ++s) starts.push_back(s);
        int h_need = 0;
        for (int s : starts) {
            std::vector<double> m((size_t)P * P, 0.0), n((size_t)P * P);
            for (int i = 0; i < P; ++i) m[(size_t)i * P + i] = 1.0;
            int h = 0;
            for (;;) {
                const int r = fwd ? s + h : s - h;
                if (r < 0 || r >= N) break;   // reached the line end: exact from here
                const double *c = row(r);
                // n = C_r m
                for (int j = 0; j < P; ++j) {
                    double v = 0.0;
                    for (int k = 0; k < P; ++k) v -= (fwd ? c[k] : c[P + 1 + k]) * m[(size_t)k * P + j];
                    n[j] = v;
                }
                for (int i = 1; i < P; ++i)
                    for (int j = 0; j < P; ++j) n[(size_t)i * P + j] = m[(size_t)(i - 1) * P + j];
                m.swap(n);
                ++h;
                double nrm = 0.0;
                for (int i = 0; i < P; ++i) {
                    double rs = 0.0;
                    for (int j = 0; j < P; ++j) rs += std::fabs(m[(size_t)i * P + j]);
                    nrm = std::max(nrm, rs);
                }
                if (nrm <= tol) break;
                if (h > hmax) return hmax + 1;
            }
            h_need = std::max(h_need, h);
        }
        return h_need;
    };
    const int h = std::max(worst(true), worst(false));
    return h > hmax ? 0 : h;
}

int warmup_rows(const iga_plan *pl, int dir)
{
    int h = 0;
    for (int op = 0; op < NOPS; ++op) {
        if (op_dir(op) != dir) continue;
        if (pl->op_host[op].H <= 0) return 0;
        h = std::max(h, pl->op_host[op].H);
    }
    return (h + 3) & ~3;   // the kernels' warm-up loops step by 4 rows
}

// warm-up rows of the correction solve of FP32 refinement (<= warmup_rows)
static int correction_warmup_rows(const iga_plan *pl, int dir)
{
    int h = 0;
    for (int op = 0; op < NOPS; ++op)
        if (op_dir(op) == dir) h = std::max(h, pl->op_host[op].Hc);
    return std::min((h + 3) & ~3, warmup_rows(pl, dir));
}

// Geometry of the windowed tables of direction dir for rows-per-lane mm and
// wpl wavefronts per line (H = 0 if windowed solves are not possible).
WinGeom window_geometry(const iga_plan *pl, int dir, int mm, int wpl)
{
    const int N = dir ? pl->Ny : pl->Nx;
    const int H = warmup_rows(pl, dir);
    WinGeom g;
    if (H <= 0) return g;
    const int lanes = 64 * wpl;
    g.H = H;
    g.Hc = pl->fp32 ? correction_warmup_rows(pl, dir) : H;
    g.tail1 = std::min(lanes, (N + mm - 1) / mm);
    // rows that are canonical in every table of the direction
    int K0 = 0, NK = N;
    for (int op = 0; op < NOPS; ++op)
        if (op_dir(op) == dir) {
            K0 = std::max(K0, pl->op_host[op].K0);
            NK = std::min(NK, pl->op_host[op].NK);
        }
    for (int b = 0; b < NBANDS; ++b)
        if ((b == BAND_BX ? 0 : 1) == dir) {
            K0 = std::max(K0, pl->band_host[b].K0);
            NK = std::min(NK, pl->band_host[b].NK);
        }
    // lane c is canonical iff rows [c mm - H, c mm + mm + H) lie in [K0, NK)
    g.nhead = std::min(g.tail1, (K0 + H + mm - 1) / mm);
    const int t0 = (NK - H - mm) >= 0 ? (NK - H - mm) / mm + 1 : 0;
    g.tail0 = std::min(g.tail1, std::max(g.nhead, t0));
    const int win = 2 * H + mm;
    const int hrows = g.nhead > 0 ? g.nhead * mm + 2 * H : 0;
    const int trows = g.tail1 > g.tail0 ? (g.tail1 - g.tail0) * mm + 2 * H : 0;
    g.off_head = 0;
    g.off_tail = hrows;
    g.off_canon = hrows + trows;
    g.off_id = g.off_canon + win;
    g.nrows = g.off_id + win;
    g.aoff_head = 0;
    g.aoff_tail = g.nhead * mm;
    g.aoff_canon = g.aoff_tail + (g.tail1 - g.tail0) * mm;
    g.aoff_id = g.aoff_canon + mm;
    g.anrows = g.aoff_id + mm;
    return g;
}

// Strip tables of direction dir for the current windowed schedule.
iga_status build_window_tables(iga_plan *pl, int dir)
{
    const Schedule &sc = pl->sched[dir];
    const int N = dir ? pl->Ny : pl->Nx, P = pl->P, RS = 2 * P + 2, mm = sc.mm;
    const WinGeom g = window_geometry(pl, dir, mm, sc.wpl);
    if (g.H <= 0 || !sc.win) return fail(IGA_EUNSUPPORTED, "no windowed solve for this direction");
    const int H = g.H;
    pl->wgeom[dir] = g;
    int K0 = 0, NK = N;
    for (int op = 0; op < NOPS; ++op)
        if (op_dir(op) == dir) {
            K0 = std::max(K0, pl->op_host[op].K0);
            NK = std::min(NK, pl->op_host[op].NK);
        }
    for (int b = 0; b < NBANDS; ++b)
        if ((b == BAND_BX ? 0 : 1) == dir) {
            K0 = std::max(K0, pl->band_host[b].K0);
            NK = std::min(NK, pl->band_host[b].NK);
        }
    const int win = 2 * H + mm;
    const int hrows = g.off_tail - g.off_head, trows = g.off_canon - g.off_tail;
    const int ahrows = g.aoff_tail - g.aoff_head, atrows = g.aoff_canon - g.aoff_tail;
    (void)NK;
    // table content: line rows r (identity / zero rows outside [0, N)); the
    // canonical window repeats line row rc (inside [K0, NK) when there is an
    // interior; unused otherwise)
    const int rc = std::min(K0, N - 1);
    auto fill = [&](std::vector<double> &t, int nrows, int off, int r_first, int count,
                    auto &&rowfn) {
        (void)nrows;
        for (int i = 0; i < count; ++i) rowfn(r_first + i, &t[(size_t)(off + i) * RS]);
    };
    iga_status st;
    for (int op = 0; op < NOPS; ++op) {
        if (op_dir(op) != dir) continue;
        const OpHost &o = pl->op_host[op];
        auto lu_row = [&](int r, double *dst) {
            if (r < 0 || r >= N) {
                std::fill(dst, dst + RS, 0.0);
                dst[P] = 1.0;
            } else {
                const double *src = &o.rows[(size_t)row_of(r, o.K0, o.NK, o.nrows) * RS];
                std::copy(src, src + RS, dst);
            }
        };
        auto a_row = [&](int r, double *dst) {
            if (r >= N) {
                std::fill(dst, dst + RS, 0.0);
                dst[P] = 1.0;
            } else {
                const double *src = &o.a64[(size_t)row_of(r, o.K0, o.NK, o.nrows) * RS];
                std::copy(src, src + RS, dst);
            }
        };
        OpHost &ow = pl->op_host[op];
        ow.wrows.assign((size_t)g.nrows * RS, 0.0);
        fill(ow.wrows, g.nrows, g.off_head, -H, hrows, lu_row);
        fill(ow.wrows, g.nrows, g.off_tail, g.tail0 * mm - H, trows, lu_row);
        for (int i = 0; i < win; ++i) lu_row(rc, &ow.wrows[(size_t)(g.off_canon + i) * RS]);
        for (int i = 0; i < win; ++i) lu_row(-1, &ow.wrows[(size_t)(g.off_id + i) * RS]);
        ow.wa64.assign((size_t)g.anrows * RS, 0.0);
        fill(ow.wa64, g.anrows, g.aoff_head, 0, ahrows, a_row);
        fill(ow.wa64, g.anrows, g.aoff_tail, g.tail0 * mm, atrows, a_row);
        for (int i = 0; i < mm; ++i) a_row(rc, &ow.wa64[(size_t)(g.aoff_canon + i) * RS]);
        for (int i = 0; i < mm; ++i) a_row(N, &ow.wa64[(size_t)(g.aoff_id + i) * RS]);
        if ((st = upload_state(pl, pl->op_wrows[op], ow.wrows))) return st;
        if (pl->fp32 && (st = upload_vec<double>(pl->op_wa64[op], ow.wa64))) return st;
    }
    for (int b = 0; b < NBANDS; ++b) {
        if ((b == BAND_BX ? 0 : 1) != dir) continue;
        BandHost &o = pl->band_host[b];
        auto b_row = [&](int r, double *dst) {
            if (r >= N) {
                std::fill(dst, dst + RS, 0.0);
            } else {
                const double *src = &o.rows[(size_t)row_of(r, o.K0, o.NK, o.nrows) * RS];
                std::copy(src, src + RS, dst);
            }
        };
        o.wrows.assign((size_t)g.anrows * RS, 0.0);
        fill(o.wrows, g.anrows, g.aoff_head, 0, ahrows, b_row);
        fill(o.wrows, g.anrows, g.aoff_tail, g.tail0 * mm, atrows, b_row);
        for (int i = 0; i < mm; ++i) b_row(rc, &o.wrows[(size_t)(g.aoff_canon + i) * RS]);
        for (int i = 0; i < mm; ++i) b_row(N, &o.wrows[(size_t)(g.aoff_id + i) * RS]);
        if ((st = upload_state(pl, pl->band_wrows[b], o.wrows))) return st;
    }
    return IGA_OK;
}

iga_status build_solve_tables(iga_plan *pl)
{
    const int P = pl->P, RS = 2 * P + 2, W = 2 * P + 1;
    // agreement of interior rows: a few ulp of double (factors converge
    // geometrically; the assembled interior rows are exactly Toeplitz)
    const double rtol = 1e-15;
    iga_status st;
    for (int op = 0; op < NOPS; ++op) {
        const int dir = op_dir(op), N = dir ? pl->Ny : pl->Nx;
        std::vector<double> lf((size_t)N * P), uf((size_t)N * (P + 1));
        IGA_HIP(hipMemcpy(lf.data(), pl->op_lf64[op].ptr, lf.size() * 8, hipMemcpyDeviceToHost));
        IGA_HIP(hipMemcpy(uf.data(), pl->op_uf64[op].ptr, uf.size() * 8, hipMemcpyDeviceToHost));
        std::vector<double> f((size_t)N * RS, 0.0), a((size_t)N * RS, 0.0);
        for (int r = 0; r < N; ++r) {
            for (int j = 0; j < P; ++j) f[(size_t)r * RS + j] = lf[(size_t)r * P + j];
            for (int j = 0; j <= P; ++j) f[(size_t)r * RS + P + j] = uf[(size_t)r * (P + 1) + j];
            for (int j = 0; j < W; ++j) a[(size_t)r * RS + j] = pl->op_band[op][(size_t)r * W + j];
        }
        int K0f, NKf, K0a, NKa;
        interior_range(f, N, RS, rtol, K0f, NKf);
        interior_range(a, N, RS, rtol, K0a, NKa);
        OpHost &o = pl->op_host[op];
        o.K0 = std::max(K0f, K0a);
        o.NK = std::min(NKf, NKa);
        if (o.NK <= o.K0) { o.K0 = N; o.NK = N; }   // no interior: keep every row
        o.rows = compress_rows(f, N, RS, o.K0, o.NK);
        o.a64 = compress_rows(a, N, RS, o.K0, o.NK);
        // identity row for the padding rows past N
        std::vector<double> id(RS, 0.0);
        id[P] = 1.0;
        o.rows.insert(o.rows.end(), id.begin(), id.end());
        id.assign(RS, 0.0);
        id[P] = 1.0;
        o.a64.insert(o.a64.end(), id.begin(), id.end());
        o.nrows = (int)(o.rows.size() / RS);
        if ((st = upload_state(pl, pl->op_rows[op], o.rows))) return st;
        if ((st = upload_vec<double>(pl->op_a64c[op], o.a64))) return st;
        // windowed solves: below float resolution of the refined FP32 solve,
        // below double rounding otherwise
        // FP64: the truncated recurrences reach 2^-55.  FP32 plans (increment
        // form, one FP64-residual refinement per line solve): the first solve
        // needs float accuracy (2^-20; what it misses is in the residual) and
        // the correction, a few bits (2^-12), so that
        // |x - x*| <~ eps32 |x| + 2^-20 * 2^-12 |x|.
        o.H = compute_warmup(o, N, P, pl->fp32 ? std::ldexp(1.0, -20) : std::ldexp(1.0, -55), 96);
        o.Hc = pl->fp32 ? compute_warmup(o, N, P, std::ldexp(1.0, -12), 96) : o.H;
    }
    for (int dir = 0; dir < 2; ++dir)
        if ((st = build_scan_tables(pl, dir))) return st;
    for (int b = 0; b < NBANDS; ++b) {
        const int N = b == BAND_BX ? pl->Nx : pl->Ny;
        std::vector<double> a((size_t)N * RS, 0.0);
        for (int r = 0; r < N; ++r)
            for (int j = 0; j < W; ++j) a[(size_t)r * RS + j] = pl->cn_band[b][(size_t)r * W + j];
        BandHost &o = pl->band_host[b];
        interior_range(a, N, RS, rtol, o.K0, o.NK);
        if (o.NK <= o.K0) { o.K0 = N; o.NK = N; }
        o.rows = compress_rows(a, N, RS, o.K0, o.NK);
        o.rows.insert(o.rows.end(), (size_t)RS, 0.0);   // zero row for the padding
        o.nrows = (int)(o.rows.size() / RS);
        if ((st = upload_state(pl, pl->band_rows[b], o.rows))) return st;
    }
    return IGA_OK;
}

// ---------------------------------------------------------------------------
// line-solve schedules
// ---------------------------------------------------------------------------
iga_status choose_schedule(iga_plan *pl, int dir, int lines, int wpl)
{
    const int N = dir ? pl->Ny : pl->Nx, P = pl->P;
    const int nlines = dir ? pl->Nx : pl->Ny;
    // wavefronts per line: the fewest that keep a lane's chunk within the
    // largest compiled register capacity
    if (wpl <= 0) {
        wpl = 1;
        while (wpl < 8 && !sweep_capacity(std::max((N + 64 * wpl - 1) / (64 * wpl), P))) wpl *= 2;
    }
    const int mm = sweep_capacity(std::max((N + 64 * wpl - 1) / (64 * wpl), P));
    if (!mm) return fail(IGA_EUNSUPPORTED, "lines of " + std::to_string(N) + " dofs need more than "
                                           "8 wavefronts per line");
    Schedule &sc = pl->sched[dir];
    const Schedule old = sc;
    sc.mm = mm;
    sc.wpl = wpl;
    sc.win = 0;
    sc.col = 0;
    const int maxw = (!pl->fp32 && pl->P == 3 && mm >= 12) ? 8 : 16;   // wavefronts per workgroup
    if (lines <= 0) {
        // widest workgroup (<= 16 wavefronts) that fits LDS and still gives
        // >= 256 workgroups; at least 4 lines for strided x-lines
        lines = 1;
        for (int w : {16, 8, 4, 2}) {
            if (w * wpl > maxw || sweep_lds_bytes(pl, dir, w, wpl) > 160 * 1024) continue;
            if ((nlines + w - 1) / w >= 256 || w == 2) { lines = w; break; }
        }
        if (dir == 0 && lines < 4 && 4 * wpl <= maxw && sweep_lds_bytes(pl, dir, 4, wpl) <= 160 * 1024)
            lines = 4;
    }
    if (lines * wpl > maxw || (lines & (lines - 1)) || (wpl & (wpl - 1))) {
        sc = old;
        return fail(IGA_EUNSUPPORTED, "a workgroup holds at most " + std::to_string(maxw) +
                                          " wavefronts (lines x waves per line) here");
    }
    if (sweep_lds_bytes(pl, dir, lines, wpl) > 160 * 1024) {
        sc = old;
        return fail(IGA_EUNSUPPORTED, "line-solve workgroup of " + std::to_string(lines) +
                                          " lines does not fit in LDS");
    }
    sc.lines = lines;
    iga_status st;
    if (old.wpl != sc.wpl || old.mm != sc.mm || old.win || old.col)
        if ((st = build_scan_tables(pl, dir))) return st;
    return sweep_prepare(pl, dir);
}

// Windowed schedule of direction dir: `lines` lines per workgroup (0: the
// widest that fits LDS and gives >= 256 workgroups), mm rows per lane in
// {9, 13, 17, 25, 33} (0: 17); the wavefronts per line follow from the line
// length.  IGA_EUNSUPPORTED if the operators decay too slowly for a
// windowed solve or the schedule does not fit.
iga_status choose_window_schedule(iga_plan *pl, int dir, int lines, int mm)
{
    const int N = dir ? pl->Ny : pl->Nx, nlines = dir ? pl->Nx : pl->Ny;
    if (warmup_rows(pl, dir) <= 0)
        return fail(IGA_EUNSUPPORTED, "the operators decay too slowly for windowed solves");
    if (mm <= 0) mm = 17;
    if (mm != 9 && mm != 13 && mm != 17 && mm != 25 && mm != 33)
        return fail(IGA_EINVAL, "rows per lane must be 9, 13, 17, 25 or 33");
    const int wpl = (N + 64 * mm - 1) / (64 * mm);
    const int maxw = wsweep_max_block(pl->fp32, mm) / 64;
    if (wpl > maxw)
        return fail(IGA_EUNSUPPORTED, "lines of " + std::to_string(N) + " rows need more than " +
                                          std::to_string(maxw) + " wavefronts at this rows-per-lane");
    if (lines <= 0) {
        lines = 0;
        for (int w : {16, 8, 4, 2, 1}) {
            if (w * wpl > maxw || wsweep_lds_bytes(pl, dir, w, wpl, mm) > 160 * 1024) continue;
            if (!lines) lines = w;   // widest that fits
            if ((nlines + w - 1) / w >= 256) { lines = w; break; }
        }
        if (!lines) return fail(IGA_EUNSUPPORTED, "windowed line buffers do not fit in LDS");
    }
    if (lines * wpl > maxw || (lines & (lines - 1)))
        return fail(IGA_EUNSUPPORTED, "a workgroup holds at most " + std::to_string(maxw) +
                                          " wavefronts (lines x waves per line) here");
    if (wsweep_lds_bytes(pl, dir, lines, wpl, mm) > 160 * 1024)
        return fail(IGA_EUNSUPPORTED, "windowed workgroup of " + std::to_string(lines) +
                                          " lines does not fit in LDS");
    Schedule &sc = pl->sched[dir];
    const Schedule old = sc;
    sc.lines = lines;
    sc.wpl = wpl;
    sc.mm = mm;
    sc.win = 1;
    sc.col = 0;
    iga_status st = build_window_tables(pl, dir);
    if (!st) st = wsweep_prepare(pl, dir);
    if (st) {
        sc = old;
        return st;
    }
    return IGA_OK;
}

// Column-wave schedule of the x-lines (FP32 plans): chunks of mm rows in
// {16, 32} (0: 32), one line per lane.  IGA_EUNSUPPORTED if the plan is not
// FP32 or its x operators decay too slowly for the kernel's warm-ups.
iga_status choose_column_schedule(iga_plan *pl, int mm)
{
    if (mm <= 0) mm = 32;
    if (!csweep_rows_ok(mm)) return fail(IGA_EINVAL, "rows per chunk must be 16 or 32");
    if (!csweep_ok(pl))
        return fail(IGA_EUNSUPPORTED, "column-wave solves need an FP32 plan whose x operators decay "
                                      "within the kernel's warm-ups");
    if ((size_t)pl->Nx * pl->Ny * 4 >= ((size_t)1 << 31))
        return fail(IGA_EUNSUPPORTED, "column-wave solves address fields below 2 GiB");
    iga_status st = build_column_edges(pl, mm);
    if (st) return st;
    Schedule &sc = pl->sched[0];
    sc.lines = 1;
    sc.wpl = 1;
    sc.mm = mm;
    sc.win = 0;
    sc.col = 1;
    return IGA_OK;
}

}  // namespace iga
