// hh_setup.cpp -- host-side setup of one grid.
//
// Per axis and level the unknowns are cell centres; the two Dirichlet ends
// are the outer edges lo and hi (half a cell from the first/last centre).
// Node maps (paper Sec. 2, eq. (ecstrans) with Simon's linear exterior
// scaling; Sec. 5.3 for the CSG map of the preconditioner):
//   H (ECS):  z = a + (x - a) e^{i th_g} for x < a,  x on [a, b],
//             z = b + (x - b) e^{i th_g} for x > b
//   M (CSG, uniform):  z_M = beta z_H with beta = e^{i th_b}
//   M (CSG, interior): interior widths times beta, layer widths unchanged.
// Shortley-Weller coefficients (Sec. 3, eq. (shortwell)) at node j with
// hl = z_j - z_{j-1}, hr = z_{j+1} - z_j, s = hl + hr:
//   a_j = 2 / (hl s),  c_j = 2 / (hr s),  d_j = a_j + c_j
// so that -u'' ~ -a_j u_{j-1} + d_j u_j - c_j u_{j+1}.
// Coarse levels rediscretise on the halved grid; coarse phi is the mean of
// the 2^d children.  The coarsest M is assembled densely (column q = M e_q),
// factorised by LU with partial pivoting and inverted explicitly (the
// paper's multigrid used a direct "backslash" solve on its hierarchy).
//
// All arithmetic follows the fixed operation order of the device kernels
// (complex multiply/divide formulas of hh_common.h, no FMA contraction).
#include "hh_setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <thread>

namespace {

// Complex node positions of one axis: the ECS contour of H and the stretched
// grid of the preconditioner M, with the Dirichlet or Sommerfeld treatment of
// the two ends.
struct AxisGeometry {
    double lo, hi, a, b;
    double theta, cg, sg;      // ECS angle and its cosine / sine
    double2 beta;              // stretching factor of M
    int mode, steps;
    int bc[2];                 // low / high side: HH_BC_*

    // How far a smooth contour has moved from its turning point after a real
    // distance t into a layer of width L: the layer is cut into `steps`
    // equal parts, part p turned by p theta / steps.
    double2 turn(double t, double L) const
    {
        const double w = L / (double)steps;
        int whole = (int)std::floor(t / w);
        whole = std::min(std::max(whole, 0), steps);
        double2 acc = cmk<double>(0.0, 0.0);
        for (int p = 1; p <= whole; ++p) {
            const double ang = theta * (double)p / (double)steps;
            acc = cadd<double>(acc, cmk<double>(w * std::cos(ang), w * std::sin(ang)));
        }
        const double part = t - (double)whole * w;
        if (whole < steps && part > 0.0) {
            const double ang = theta * (double)(whole + 1) / (double)steps;
            acc = cadd<double>(acc, cmk<double>(part * std::cos(ang), part * std::sin(ang)));
        }
        return acc;
    }
    double2 zH(double x) const
    {
        const bool left = x < a, right = x > b;
        if (!left && !right) return cmk<double>(x, 0.0);
        if (steps <= 1) {
            const double r = left ? a : b, t = x - r;
            return cmk<double>(r + t * cg, t * sg);
        }
        return left ? csub<double>(cmk<double>(a, 0.0), turn(a - x, a - lo))
                    : cadd<double>(cmk<double>(b, 0.0), turn(x - b, hi - b));
    }
    double2 zM(double x) const
    {
        if (mode != HH_CSG_INTERIOR) return cmul<double>(beta, zH(x));
        const bool left = x < a, right = x > b;
        if (!left && !right) return cmk<double>(x * beta.x, x * beta.y);
        const double r = left ? a : b;
        if (steps <= 1) {
            const double t = x - r;
            return cmk<double>(r * beta.x + t * cg, r * beta.y + t * sg);
        }
        const double2 rb = cmk<double>(r * beta.x, r * beta.y);
        return left ? csub<double>(rb, turn(a - x, a - lo)) : cadd<double>(rb, turn(x - b, hi - b));
    }
};

// Principal square root of a nonzero complex number.
double2 principal_sqrt(double2 v)
{
    const double r = std::sqrt(v.x * v.x + v.y * v.y);
    if (v.x >= 0.0) {
        const double re = std::sqrt(0.5 * (r + v.x));
        return cmk<double>(re, v.y / (2.0 * re));
    }
    double im = std::sqrt(0.5 * (r - v.x));
    if (v.y < 0.0) im = -im;
    return cmk<double>(v.y / (2.0 * im), im);
}

// u_ghost = rho u_last from the centred difference of du/dn = -i k u at the
// face between the last unknown and the ghost at complex distance w.
double2 ghost_factor(double k, double2 w)
{
    const double hk = 0.5 * k;
    return cdiv<double>(cmk<double>(1.0 + hk * w.y, -(hk * w.x)), cmk<double>(1.0 - hk * w.y, hk * w.x));
}

void sw(int n, const std::vector<double2> &z, std::vector<double2> &A, std::vector<double2> &C,
        std::vector<double2> &D)
{
    A.resize(n);
    C.resize(n);
    D.resize(n);
    const double2 two = cmk<double>(2.0, 0.0);
    for (int j = 1; j <= n; ++j) {
        double2 hl = csub<double>(z[j], z[j - 1]);
        double2 hr = csub<double>(z[j + 1], z[j]);
        double2 s = cadd<double>(hl, hr);
        double2 aj = cdiv<double>(two, cmul<double>(hl, s));
        double2 cj = cdiv<double>(two, cmul<double>(hr, s));
        A[j - 1] = aj;
        C[j - 1] = cj;
        D[j - 1] = cadd<double>(aj, cj);
    }
}

double abs1(double2 z) { return std::fabs(z.x) + std::fabs(z.y); }

// LU with partial pivoting (first maximum of |re|+|im|), k-i-j order.
bool lu(std::vector<double2> &A, int n, std::vector<int> &perm)
{
    perm.resize(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = abs1(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = abs1(A[(size_t)i * n + k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        if (best == 0.0) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
            std::swap(perm[k], perm[p]);
        }
        const double2 piv = A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double2 l = cdiv<double>(A[(size_t)i * n + k], piv);
            A[(size_t)i * n + k] = l;
            double2 *ri = &A[(size_t)i * n];
            const double2 *rk = &A[(size_t)k * n];
            for (int j = k + 1; j < n; ++j) ri[j] = csub<double>(ri[j], cmul<double>(l, rk[j]));
        }
    }
    return true;
}

void lu_solve_unit(const std::vector<double2> &LU, int n, const std::vector<int> &perm, int col, double2 *x)
{
    for (int i = 0; i < n; ++i) {
        double2 s = cmk<double>(perm[i] == col ? 1.0 : 0.0, 0.0);
        for (int j = 0; j < i; ++j) s = csub<double>(s, cmul<double>(LU[(size_t)i * n + j], x[j]));
        x[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double2 s = x[i];
        for (int j = i + 1; j < n; ++j) s = csub<double>(s, cmul<double>(LU[(size_t)i * n + j], x[j]));
        x[i] = cdiv<double>(s, LU[(size_t)i * n + i]);
    }
}

} // namespace

int auto_levels(int dim, const int *n)
{
    const int thr = dim == 3 ? 8 : 16;
    int m[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
    int nl = 1;
    for (;;) {
        bool even = true;
        int mx = 0;
        for (int d = 0; d < dim; ++d) {
            if (m[d] % 2) even = false;
            if (m[d] > mx) mx = m[d];
        }
        if (!even || mx <= thr || nl >= HH_MAXLEV) break;
        for (int d = 0; d < dim; ++d) m[d] /= 2;
        ++nl;
    }
    return nl;
}

void host_apply_M(const HostSetup &hs, int lev, const double2 *x, double2 *y)
{
    const HostLevel &L = hs.lev[lev];
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const double2 zero = cmk<double>(0.0, 0.0);
    if (!L.gal.empty()) {
        // Galerkin level (2D): centre entry first, then the others in entry order
        const int64_t N = L.N;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t p = i + sy * j;
                double2 t = cmul<double>(L.gal[12 * N + p], x[p]);
                for (int s = 0; s < 25; ++s) {
                    if (s == 12) continue;
                    const int ii = i + s % 5 - 2, jj = j + s / 5 - 2;
                    const double2 xq = (ii >= 0 && ii < nx && jj >= 0 && jj < ny) ? x[ii + sy * jj] : zero;
                    t = cadd<double>(t, cmul<double>(L.gal[s * N + p], xq));
                }
                y[p] = t;
            }
        return;
    }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t p = i + sy * j + sz * k;
                double2 d = L.dM[0][i];
                d = cadd<double>(d, L.dM[1][j]);
                if (hs.dim == 3) d = cadd<double>(d, L.dM[2][k]);
                double2 D = cmk<double>(d.x - L.phi[p], d.y);
                double2 t = cmul<double>(D, x[p]);
                t = csub<double>(t, cmul<double>(L.aM[0][i], i > 0 ? x[p - 1] : zero));
                t = csub<double>(t, cmul<double>(L.cM[0][i], i < nx - 1 ? x[p + 1] : zero));
                t = csub<double>(t, cmul<double>(L.aM[1][j], j > 0 ? x[p - sy] : zero));
                t = csub<double>(t, cmul<double>(L.cM[1][j], j < ny - 1 ? x[p + sy] : zero));
                if (hs.dim == 3) {
                    t = csub<double>(t, cmul<double>(L.aM[2][k], k > 0 ? x[p - sz] : zero));
                    t = csub<double>(t, cmul<double>(L.cM[2][k], k < nz - 1 ? x[p + sz] : zero));
                }
                y[p] = t;
            }
}

// Galerkin operator of level lc (Sec. 6.1), M_lc = R M_{lc-1} P, for the
// coarse rows [j0, j1): column J is R (M_{lc-1} (P e_J)), evaluated only on
// the cells it reaches.  Per axis, P e_J is 3/4 or 1/4 on fine cells 2J-1 ..
// 2J+2 (exact products of the two); M widens that by its bandwidth b (1 for
// the rediscretised stencil, 2 for a Galerkin one); a restriction row covers
// fine cells 2I-1 .. 2I+2, so only rows |I - J| <= 2 per axis are nonzero.
// Values follow the V-cycle's arithmetic: the level's stencil as in
// host_apply_M, full weighting along x and then y with zero outside the grid,
// so each entry is what R (M (P e_J)) over whole vectors gives.  Columns are
// independent; entry (s, I) belongs to column I + offset(s) alone.
static void galerkin_rows(HostSetup &hs, int lc, int j0, int j1)
{
    const HostLevel &F = hs.lev[lc - 1];
    HostLevel &C = hs.lev[lc];
    const int nfx = F.n[0], nfy = F.n[1], ncx = C.n[0], ncy = C.n[1];
    const int64_t Nc = C.N, Nf = F.N;
    const int b = F.gal.empty() ? 1 : 2;
    const int W = 4 + 2 * b;   // side of the window of M P e_J
    const double2 zero = cmk<double>(0.0, 0.0);
    const double RW[4] = {0.125, 0.375, 0.375, 0.125};
    // weight of coarse J at fine i along one axis (the prolongation of a unit vector)
    auto pw = [](int i, int J, int ncoarse) -> double {
        const int I = i / 2, Io = (i % 2) ? I + 1 : I - 1;
        if (I == J) return 0.75;
        return (Io == J && Io >= 0 && Io < ncoarse) ? 0.25 : 0.0;
    };
    double2 w[4][4], y[8][8];
    for (int Jy = j0; Jy < j1; ++Jy)
        for (int Jx = 0; Jx < ncx; ++Jx) {
            const int wx0 = 2 * Jx - 1, wy0 = 2 * Jy - 1;
            for (int v = 0; v < 4; ++v)
                for (int u = 0; u < 4; ++u) {
                    const int i = wx0 + u, j = wy0 + v;
                    const bool in = i >= 0 && i < nfx && j >= 0 && j < nfy;
                    w[v][u] = in ? cmk<double>(pw(j, Jy, ncy) * pw(i, Jx, ncx), 0.0) : zero;
                }
            auto wv = [&](int i, int j) -> double2 {
                const int u = i - wx0, v = j - wy0;
                return (u >= 0 && u < 4 && v >= 0 && v < 4) ? w[v][u] : zero;
            };
            const int yx0 = wx0 - b, yy0 = wy0 - b;
            for (int v = 0; v < W; ++v)
                for (int u = 0; u < W; ++u) {
                    const int i = yx0 + u, j = yy0 + v;
                    double2 t = zero;
                    if (i >= 0 && i < nfx && j >= 0 && j < nfy) {
                        const int64_t p = i + (int64_t)nfx * j;
                        if (F.gal.empty()) {
                            double2 d = cadd<double>(F.dM[0][i], F.dM[1][j]);
                            const double2 D = cmk<double>(d.x - F.phi[p], d.y);
                            t = cmul<double>(D, wv(i, j));
                            t = csub<double>(t, cmul<double>(F.aM[0][i], i > 0 ? wv(i - 1, j) : zero));
                            t = csub<double>(t, cmul<double>(F.cM[0][i], i < nfx - 1 ? wv(i + 1, j) : zero));
                            t = csub<double>(t, cmul<double>(F.aM[1][j], j > 0 ? wv(i, j - 1) : zero));
                            t = csub<double>(t, cmul<double>(F.cM[1][j], j < nfy - 1 ? wv(i, j + 1) : zero));
                        } else {
                            t = cmul<double>(F.gal[12 * Nf + p], wv(i, j));
                            for (int s = 0; s < 25; ++s) {
                                if (s == 12) continue;
                                const int ii = i + s % 5 - 2, jj = j + s / 5 - 2;
                                const double2 xq = (ii >= 0 && ii < nfx && jj >= 0 && jj < nfy) ? wv(ii, jj) : zero;
                                t = cadd<double>(t, cmul<double>(F.gal[s * Nf + p], xq));
                            }
                        }
                    }
                    y[v][u] = t;
                }
            auto yv = [&](int i, int j) -> double2 {
                const int u = i - yx0, v = j - yy0;
                return (u >= 0 && u < W && v >= 0 && v < W) ? y[v][u] : zero;
            };
            for (int Iy = Jy - 2; Iy <= Jy + 2; ++Iy)
                for (int Ix = Jx - 2; Ix <= Jx + 2; ++Ix) {
                    if (Ix < 0 || Ix >= ncx || Iy < 0 || Iy >= ncy) continue;
                    double2 rows[4];
                    for (int q = 0; q < 4; ++q) {
                        const int j = 2 * Iy - 1 + q;
                        double2 sx = zero;
                        for (int r = 0; r < 4; ++r) {
                            const int i = 2 * Ix - 1 + r;
                            const double2 val = (i >= 0 && i < nfx) ? yv(i, j) : zero;
                            sx = r == 0 ? crs<double>(RW[r], val) : cadd<double>(sx, crs<double>(RW[r], val));
                        }
                        rows[q] = (j >= 0 && j < nfy) ? sx : zero;
                    }
                    double2 z = zero;
                    for (int q = 0; q < 4; ++q) z = q == 0 ? crs<double>(RW[q], rows[q]) : cadd<double>(z, crs<double>(RW[q], rows[q]));
                    const int s = (Jx - Ix + 2) + 5 * (Jy - Iy + 2);
                    C.gal[s * Nc + (Ix + (int64_t)ncx * Iy)] = z;
                }
        }
}

static void galerkin_level(HostSetup &hs, int lc)
{
    HostLevel &C = hs.lev[lc];
    C.gal.assign((size_t)25 * C.N, cmk<double>(0.0, 0.0));
    const int ny = C.n[1];
    const int nt = std::max(1, std::min(16, std::min(ny, (int)std::thread::hardware_concurrency())));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const int j0 = (int)((int64_t)ny * t / nt), j1 = (int)((int64_t)ny * (t + 1) / nt);
        th.emplace_back(galerkin_rows, std::ref(hs), lc, j0, j1);
    }
    for (auto &x : th) x.join();
}

// ILU(0) of the 2D level operator M_l on its nonzero pattern (Sec. 6.1, the
// paper's smoother; the incomplete row-wise elimination, rows in
// lexicographic order).  Entries use the Galerkin layout s = (dx+2) +
// 5(dy+2); a rediscretised level has the 5-point set {7, 11, 12, 13, 17}.
// The pattern is the diagonal and the nonzero in-grid entries.  With at
// least 5 cells per side (checked by desc_check) ascending s is ascending
// column, so row p eliminates its entries below the diagonal in s order:
// l = a[p][s] / a[q][12] with q the column of s, then every pattern entry t
// of row p beyond s loses l times entry (q, column of t) when that entry is
// in row q's pattern.  Returns false on a zero pivot.
static bool ilu_level(HostSetup &hs, int l)
{
    HostLevel &L = hs.lev[l];
    const int nx = L.n[0], ny = L.n[1];
    const int64_t N = L.N;
    const bool gal = !L.gal.empty();
    std::vector<double2> &A = L.ilu;
    A.assign((size_t)25 * N, cmk<double>(0.0, 0.0));
    std::vector<uint8_t> in((size_t)25 * N, 0);
    auto member = [gal](int s) { return gal || s == 7 || s == 11 || s == 12 || s == 13 || s == 17; };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int64_t p = i + (int64_t)nx * j;
            for (int s = 0; s < 25; ++s) {
                const int dx = s % 5 - 2, dy = s / 5 - 2;
                if (!member(s) || i + dx < 0 || i + dx >= nx || j + dy < 0 || j + dy >= ny) continue;
                double2 v;
                if (gal) {
                    v = L.gal[s * N + p];
                } else if (s == 12) {
                    const double2 d = cadd<double>(L.dM[0][i], L.dM[1][j]);
                    v = cmk<double>(d.x - L.phi[p], d.y);
                } else {
                    const double2 c = s == 11 ? L.aM[0][i] : s == 13 ? L.cM[0][i] : s == 7 ? L.aM[1][j] : L.cM[1][j];
                    v = cmk<double>(-c.x, -c.y);
                }
                if (s != 12 && v.x == 0.0 && v.y == 0.0) continue;
                A[s * N + p] = v;
                in[s * N + p] = 1;
            }
        }
    for (int64_t p = 0; p < N; ++p)
        for (int s = 0; s < 12; ++s) {
            if (!in[s * N + p]) continue;
            const int64_t q = p + (s % 5 - 2) + (int64_t)nx * (s / 5 - 2);
            const double2 piv = A[12 * N + q];
            if (piv.x == 0.0 && piv.y == 0.0) return false;
            const double2 lv = cdiv<double>(A[s * N + p], piv);
            A[s * N + p] = lv;
            for (int t = s + 1; t < 25; ++t) {
                if (!in[t * N + p]) continue;
                const int ux = t % 5 - s % 5, uy = t / 5 - s / 5;
                if (ux < -2 || ux > 2 || uy < -2 || uy > 2) continue;
                const int r = (ux + 2) + 5 * (uy + 2);
                if (!in[r * N + q]) continue;
                A[t * N + p] = csub<double>(A[t * N + p], cmul<double>(lv, A[r * N + q]));
            }
        }
    return true;
}

hh_status desc_check(const hh_grid_desc *d, int &levels, int &coarse, std::string &err)
{
    char buf[256];
    if (!d) { err = "null grid description"; return HH_ERR_ARG; }
    if (d->dim != 2 && d->dim != 3) { err = "dim must be 2 or 3"; return HH_ERR_ARG; }
    const int dim = d->dim;
    const double half_pi = 1.5707963267948966;
    if (!(d->theta_ecs > 0.0 && d->theta_ecs < half_pi)) { err = "theta_ecs must lie in (0, pi/2)"; return HH_ERR_ARG; }
    if (d->csg_mode != HH_CSG_UNIFORM && d->csg_mode != HH_CSG_INTERIOR && d->csg_mode != HH_CSL) {
        err = "csg_mode must be 0 (uniform CSG), 1 (interior CSG) or 2 (CSL)";
        return HH_ERR_ARG;
    }
    if (d->csg_mode != HH_CSL && !(std::fabs(d->theta_csg) < half_pi)) { err = "theta_csg must lie in (-pi/2, pi/2)"; return HH_ERR_ARG; }
    if (d->csg_mode == HH_CSL && !(std::isfinite(d->csl_shift[0]) && std::isfinite(d->csl_shift[1]) &&
                                   (d->csl_shift[0] != 0.0 || d->csl_shift[1] != 0.0))) {
        err = "the CSL shift must be finite and nonzero";
        return HH_ERR_ARG;
    }
    if (d->contour_steps < 0 || d->contour_steps > 65536) { err = "contour_steps must lie in [0, 65536]"; return HH_ERR_ARG; }
    if (d->centering != HH_CELL && d->centering != HH_VERTEX) { err = "centering must be 0 (cell) or 1 (vertex)"; return HH_ERR_ARG; }
    if ((d->nu1 != 0 && d->nu1 != 1) || d->nu2 != 1) {
        err = "the cycle is V(1,1) or the paper's V(0,1): nu1 = 0 or 1, nu2 = 1";
        return HH_ERR_ARG;
    }
    if (!(d->omega > 0.0 && d->omega < 2.0)) { err = "omega must lie in (0, 2)"; return HH_ERR_ARG; }
    if (d->coarse_op != HH_COARSE_REDISCRETISED && d->coarse_op != HH_COARSE_GALERKIN) {
        err = "coarse_op must be 0 (rediscretised) or 1 (Galerkin)";
        return HH_ERR_ARG;
    }
    if (d->coarse_op == HH_COARSE_GALERKIN && (dim != 2 || d->centering != HH_CELL)) {
        err = "Galerkin coarse operators need a 2D cell-centred grid";
        return HH_ERR_ARG;
    }
    if (d->smoother != HH_SMOOTH_JACOBI && d->smoother != HH_SMOOTH_ILU0) {
        err = "smoother must be 0 (weighted Jacobi) or 1 (ILU(0))";
        return HH_ERR_ARG;
    }
    if (d->smoother == HH_SMOOTH_ILU0 && (dim != 2 || d->centering != HH_CELL || d->nu1 != 0)) {
        err = "ILU(0) smoothing needs a 2D cell-centred grid and the V(0,1) cycle (nu1 = 0)";
        return HH_ERR_ARG;
    }
    int64_t N = 1;
    for (int a = 0; a < dim; ++a) {
        if (d->n[a] < 2) { err = "every side needs at least 2 cells"; return HH_ERR_ARG; }
        if (!(d->lo[a] <= d->a[a] && d->a[a] < d->b[a] && d->b[a] <= d->hi[a] && d->lo[a] < d->hi[a])) {
            snprintf(buf, sizeof buf, "axis %d: need lo <= a < b <= hi", a);
            err = buf;
            return HH_ERR_ARG;
        }
        for (int side = 0; side < 2; ++side) {
            const int bc = d->bc[a][side];
            if (bc != HH_BC_DIRICHLET && bc != HH_BC_SOMMERFELD) { err = "bc must be 0 (Dirichlet) or 1 (Sommerfeld)"; return HH_ERR_ARG; }
            if (bc != HH_BC_SOMMERFELD) continue;
            if (side == 0 ? d->a[a] != d->lo[a] : d->b[a] != d->hi[a]) {
                snprintf(buf, sizeof buf, "axis %d: a Sommerfeld side has no layer (need %s)", a, side == 0 ? "a == lo" : "b == hi");
                err = buf;
                return HH_ERR_ARG;
            }
            if (d->centering != HH_CELL) { err = "Sommerfeld sides need a cell-centred grid"; return HH_ERR_ARG; }
            if (!(d->k_bc > 0.0 && std::isfinite(d->k_bc))) { err = "a Sommerfeld side needs k_bc > 0"; return HH_ERR_ARG; }
        }
        N *= d->n[a];
    }
    // the finaliser stages at most 64 blocks of HH_FIN_STAGE chunk partials
    if (N > ((int64_t)1 << 28)) { err = "more than 2^28 unknowns"; return HH_ERR_ARG; }
    if (d->centering == HH_VERTEX) {
        // the operator of Sec. 3 on its vertex grid: no multigrid hierarchy
        if (d->levels > 1) { err = "a vertex-centred grid has one level (levels 0 or 1)"; return HH_ERR_ARG; }
        levels = 1;
        coarse = 0;
        return HH_OK;
    }
    const int nl = d->levels > 0 ? d->levels : auto_levels(dim, d->n);
    if (nl > HH_MAXLEV) { err = "too many levels"; return HH_ERR_ARG; }
    if (nl < 2) { err = "the multigrid preconditioner needs at least 2 levels (set levels, or use a larger grid)"; return HH_ERR_ARG; }
    for (int a = 0; a < dim; ++a)
        if (d->n[a] % (1 << (nl - 1))) {
            snprintf(buf, sizeof buf, "side %d (%d cells) is not divisible by 2^(levels-1) = %d", a, d->n[a], 1 << (nl - 1));
            err = buf;
            return HH_ERR_ARG;
        }
    int64_t Nc = 1;
    for (int a = 0; a < dim; ++a) Nc *= d->n[a] >> (nl - 1);
    if (Nc > HH_MAX_COARSE) {
        snprintf(buf, sizeof buf, "coarsest grid has %lld unknowns (limit %d); use more levels",
                 (long long)Nc, HH_MAX_COARSE);
        err = buf;
        return HH_ERR_ARG;
    }
    if (d->smoother == HH_SMOOTH_ILU0)
        for (int a = 0; a < dim; ++a)
            if ((d->n[a] >> (nl - 2)) < 5) {
                snprintf(buf, sizeof buf, "ILU(0) smoothing needs at least 5 cells per side on level %d (side %d has %d)",
                         nl - 2, a, d->n[a] >> (nl - 2));
                err = buf;
                return HH_ERR_ARG;
            }
    levels = nl;
    coarse = (int)Nc;
    return HH_OK;
}

hh_status host_setup(const hh_grid_desc *d, HostSetup &hs, std::string &err)
{
    int nl = 0, ncoarse = 0;
    hh_status st = desc_check(d, nl, ncoarse, err);
    if (st != HH_OK) return st;
    const int dim = d->dim;
    const int64_t Nc = ncoarse;
    hs.dim = dim;
    hs.nlev = nl;
    hs.omega = d->omega;
    hs.centering = d->centering;
    hs.nu1 = d->nu1;
    const bool vertex = d->centering == HH_VERTEX;
    const double cg = std::cos(d->theta_ecs), sg = std::sin(d->theta_ecs);
    const double2 beta = d->csg_mode == HH_CSL ? principal_sqrt(cmk<double>(d->csl_shift[0], d->csl_shift[1]))
                                               : cmk<double>(std::cos(d->theta_csg), std::sin(d->theta_csg));
    for (int l = 0; l < nl; ++l) {
        HostLevel &L = hs.lev[l];
        L.N = 1;
        for (int a = 0; a < 3; ++a) {
            L.n[a] = a < dim ? d->n[a] >> l : 1;
            L.N *= L.n[a];
        }
        for (int a = 0; a < dim; ++a) {
            const int n = L.n[a];
            const AxisGeometry geo{d->lo[a], d->hi[a], d->a[a], d->b[a], d->theta_ecs, cg, sg, beta,
                                   d->csg_mode, d->contour_steps, {d->bc[a][0], d->bc[a][1]}};
            // real nodes: the two ends and the n unknowns between them, at
            // cell centres or at the vertices of n + 1 equal intervals; the
            // end of a Sommerfeld side is a ghost one cell beyond the last
            // unknown, on the continuation of the interior (no layer there)
            const double lo = d->lo[a], hi = d->hi[a];
            const double h = vertex ? (hi - lo) / (double)(n + 1) : (hi - lo) / (double)n;
            std::vector<double> x(n + 2);
            for (int j = 1; j <= n; ++j) x[j] = vertex ? lo + (double)j * h : lo + ((double)j - 0.5) * h;
            x[0] = geo.bc[0] == HH_BC_SOMMERFELD ? lo - 0.5 * h : lo;
            x[n + 1] = geo.bc[1] == HH_BC_SOMMERFELD ? hi + 0.5 * h : hi;
            std::vector<double2> zH(n + 2), zM(n + 2);
            for (int j = 0; j <= n + 1; ++j) {
                const bool ghost = (j == 0 && geo.bc[0] == HH_BC_SOMMERFELD) || (j == n + 1 && geo.bc[1] == HH_BC_SOMMERFELD);
                zH[j] = ghost ? cmk<double>(x[j], 0.0) : geo.zH(x[j]);
                zM[j] = ghost ? cmk<double>(beta.x * x[j], beta.y * x[j]) : geo.zM(x[j]);
            }
            sw(n, zM, L.aM[a], L.cM[a], L.dM[a]);
            if (l == 0) sw(n, zH, hs.aH[a], hs.cH[a], hs.dH[a]);
            // Sommerfeld sides: the ghost's coefficient folds onto the diagonal
            // of the unknown next to the boundary
            for (int side = 0; side < 2; ++side) {
                if (geo.bc[side] != HH_BC_SOMMERFELD) continue;
                const int j = side == 0 ? 0 : n - 1;                  // unknown next to the boundary
                const int inner = side == 0 ? 1 : n, outer = side == 0 ? 0 : n + 1;
                const double2 rM = ghost_factor(d->k_bc, csub<double>(zM[side == 0 ? inner : outer], zM[side == 0 ? outer : inner]));
                L.dM[a][j] = csub<double>(L.dM[a][j], cmul<double>(side == 0 ? L.aM[a][j] : L.cM[a][j], rM));
                if (l == 0) {
                    const double2 rH = ghost_factor(d->k_bc, csub<double>(zH[side == 0 ? inner : outer], zH[side == 0 ? outer : inner]));
                    hs.dH[a][j] = csub<double>(hs.dH[a][j], cmul<double>(side == 0 ? hs.aH[a][j] : hs.cH[a][j], rH));
                }
            }
        }
        L.phi.resize(L.N);
        if (l == 0) {
            for (int64_t p = 0; p < L.N; ++p) {
                double v = d->phi ? d->phi[p] : d->phi_const;
                if (!std::isfinite(v)) { err = "phi has a non-finite value"; return HH_ERR_ARG; }
                L.phi[p] = v;
            }
        } else {
            const HostLevel &F = hs.lev[l - 1];
            const double scale = dim == 2 ? 0.25 : 0.125;
            const int cz = dim == 3 ? 2 : 1;
            for (int k = 0; k < L.n[2]; ++k)
                for (int j = 0; j < L.n[1]; ++j)
                    for (int i = 0; i < L.n[0]; ++i) {
                        double s = 0.0;
                        for (int dz = 0; dz < cz; ++dz)
                            for (int dy = 0; dy < 2; ++dy)
                                for (int dx = 0; dx < 2; ++dx) {
                                    int64_t fi = (2 * i + dx) + (int64_t)F.n[0] * ((2 * j + dy) + (int64_t)F.n[1] * (cz == 2 ? 2 * k + dz : k));
                                    s = s + F.phi[fi];
                                }
                        L.phi[i + (int64_t)L.n[0] * (j + (int64_t)L.n[1] * k)] = s * scale;
                    }
        }
    }
    // Galerkin coarse operators, level after level from the finest preconditioner
    hs.coarse_op = d->coarse_op;
    if (hs.coarse_op == HH_COARSE_GALERKIN)
        for (int l = 1; l < nl; ++l) galerkin_level(hs, l);
    // ILU(0) factors of every smoothing level
    hs.smoother = d->smoother;
    if (hs.smoother == HH_SMOOTH_ILU0)
        for (int l = 0; l + 1 < nl; ++l)
            if (!ilu_level(hs, l)) {
                err = "ILU(0) of level " + std::to_string(l) + " met a zero pivot";
                return HH_ERR_ARG;
            }
    // coarsest inverse (a vertex-centred grid has no hierarchy)
    const int n = (int)Nc;
    hs.Nc = n;
    if (vertex) return HH_OK;
    std::vector<double2> A((size_t)n * n), e(n), col(n);
    for (int q = 0; q < n; ++q) {
        for (int p = 0; p < n; ++p) e[p] = cmk<double>(p == q ? 1.0 : 0.0, 0.0);
        host_apply_M(hs, nl - 1, e.data(), col.data());
        for (int p = 0; p < n; ++p) A[(size_t)p * n + q] = col[p];
    }
    std::vector<int> perm;
    if (!lu(A, n, perm)) { err = "the coarsest preconditioner matrix is singular"; return HH_ERR_ARG; }
    hs.Minv.assign((size_t)n * n, cmk<double>(0.0, 0.0));
    std::vector<double2> x(n);
    for (int c = 0; c < n; ++c) {
        lu_solve_unit(A, n, perm, c, x.data());
        for (int p = 0; p < n; ++p) hs.Minv[(size_t)p * n + c] = x[p];
    }
    return HH_OK;
}
