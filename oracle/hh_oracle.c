/*
 * hh_oracle.c -- plain CPU FP64 oracle for the ECS/CSG Helmholtz hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or run this code.  It shares no
 * source, header, table or helper with the HIP library: it is written from
 * the paper (Reps, Vanroose, bin Zubair, "On the indefinite Helmholtz
 * equation: complex stretched absorbing boundary layers, iterative analysis,
 * and preconditioning") and from the textbook definitions of the solvers it
 * names.  Everything is complex FP64, no FMA contraction (built with
 * -ffp-contract=off), with the fixed operation orders spelled out below so
 * that a device implementation following the same arithmetic contract can be
 * compared value for value.
 *
 * What is computed, with the passage it follows:
 *   geometry        Sec. 2, eq. (ecstrans) and the linear ECS map of Simon
 *                   (exterior complex scaling): z(x) = r + (x - r) e^{i th}
 *                   on the layer, or (Sec. 6.2, remark on a smooth ECS
 *                   transition) a contour that turns to th in m equal angle
 *                   steps over m equal parts of the layer; Sec. 5.3, eq.
 *                   (CSL-CSG) and eq. (lapctucsg): the complex stretched grid
 *                   (CSG) map of the preconditioner, uniform (z -> beta z) or
 *                   interior-only; Sec. 5.2, eq. (helmctucsl): the complex
 *                   shifted Laplacian -(L + beta^2 phi), taken through eq.
 *                   (CSL-CSG) as the uniform CSG with beta the principal
 *                   square root of the shift (M_CSL = beta^2 M_CSG).
 *   boundaries      Dirichlet at the contour ends (eq. (lapctuecs)), or on
 *                   an edge without a layer the first-order Sommerfeld
 *                   condition du/dn = -i k u (Sec. 2, eq. (sommerfeld1);
 *                   Sec. 4, eq. (BC)), by a ghost node one cell beyond the
 *                   boundary and the centred difference of the condition at
 *                   the boundary face.
 *   operator        Sec. 3, eq. (shortwell): Shortley-Weller 3-point second
 *                   derivative on complex, non-uniform widths, per axis;
 *                   Sec. 4, eq. (Helgen): -(Lap + phi) u with phi = k(x)^2;
 *                   homogeneous Dirichlet at the contour ends, eq.
 *                   (lapctuecs).  Cell-centred topology (Sec. 6) by default,
 *                   vertex-centred (Sec. 3, eq. (ecsgrid)) for closed forms.
 *   multigrid       Sec. 5.1 / 6.1: geometric multigrid with weighted Jacobi
 *                   smoothing or (2D, Sec. 6.1, the paper's choice) ILU(0)
 *                   smoothing, full-weighting restriction, bilinear
 *                   (trilinear) prolongation, rediscretised coarse
 *                   operators or (2D, Sec. 6.1) Galerkin coarse operators
 *                   M_{l+1} = R M_l P (25-point: the cell-centred transfers
 *                   reach two coarse cells), exact coarsest solve; one V(nu1,nu2)
 *                   cycle per preconditioner application (Sec. 6.2).
 *   Krylov          Sec. 6.2: right-preconditioned Bi-CGSTAB (van der Vorst
 *                   1992) and IDR(s) (Sonneveld & van Gijzen 2008, the
 *                   prototype with minimal-residual omega), stopping on the
 *                   relative residual, matvec counting as in Sec. 6.2 (one
 *                   matvec = one preconditioner application + one operator
 *                   apply).
 *
 * Parity pins live in tests/test_oracle_pins.py (closed-form eigenpairs,
 * Lemma 3.1 box, Lemma 3.2 eigenvalue condition, CSL/CSG identity of eq.
 * (CSL-CSG), the 1D outgoing Green's function, dense direct solves, grid
 * transfer identities, Galerkin products, the ILU(0) factors' L U = M on the
 * pattern of M).  The multigrid convergence factor and the Krylov
 * iteration counts are "parity unpinned" by the paper (its numbers are for a
 * different smoother and coarse operator); they are checked only for
 * self-consistency and against the device path.
 *
 * Arithmetic contract (fixed operation order, shared by definition -- not by
 * code -- with the device path):
 *   complex multiply   (ar*br - ai*bi, ar*bi + ai*br)
 *   complex divide     d = br*br + bi*bi; ((ar*br + ai*bi)/d, (ai*br - ar*bi)/d)
 *   principal sqrt     of (x, y): r = sqrt(x*x + y*y); x >= 0: re = sqrt(0.5*(r + x)),
 *                      im = y/(2 re); x < 0: im = +-sqrt(0.5*(r - x)) (sign of y),
 *                      re = y/(2 im)
 *   Sommerfeld factor  hk = 0.5*k; rho = (1 + hk*w.im, -(hk*w.re)) / (1 - hk*w.im, hk*w.re)
 *                      (contract divide), d_last = d_last - c_last*rho (a_first*rho on the
 *                      low side), w = complex width from the last unknown to the ghost
 *   smooth contour     w = L/m; q = floor(t/w) (at most m); s = 0; for p = 1..q:
 *                      s = s + (w cos(p th/m), w sin(p th/m)); if q < m and t - q w > 0:
 *                      s = s + ((t - q w) cos((q+1) th/m), (t - q w) sin((q+1) th/m))
 *   stencil            y = Dg*u - a_x*u_w - c_x*u_e - a_y*u_s - c_y*u_n
 *                          - a_z*u_d - c_z*u_u,  Dg = (d_x + d_y + d_z) - phi
 *   Galerkin stencil   (2D levels >= 1) entries G_s = M_l[p, p + dx + nx*dy],
 *                      |dx|, |dy| <= 2, s = (dx+2) + 5(dy+2); y = G_12*u_p, then
 *                      y = y + G_s*u_q for s = 0..24 ascending, s != 12 (u_q = 0
 *                      outside); Dg = G_12.
 *                      Column J of M_{l+1} is R (M_l (P e_J)), computed with the
 *                      transfer and apply functions below.
 *   ILU(0) smoother    (2D, Sec. 6.1) on levels 0 .. nlev-2.  Stencil of M_l in the
 *                      Galerkin layout s = (dx+2) + 5(dy+2): the Galerkin stencil, or
 *                      on a rediscretised level the 5-point set s = 12: Dg, 11: -a_x,
 *                      13: -c_x, 7: -a_y, 17: -c_y (in-grid neighbours only).  Pattern:
 *                      the diagonal and the in-grid entries that are nonzero.  Rows p
 *                      ascending; in row p the pattern's columns q < p ascending:
 *                      l = a[p,q] / a[q,q] (contract divide), then for each pattern
 *                      column c > q of row p whose entry (q, c) is in row q's pattern:
 *                      a[p,c] = a[p,c] - l*a[q,c].  Stored: l below the diagonal,
 *                      u on and above it (zero off the pattern).  A sweep: r = f - M u
 *                      (stencil above); forward, p ascending: y = r_p, then
 *                      y = y - l_s*y_q over the level's offsets (the 5-point set, or all
 *                      25) below the diagonal, in-grid, columns ascending; backward, p
 *                      descending: z = y_p, z = z - u_s*z_c over those above the
 *                      diagonal, columns ascending, z = z / u_12 (contract divide);
 *                      u = u + omega*z (omega real, separate products).
 *   Jacobi weight      g = omega*conj(Dg)/|Dg|^2 : q = omega/(Dr*Dr + Di*Di),
 *                      g = (Dr*q, -(Di*q))
 *   reductions         chunks of 256 elements; slot t (0..255) of a chunk
 *                      holds 0.0 + its element (0.0 past the end); the 256
 *                      slots are summed by a pairwise (recursive halving)
 *                      tree; chunk partials are summed by a pairwise tree
 *                      after zero padding to a power of two.
 *   dense solves       LU with partial pivoting (first maximum of |re|+|im|),
 *                      k-i-j elimination, unit-lower forward substitution and
 *                      upper back substitution with ascending inner loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_MAXLEV 16
#define OG_PAR_MIN 16384   /* smaller loops run on one thread */

enum { OG_OK = 0, OG_ERR_ARG = -1, OG_ERR_NOCONV = -4, OG_ERR_BREAKDOWN = -5, OG_ERR_NONFINITE = -6 };

typedef struct { double re, im; } cx;

static inline cx cx_make(double re, double im) { cx z; z.re = re; z.im = im; return z; }
static inline cx cx_add(cx a, cx b) { return cx_make(a.re + b.re, a.im + b.im); }
static inline cx cx_sub(cx a, cx b) { return cx_make(a.re - b.re, a.im - b.im); }
static inline cx cx_mul(cx a, cx b) { return cx_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static inline cx cx_div(cx a, cx b)
{
    double d = b.re * b.re + b.im * b.im;
    return cx_make((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
static inline cx cx_rscale(double s, cx a) { return cx_make(s * a.re, s * a.im); }
static inline double cx_abs1(cx a) { return fabs(a.re) + fabs(a.im); }
static inline int cx_finite(cx a) { return isfinite(a.re) && isfinite(a.im); }

/* ------------------------------------------------------------------------ */
/* Grid, levels, coefficients                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;                 /* unknowns on this axis                         */
    cx *aH, *cH, *dH;      /* Helmholtz (ECS) lower/upper/centre, level 0    */
    cx *aM, *cM, *dM;      /* preconditioner (CSG) lower/upper/centre        */
} og_axis;

typedef struct {
    int n[3];
    long N;
    og_axis ax[3];
    double *phi;           /* N reals, x fastest                            */
    cx *gal;               /* Galerkin levels: 25 x N stencil (see the contract), else NULL */
    cx *ilu;               /* ILU(0) smoother: 25 x N factors (see the contract), else NULL */
} og_level;

typedef struct og_grid {
    int dim, nlev, centering, csg_mode, nu1, nu2;
    int coarse_op;             /* 0 rediscretised coarse operators, 1 Galerkin (2D)       */
    int smoother;              /* 0 weighted Jacobi, 1 ILU(0) (2D, V(0,1))                */
    double lo[3], hi[3], a[3], b[3];
    double th_ecs, th_csg, omega;
    double beta_re, beta_im;   /* CSG scale factor beta (CSL: principal sqrt of the shift) */
    int steps;                 /* ECS contour: <= 1 linear, m > 1 m equal angle steps   */
    int bc[3][2];              /* per axis and side: 0 Dirichlet, 1 Sommerfeld           */
    double k_bc;               /* wave number of the Sommerfeld condition                 */
    og_level lev[OG_MAXLEV];
    long Nc;
    cx *Minv;              /* Nc x Nc, row major: explicit inverse of the coarsest M */
} og_grid;

/* Linear ECS map of one real coordinate (Sec. 2): identity on [a,b], rotated
 * by e^{i th} on the layers, continuous at the turning points. */
static cx ecs_map(double x, double a, double b, double c, double s)
{
    if (x < a) { double t = x - a; return cx_make(a + t * c, t * s); }
    if (x > b) { double t = x - b; return cx_make(b + t * c, t * s); }
    return cx_make(x, 0.0);
}

/* Displacement of a smooth ECS contour from its turning point after a real
 * distance t >= 0 into a layer of real width L (Sec. 6.2, remark on a smooth
 * ECS transition): the layer is cut into m equal parts and part p is rotated
 * by p th / m, so the contour turns gradually to the angle th. */
static cx contour_disp(double t, double L, double th, int m)
{
    double w = L / (double)m;
    int q = (int)floor(t / w);
    if (q > m) q = m;
    if (q < 0) q = 0;
    cx s = cx_make(0.0, 0.0);
    for (int p = 1; p <= q; ++p) {
        double ang = th * (double)p / (double)m;
        s = cx_add(s, cx_make(w * cos(ang), w * sin(ang)));
    }
    double rem = t - (double)q * w;
    if (q < m && rem > 0.0) {
        double ang = th * (double)(q + 1) / (double)m;
        s = cx_add(s, cx_make(rem * cos(ang), rem * sin(ang)));
    }
    return s;
}

/* ECS map of one axis (linear, or smooth with g->steps > 1 parts). */
static cx ecs_map_axis(const og_grid *g, int ax, double x, double cg, double sg)
{
    double a = g->a[ax], b = g->b[ax];
    if (g->steps <= 1) return ecs_map(x, a, b, cg, sg);
    if (x < a) return cx_sub(cx_make(a, 0.0), contour_disp(a - x, a - g->lo[ax], g->th_ecs, g->steps));
    if (x > b) return cx_add(cx_make(b, 0.0), contour_disp(x - b, g->hi[ax] - b, g->th_ecs, g->steps));
    return cx_make(x, 0.0);
}

/* CSG map of the preconditioner (Sec. 5.3).  Uniform: every width of the ECS
 * grid is multiplied by beta (e^{i th_b}, or for the CSL the square root of
 * the shift, eq. (CSL-CSG)).  Interior: the interior widths are multiplied by
 * beta, the layer keeps the ECS contour. */
static cx csg_map_axis(const og_grid *g, int ax, double x, double cg, double sg)
{
    double a = g->a[ax], b = g->b[ax], cb = g->beta_re, sb = g->beta_im;
    if (g->csg_mode != 1) return cx_mul(cx_make(cb, sb), ecs_map_axis(g, ax, x, cg, sg));
    if (g->steps <= 1) {
        if (x < a) { double t = x - a; return cx_make(a * cb + t * cg, a * sb + t * sg); }
        if (x > b) { double t = x - b; return cx_make(b * cb + t * cg, b * sb + t * sg); }
        return cx_make(x * cb, x * sb);
    }
    if (x < a) return cx_sub(cx_make(a * cb, a * sb), contour_disp(a - x, a - g->lo[ax], g->th_ecs, g->steps));
    if (x > b) return cx_add(cx_make(b * cb, b * sb), contour_disp(x - b, g->hi[ax] - b, g->th_ecs, g->steps));
    return cx_make(x * cb, x * sb);
}

/* Principal square root of x + i y. */
static cx sqrt_principal(double x, double y)
{
    double r = sqrt(x * x + y * y);
    if (x >= 0.0) {
        double re = sqrt(0.5 * (r + x));
        return cx_make(re, y / (2.0 * re));
    }
    double im = sqrt(0.5 * (r - x));
    if (y < 0.0) im = -im;
    return cx_make(y / (2.0 * im), im);
}

/* Factor rho of the Sommerfeld ghost value u_ghost = rho u_last: the centred
 * difference of du/dn = -i k u at the boundary face between the last unknown
 * and a ghost at complex distance w, (u_g - u_l)/w = -i k (u_g + u_l)/2. */
static cx sommerfeld_rho(double k, cx w)
{
    double hk = 0.5 * k;
    cx num = cx_make(1.0 + hk * w.im, -(hk * w.re));
    cx den = cx_make(1.0 - hk * w.im, hk * w.re);
    return cx_div(num, den);
}

/* Real node coordinates of one axis with n unknowns: x[0] and x[n+1] are the
 * Dirichlet ends lo and hi. */
static void axis_nodes(int n, double lo, double hi, int centering, const int *bc, double *x)
{
    if (centering == 0) {
        double h = (hi - lo) / (double)n;
        /* a Sommerfeld side's end node is the ghost one cell beyond the last
         * unknown (the boundary is the face half a cell beyond it) */
        x[0] = bc[0] ? lo - 0.5 * h : lo;
        for (int j = 1; j <= n; ++j) x[j] = lo + ((double)j - 0.5) * h;
        x[n + 1] = bc[1] ? hi + 0.5 * h : hi;
    } else {
        double h = (hi - lo) / (double)(n + 1);
        x[0] = lo;
        for (int j = 1; j <= n; ++j) x[j] = lo + (double)j * h;
        x[n + 1] = hi;
    }
}

/* Shortley-Weller coefficients (Sec. 3, eq. (shortwell)) of -d^2/dz^2 at the
 * unknowns j = 1..n of complex nodes z[0..n+1]:
 *   -u'' ~ -a_j u_{j-1} + (a_j + c_j) u_j - c_j u_{j+1},
 *   a_j = 2 / (hl (hl + hr)),  c_j = 2 / (hr (hl + hr)). */
static void sw_coeffs(int n, const cx *z, cx *A, cx *C, cx *D)
{
    for (int j = 1; j <= n; ++j) {
        cx hl = cx_sub(z[j], z[j - 1]);
        cx hr = cx_sub(z[j + 1], z[j]);
        cx s = cx_add(hl, hr);
        cx two = cx_make(2.0, 0.0);
        cx aj = cx_div(two, cx_mul(hl, s));
        cx cj = cx_div(two, cx_mul(hr, s));
        A[j - 1] = aj;
        C[j - 1] = cj;
        D[j - 1] = cx_add(aj, cj);
    }
}

static void build_axis(og_grid *g, int lev, int ax)
{
    og_axis *A = &g->lev[lev].ax[ax];
    int n = A->n;
    double *x = (double *)malloc(sizeof(double) * (size_t)(n + 2));
    cx *zH = (cx *)malloc(sizeof(cx) * (size_t)(n + 2));
    cx *zM = (cx *)malloc(sizeof(cx) * (size_t)(n + 2));
    axis_nodes(n, g->lo[ax], g->hi[ax], g->centering, g->bc[ax], x);
    double cg = cos(g->th_ecs), sg = sin(g->th_ecs);
    for (int j = 0; j <= n + 1; ++j) {
        zH[j] = ecs_map_axis(g, ax, x[j], cg, sg);
        zM[j] = csg_map_axis(g, ax, x[j], cg, sg);
    }
    /* a Sommerfeld side has no layer: its ghost continues the interior map
     * (real for H, scaled by beta for M) */
    for (int side = 0; side < 2; ++side) {
        if (!g->bc[ax][side]) continue;
        int j = side == 0 ? 0 : n + 1;
        zH[j] = cx_make(x[j], 0.0);
        zM[j] = cx_make(g->beta_re * x[j], g->beta_im * x[j]);
    }
    size_t bytes = sizeof(cx) * (size_t)n;
    A->aH = (cx *)malloc(bytes); A->cH = (cx *)malloc(bytes); A->dH = (cx *)malloc(bytes);
    A->aM = (cx *)malloc(bytes); A->cM = (cx *)malloc(bytes); A->dM = (cx *)malloc(bytes);
    sw_coeffs(n, zH, A->aH, A->cH, A->dH);
    sw_coeffs(n, zM, A->aM, A->cM, A->dM);
    /* Sommerfeld sides: eliminate the ghost (its coefficient moves onto the
     * diagonal of the unknown next to the boundary); the preconditioner takes
     * the condition in its own stretched coordinate (its complex widths) */
    if (g->bc[ax][0]) {
        cx rH = sommerfeld_rho(g->k_bc, cx_sub(zH[1], zH[0])), rM = sommerfeld_rho(g->k_bc, cx_sub(zM[1], zM[0]));
        A->dH[0] = cx_sub(A->dH[0], cx_mul(A->aH[0], rH));
        A->dM[0] = cx_sub(A->dM[0], cx_mul(A->aM[0], rM));
    }
    if (g->bc[ax][1]) {
        cx rH = sommerfeld_rho(g->k_bc, cx_sub(zH[n + 1], zH[n])), rM = sommerfeld_rho(g->k_bc, cx_sub(zM[n + 1], zM[n]));
        A->dH[n - 1] = cx_sub(A->dH[n - 1], cx_mul(A->cH[n - 1], rH));
        A->dM[n - 1] = cx_sub(A->dM[n - 1], cx_mul(A->cM[n - 1], rM));
    }
    free(x); free(zH); free(zM);
}

/* Coarse phi: mean of the 2^d children, summed z-then-y-then-x outermost to
 * innermost, scaled by 2^-d. */
static void coarsen_phi(const og_level *F, og_level *C, int dim)
{
    double scale = dim == 1 ? 0.5 : (dim == 2 ? 0.25 : 0.125);
    int cz = dim >= 3 ? 2 : 1, cy = dim >= 2 ? 2 : 1;
    for (int k = 0; k < C->n[2]; ++k)
        for (int j = 0; j < C->n[1]; ++j)
            for (int i = 0; i < C->n[0]; ++i) {
                double s = 0.0;
                for (int dz = 0; dz < cz; ++dz)
                    for (int dy = 0; dy < cy; ++dy)
                        for (int dx = 0; dx < 2; ++dx) {
                            long fi = (long)(2 * i + dx) + (long)F->n[0] * ((long)(cy == 2 ? 2 * j + dy : j) + (long)F->n[1] * (long)(cz == 2 ? 2 * k + dz : k));
                            s = s + F->phi[fi];
                        }
                C->phi[(long)i + (long)C->n[0] * ((long)j + (long)C->n[1] * (long)k)] = s * scale;
            }
}

/* ------------------------------------------------------------------------ */
/* Operator apply                                                            */
/* ------------------------------------------------------------------------ */

static inline cx diag_at(const og_level *L, int dim, int op, int i, int j, int k, long p)
{
    if (op == 1 && L->gal) return L->gal[12 * L->N + p];
    cx d = op == 0 ? L->ax[0].dH[i] : L->ax[0].dM[i];
    if (dim >= 2) d = cx_add(d, op == 0 ? L->ax[1].dH[j] : L->ax[1].dM[j]);
    if (dim >= 3) d = cx_add(d, op == 0 ? L->ax[2].dH[k] : L->ax[2].dM[k]);
    return cx_make(d.re - L->phi[p], d.im);
}

/* y = A x on level lev, A = H (op 0, ECS coefficients) or M (op 1, CSG
 * coefficients); values outside the grid are the Dirichlet zero. */
static void apply_level(const og_grid *g, int op, int lev, const cx *x, cx *y)
{
    const og_level *L = &g->lev[lev];
    int dim = g->dim, nx = L->n[0], ny = L->n[1], nz = L->n[2];
    long sy = nx, sz = (long)nx * ny;
    const cx zero = cx_make(0.0, 0.0);
    if (op == 1 && L->gal) {
        /* Galerkin level (2D): the stored 25-point stencil */
        const cx *G = L->gal;
        long N = L->N;
#pragma omp parallel for schedule(static) if (L->N > OG_PAR_MIN)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = (long)i + sy * j;
                cx t = cx_mul(G[12 * N + p], x[p]);
                for (int s = 0; s < 25; ++s) {
                    if (s == 12) continue;
                    int ii = i + s % 5 - 2, jj = j + s / 5 - 2;
                    cx xq = (ii >= 0 && ii < nx && jj >= 0 && jj < ny) ? x[(long)ii + sy * jj] : zero;
                    t = cx_add(t, cx_mul(G[s * N + p], xq));
                }
                y[p] = t;
            }
        return;
    }
#pragma omp parallel for schedule(static) if (L->N > OG_PAR_MIN)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = (long)i + sy * j + sz * k;
                cx t = cx_mul(diag_at(L, dim, op, i, j, k, p), x[p]);
                const og_axis *X = &L->ax[0];
                cx uw = i > 0 ? x[p - 1] : zero, ue = i < nx - 1 ? x[p + 1] : zero;
                t = cx_sub(t, cx_mul(op == 0 ? X->aH[i] : X->aM[i], uw));
                t = cx_sub(t, cx_mul(op == 0 ? X->cH[i] : X->cM[i], ue));
                if (dim >= 2) {
                    const og_axis *Y = &L->ax[1];
                    cx us = j > 0 ? x[p - sy] : zero, un = j < ny - 1 ? x[p + sy] : zero;
                    t = cx_sub(t, cx_mul(op == 0 ? Y->aH[j] : Y->aM[j], us));
                    t = cx_sub(t, cx_mul(op == 0 ? Y->cH[j] : Y->cM[j], un));
                }
                if (dim >= 3) {
                    const og_axis *Z = &L->ax[2];
                    cx ud = k > 0 ? x[p - sz] : zero, uu = k < nz - 1 ? x[p + sz] : zero;
                    t = cx_sub(t, cx_mul(op == 0 ? Z->aH[k] : Z->aM[k], ud));
                    t = cx_sub(t, cx_mul(op == 0 ? Z->cH[k] : Z->cM[k], uu));
                }
                y[p] = t;
            }
}

/* ------------------------------------------------------------------------ */
/* Reductions (fixed blocked pairwise order)                                 */
/* ------------------------------------------------------------------------ */

#define OG_SLOTS 256
#define OG_PER_SLOT 1
#define OG_CHUNK (OG_SLOTS * OG_PER_SLOT)

/* Pairwise (recursive halving) sum of v[0..n), n a power of two. */
static double pairwise(const double *v, long n)
{
    if (n == 1) return v[0];
    long h = n / 2;
    return pairwise(v, h) + pairwise(v + h, h);
}

static long next_pow2(long n)
{
    long p = 1;
    while (p < n) p *= 2;
    return p;
}

/* Sum of term(e) over e = 0..n-1 in the contract order.  kind 0: Re conj(x)y,
 * kind 1: Im conj(x)y, kind 2: |x|^2. */
static double term(int kind, const cx *x, const cx *y, long e)
{
    cx a = x[e];
    if (kind == 2) return a.re * a.re + a.im * a.im;
    cx b = y[e];
    if (kind == 0) return a.re * b.re + a.im * b.im;
    return a.re * b.im - a.im * b.re;
}

static double blocked_sum(int kind, const cx *x, const cx *y, long n)
{
    long nch = (n + OG_CHUNK - 1) / OG_CHUNK;
    if (nch == 0) return 0.0;
    long np = next_pow2(nch);
    double *part = (double *)calloc((size_t)np, sizeof(double));
#pragma omp parallel for schedule(static) if (n > OG_PAR_MIN)
    for (long c = 0; c < nch; ++c) {
        double slot[OG_SLOTS];
        for (int t = 0; t < OG_SLOTS; ++t) {
            double acc = 0.0;
            for (int j = 0; j < OG_PER_SLOT; ++j) {
                long e = c * OG_CHUNK + t + (long)OG_SLOTS * j;
                if (e < n) acc = acc + term(kind, x, y, e);
            }
            slot[t] = acc;
        }
        part[c] = pairwise(slot, OG_SLOTS);
    }
    double s = pairwise(part, np);
    free(part);
    return s;
}

static cx dotc(const cx *x, const cx *y, long n)
{
    return cx_make(blocked_sum(0, x, y, n), blocked_sum(1, x, y, n));
}

static double nrm2(const cx *x, long n) { return sqrt(blocked_sum(2, x, x, n)); }

/* Pairwise sum of exactly n values (zero padded to a power of two). */
static double pairwise_padded(const double *v, long n)
{
    long np = next_pow2(n);
    double *w = (double *)calloc((size_t)np, sizeof(double));
    memcpy(w, v, sizeof(double) * (size_t)n);
    double s = pairwise(w, np);
    free(w);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting, explicit inverse                         */
/* ------------------------------------------------------------------------ */

/* In-place LU of the n x n row-major matrix A with row permutation perm.
 * Returns 0, or -1 for an exactly singular pivot. */
static int lu_factor(cx *A, int n, int *perm)
{
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cx_abs1(A[(long)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = cx_abs1(A[(long)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                cx t = A[(long)k * n + j];
                A[(long)k * n + j] = A[(long)p * n + j];
                A[(long)p * n + j] = t;
            }
            int t = perm[k]; perm[k] = perm[p]; perm[p] = t;
        }
        cx piv = A[(long)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            cx l = cx_div(A[(long)i * n + k], piv);
            A[(long)i * n + k] = l;
            for (int j = k + 1; j < n; ++j)
                A[(long)i * n + j] = cx_sub(A[(long)i * n + j], cx_mul(l, A[(long)k * n + j]));
        }
    }
    return 0;
}

/* Solve LU x = P b for one right-hand side (x may alias nothing). */
static void lu_solve(const cx *LU, int n, const int *perm, const cx *b, cx *x)
{
    for (int i = 0; i < n; ++i) {
        cx s = b[perm[i]];
        for (int j = 0; j < i; ++j) s = cx_sub(s, cx_mul(LU[(long)i * n + j], x[j]));
        x[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        cx s = x[i];
        for (int j = i + 1; j < n; ++j) s = cx_sub(s, cx_mul(LU[(long)i * n + j], x[j]));
        x[i] = cx_div(s, LU[(long)i * n + i]);
    }
}

/* Dense matrix of M on the coarsest level: column q is M applied to the unit
 * vector e_q. */
static int build_coarse_inverse(og_grid *g)
{
    int L = g->nlev - 1;
    long n = g->lev[L].N;
    g->Nc = n;
    cx *A = (cx *)calloc((size_t)(n * n), sizeof(cx));
    cx *e = (cx *)calloc((size_t)n, sizeof(cx));
    cx *col = (cx *)calloc((size_t)n, sizeof(cx));
    for (long q = 0; q < n; ++q) {
        e[q] = cx_make(1.0, 0.0);
        apply_level(g, 1, L, e, col);
        e[q] = cx_make(0.0, 0.0);
        for (long p = 0; p < n; ++p) A[p * n + q] = col[p];
    }
    int *perm = (int *)malloc(sizeof(int) * (size_t)n);
    int rc = lu_factor(A, (int)n, perm);
    g->Minv = (cx *)calloc((size_t)(n * n), sizeof(cx));
    if (rc == 0) {
        cx *x = (cx *)calloc((size_t)n, sizeof(cx));
        for (long c = 0; c < n; ++c) {
            for (long p = 0; p < n; ++p) e[p] = cx_make(p == c ? 1.0 : 0.0, 0.0);
            lu_solve(A, (int)n, perm, e, x);
            for (long p = 0; p < n; ++p) g->Minv[p * n + c] = x[p];
        }
        free(x);
    }
    free(A); free(e); free(col); free(perm);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Creation                                                                  */
/* ------------------------------------------------------------------------ */

void og_free(og_grid *g);
static void restrict_level(const og_grid *g, int lev, const cx *r, cx *rc);
static void prolong_level(const og_grid *g, int lev, const cx *ec, cx *ef);

/* Galerkin coarse operators (Sec. 6.1): M_{l+1} = R M_l P for levels 1 ..
 * nlev-1 in turn, M_0 the rediscretised preconditioner of the finest level.
 * Column J of M_{l+1} is R (M_l (P e_J)), from the same transfer and apply
 * functions the V-cycle uses.  P e_J covers fine cells 2J-1 .. 2J+2 per
 * axis, M_l widens that by its bandwidth (1 on level 0, 2 below), and a
 * restriction row covers four fine cells, so the nonzeros lie on the 5 x 5
 * coarse points around J; a nonzero anywhere else is reported as an error. */
static int build_galerkin(og_grid *g)
{
    int bad = 0;
    for (int l = 1; l < g->nlev; ++l) {
        og_level *C = &g->lev[l];
        const og_level *F = &g->lev[l - 1];
        const long Nc = C->N, Nf = F->N;
        const int cxn = C->n[0];
        C->gal = (cx *)calloc((size_t)(25 * Nc), sizeof(cx));
#pragma omp parallel
        {
            cx *e = (cx *)calloc((size_t)Nc, sizeof(cx));
            cx *w = (cx *)malloc(sizeof(cx) * (size_t)Nf);
            cx *y = (cx *)malloc(sizeof(cx) * (size_t)Nf);
            cx *z = (cx *)malloc(sizeof(cx) * (size_t)Nc);
#pragma omp for schedule(dynamic, 16)
            for (long J = 0; J < Nc; ++J) {
                e[J] = cx_make(1.0, 0.0);
                prolong_level(g, l - 1, e, w);
                apply_level(g, 1, l - 1, w, y);
                restrict_level(g, l - 1, y, z);
                e[J] = cx_make(0.0, 0.0);
                const int Jx = (int)(J % cxn), Jy = (int)(J / cxn);
                for (long I = 0; I < Nc; ++I) {
                    const int dx = Jx - (int)(I % cxn), dy = Jy - (int)(I / cxn);
                    if (dx >= -2 && dx <= 2 && dy >= -2 && dy <= 2) {
                        C->gal[((dx + 2) + 5 * (dy + 2)) * Nc + I] = z[I];
                    } else if (z[I].re != 0.0 || z[I].im != 0.0) {
#pragma omp atomic write
                        bad = 1;
                    }
                }
            }
            free(e); free(w); free(y); free(z);
        }
    }
    return bad ? OG_ERR_ARG : OG_OK;
}

/* Entry s (Galerkin layout, s = (dx+2) + 5(dy+2)) of row p of M_l, 2D; zero
 * for a neighbour outside the grid and, on a rediscretised level, off the
 * 5-point set. */
static cx level_entry(const og_grid *g, int lev, int s, int i, int j)
{
    const og_level *L = &g->lev[lev];
    int nx = L->n[0], ny = L->n[1], dx = s % 5 - 2, dy = s / 5 - 2;
    long p = (long)i + (long)nx * j;
    if (i + dx < 0 || i + dx >= nx || j + dy < 0 || j + dy >= ny) return cx_make(0.0, 0.0);
    if (L->gal) return L->gal[s * L->N + p];
    const og_axis *X = &L->ax[0], *Y = &L->ax[1];
    if (s == 12) return diag_at(L, 2, 1, i, j, 0, p);
    if (s == 11) return cx_make(-X->aM[i].re, -X->aM[i].im);
    if (s == 13) return cx_make(-X->cM[i].re, -X->cM[i].im);
    if (s == 7) return cx_make(-Y->aM[j].re, -Y->aM[j].im);
    if (s == 17) return cx_make(-Y->cM[j].re, -Y->cM[j].im);
    return cx_make(0.0, 0.0);
}

/* The level's stencil offsets (the 5-point set or all 25) in ascending
 * column order (column offset dx + nx*dy); returns their count. */
static int level_offsets(const og_level *L, int *ord)
{
    int m = 0, nx = L->n[0];
    for (int s = 0; s < 25; ++s)
        if (L->gal || s == 7 || s == 11 || s == 12 || s == 13 || s == 17) ord[m++] = s;
    for (int a = 1; a < m; ++a)   /* insertion sort by column offset */
        for (int b = a; b > 0; --b) {
            int s0 = ord[b - 1], s1 = ord[b];
            long c0 = (s0 % 5 - 2) + (long)nx * (s0 / 5 - 2), c1 = (s1 % 5 - 2) + (long)nx * (s1 / 5 - 2);
            if (c0 <= c1) break;
            ord[b - 1] = s1; ord[b] = s0;
        }
    return m;
}

/* ILU(0) of M_l on its nonzero pattern (Saad's row-wise incomplete
 * elimination), for the smoothing levels 0 .. nlev-2.  Fails on a zero
 * pivot. */
static int build_ilu(og_grid *g)
{
    for (int l = 0; l + 1 < g->nlev; ++l) {
        og_level *L = &g->lev[l];
        const long N = L->N;
        const int nx = L->n[0], ny = L->n[1];
        int ord[25];
        const int m = level_offsets(L, ord);
        cx *a = (cx *)calloc((size_t)(25 * N), sizeof(cx));
        unsigned char *pat = (unsigned char *)calloc((size_t)(25 * N), 1);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = (long)i + (long)nx * j;
                for (int k = 0; k < m; ++k) {
                    int s = ord[k];
                    cx v = level_entry(g, l, s, i, j);
                    int dx = s % 5 - 2, dy = s / 5 - 2;
                    int in = i + dx >= 0 && i + dx < nx && j + dy >= 0 && j + dy < ny;
                    if (in && (s == 12 || v.re != 0.0 || v.im != 0.0)) { a[s * N + p] = v; pat[s * N + p] = 1; }
                }
            }
        int bad = 0;
        for (long p = 0; p < N && !bad; ++p) {
            for (int k = 0; k < m; ++k) {
                int s = ord[k];
                long cs = (s % 5 - 2) + (long)nx * (s / 5 - 2);
                if (cs >= 0) break;                       /* diagonal reached */
                if (!pat[s * N + p]) continue;
                long q = p + cs;
                cx piv = a[12 * N + q];
                if (piv.re == 0.0 && piv.im == 0.0) { bad = 1; break; }
                cx lv = cx_div(a[s * N + p], piv);
                a[s * N + p] = lv;
                for (int kk = k + 1; kk < m; ++kk) {
                    int t = ord[kk];
                    if (!pat[t * N + p]) continue;
                    int ux = (t % 5) - (s % 5), uy = (t / 5) - (s / 5);   /* offset of (q, c) from q */
                    if (ux < -2 || ux > 2 || uy < -2 || uy > 2) continue;
                    long cu = (long)ux + (long)nx * uy;
                    if (cu <= 0) continue;                    /* only row q's upper part */
                    int u = (ux + 2) + 5 * (uy + 2);
                    if (!pat[u * N + q]) continue;
                    a[t * N + p] = cx_sub(a[t * N + p], cx_mul(lv, a[u * N + q]));
                }
            }
        }
        free(pat);
        if (bad) { free(a); return OG_ERR_ARG; }
        L->ilu = a;
    }
    return OG_OK;
}

/* One ILU(0) sweep u <- u + omega (L U)^{-1} (f - M u) on level lev. */
static void ilu_sweep(const og_grid *g, int lev, const cx *f, cx *u, cx *tmp)
{
    const og_level *L = &g->lev[lev];
    const long N = L->N;
    const int nx = L->n[0], ny = L->n[1];
    const cx *F = L->ilu;
    int ord[25];
    const int m = level_offsets(L, ord);
    apply_level(g, 1, lev, u, tmp);
    for (long p = 0; p < N; ++p) tmp[p] = cx_sub(f[p], tmp[p]);
    for (long p = 0; p < N; ++p) {
        int i = (int)(p % nx), j = (int)(p / nx);
        cx y = tmp[p];
        for (int k = 0; k < m; ++k) {
            int s = ord[k], dx = s % 5 - 2, dy = s / 5 - 2;
            if (dx + (long)nx * dy >= 0) break;
            if (i + dx < 0 || i + dx >= nx || j + dy < 0 || j + dy >= ny) continue;
            y = cx_sub(y, cx_mul(F[s * N + p], tmp[p + dx + (long)nx * dy]));
        }
        tmp[p] = y;
    }
    for (long p = N - 1; p >= 0; --p) {
        int i = (int)(p % nx), j = (int)(p / nx);
        cx z = tmp[p];
        for (int k = 0; k < m; ++k) {
            int s = ord[k], dx = s % 5 - 2, dy = s / 5 - 2;
            if (dx + (long)nx * dy <= 0) continue;
            if (i + dx < 0 || i + dx >= nx || j + dy < 0 || j + dy >= ny) continue;
            z = cx_sub(z, cx_mul(F[s * N + p], tmp[p + dx + (long)nx * dy]));
        }
        tmp[p] = cx_div(z, F[12 * N + p]);
    }
    for (long p = 0; p < N; ++p) u[p] = cx_add(u[p], cx_rscale(g->omega, tmp[p]));
}

/* csg_mode: 0 uniform CSG, 1 interior CSG, 2 CSL with shift (shift_re,
 * shift_im); contour_steps: ECS contour parts (<= 1 linear); bc: 6 ints, per
 * axis (low side, high side), 1 = Sommerfeld with wave number k_bc. */
og_grid *og_create(int dim, const int *n, const double *lo, const double *hi,
                   const double *a, const double *b, double theta_ecs, double theta_csg,
                   int csg_mode, int centering, int levels, int nu1, int nu2, double omega,
                   const double *phi, double shift_re, double shift_im, int contour_steps,
                   const int *bc, double k_bc, int coarse_op, int smoother)
{
    if (dim < 1 || dim > 3) return NULL;
    if (coarse_op != 0 && (coarse_op != 1 || dim != 2 || centering != 0)) return NULL;
    if (smoother != 0 && (smoother != 1 || dim != 2 || centering != 0 || nu1 != 0)) return NULL;
    og_grid *g = (og_grid *)calloc(1, sizeof(og_grid));
    g->dim = dim; g->centering = centering; g->csg_mode = csg_mode; g->coarse_op = coarse_op;
    g->smoother = smoother;
    g->nu1 = nu1; g->nu2 = nu2; g->omega = omega;
    g->th_ecs = theta_ecs; g->th_csg = theta_csg;
    g->steps = contour_steps;
    g->k_bc = k_bc;
    for (int d = 0; d < 3; ++d) {
        g->bc[d][0] = bc && d < dim ? bc[2 * d] : 0;
        g->bc[d][1] = bc && d < dim ? bc[2 * d + 1] : 0;
    }
    if (csg_mode == 2) {
        cx be = sqrt_principal(shift_re, shift_im);
        g->beta_re = be.re; g->beta_im = be.im;
    } else {
        g->beta_re = cos(theta_csg); g->beta_im = sin(theta_csg);
    }
    int n0[3] = {1, 1, 1};
    for (int d = 0; d < 3; ++d) {
        if (d < dim) {
            n0[d] = n[d]; g->lo[d] = lo[d]; g->hi[d] = hi[d]; g->a[d] = a[d]; g->b[d] = b[d];
            if (n[d] < 1) { free(g); return NULL; }
        }
    }
    /* Level count: given, or halve while every side is even and the largest
     * side exceeds 16 (1D/2D) or 8 (3D). */
    int nl = levels;
    if (nl <= 0) {
        int thr = dim == 3 ? 8 : 16;
        int m[3] = {n0[0], n0[1], n0[2]};
        nl = 1;
        for (;;) {
            int even = 1, mx = 0;
            for (int d = 0; d < dim; ++d) { if (m[d] % 2) even = 0; if (m[d] > mx) mx = m[d]; }
            if (!even || mx <= thr || nl >= OG_MAXLEV) break;
            for (int d = 0; d < dim; ++d) m[d] /= 2;
            ++nl;
        }
    }
    if (nl > OG_MAXLEV || (centering == 1 && nl != 1)) { free(g); return NULL; }
    for (int d = 0; d < dim; ++d)
        if (n0[d] % (1 << (nl - 1))) { free(g); return NULL; }
    g->nlev = nl;
    for (int l = 0; l < nl; ++l) {
        og_level *L = &g->lev[l];
        for (int d = 0; d < 3; ++d) L->n[d] = d < dim ? n0[d] >> l : 1;
        L->N = (long)L->n[0] * L->n[1] * L->n[2];
        for (int d = 0; d < dim; ++d) { L->ax[d].n = L->n[d]; build_axis(g, l, d); }
        L->phi = (double *)malloc(sizeof(double) * (size_t)L->N);
        if (l == 0) memcpy(L->phi, phi, sizeof(double) * (size_t)L->N);
        else coarsen_phi(&g->lev[l - 1], L, dim);
    }
    if (coarse_op == 1 && (nl < 2 || build_galerkin(g) != 0)) { og_free(g); return NULL; }
    if (smoother == 1 && build_ilu(g) != 0) { og_free(g); return NULL; }
    if (build_coarse_inverse(g) != 0) { og_free(g); return NULL; }
    return g;
}

void og_free(og_grid *g)
{
    if (!g) return;
    for (int l = 0; l < g->nlev; ++l) {
        og_level *L = &g->lev[l];
        for (int d = 0; d < g->dim; ++d) {
            og_axis *A = &L->ax[d];
            free(A->aH); free(A->cH); free(A->dH); free(A->aM); free(A->cM); free(A->dM);
        }
        free(L->phi);
        free(L->gal);
        free(L->ilu);
    }
    free(g->Minv);
    free(g);
}

int og_levels(const og_grid *g) { return g->nlev; }

void og_level_dims(const og_grid *g, int lev, int *n)
{
    for (int d = 0; d < 3; ++d) n[d] = g->lev[lev].n[d];
}

long og_coarse_size(const og_grid *g) { return g->Nc; }

/* which: 0 aH, 1 cH, 2 dH, 3 aM, 4 cM, 5 dM.  Writes n complex values. */
int og_coeffs(const og_grid *g, int lev, int axis, int which, double *out)
{
    if (lev < 0 || lev >= g->nlev || axis < 0 || axis >= g->dim) return OG_ERR_ARG;
    const og_axis *A = &g->lev[lev].ax[axis];
    const cx *src = which == 0 ? A->aH : which == 1 ? A->cH : which == 2 ? A->dH
                  : which == 3 ? A->aM : which == 4 ? A->cM : A->dM;
    memcpy(out, src, sizeof(cx) * (size_t)A->n);
    return A->n;
}

int og_phi(const og_grid *g, int lev, double *out)
{
    if (lev < 0 || lev >= g->nlev) return OG_ERR_ARG;
    memcpy(out, g->lev[lev].phi, sizeof(double) * (size_t)g->lev[lev].N);
    return OG_OK;
}

/* The Galerkin stencil of level lev (25 x N complex values, entry s of point
 * p at s*N + p); OG_ERR_ARG if the level has none. */
int og_galerkin(const og_grid *g, int lev, double *out)
{
    if (lev < 1 || lev >= g->nlev || !g->lev[lev].gal) return OG_ERR_ARG;
    memcpy(out, g->lev[lev].gal, sizeof(cx) * (size_t)(25 * g->lev[lev].N));
    return OG_OK;
}

int og_ilu(const og_grid *g, int lev, double *out)
{
    if (lev < 0 || lev >= g->nlev || !g->lev[lev].ilu) return OG_ERR_ARG;
    memcpy(out, g->lev[lev].ilu, sizeof(cx) * (size_t)(25 * g->lev[lev].N));
    return OG_OK;
}

void og_coarse_inverse(const og_grid *g, double *out)
{
    memcpy(out, g->Minv, sizeof(cx) * (size_t)(g->Nc * g->Nc));
}

void og_apply(const og_grid *g, int op, int lev, const double *x, double *y)
{
    apply_level(g, op, lev, (const cx *)x, (cx *)y);
}

/* ------------------------------------------------------------------------ */
/* Multigrid components                                                      */
/* ------------------------------------------------------------------------ */

/* One weighted-Jacobi sweep u <- u + omega D^{-1} (f - M u) on level lev. */
static void jacobi(const og_grid *g, int lev, const cx *f, cx *u, cx *tmp)
{
    const og_level *L = &g->lev[lev];
    apply_level(g, 1, lev, u, tmp);
    int nx = L->n[0], ny = L->n[1], nz = L->n[2];
#pragma omp parallel for schedule(static) if (L->N > OG_PAR_MIN)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = (long)i + (long)nx * ((long)j + (long)ny * k);
                cx D = diag_at(L, g->dim, 1, i, j, k, p);
                double q = g->omega / (D.re * D.re + D.im * D.im);
                cx w = cx_make(D.re * q, -(D.im * q));
                tmp[p] = cx_add(u[p], cx_mul(w, cx_sub(f[p], tmp[p])));
            }
    memcpy(u, tmp, sizeof(cx) * (size_t)L->N);
}

/* Full-weighting restriction for cell-centred grids, per axis the weights
 * (1,3,3,1)/8 on fine cells 2I-1, 2I, 2I+1, 2I+2 (zero outside), applied axis
 * by axis x, then y, then z. */
static const double RW[4] = {0.125, 0.375, 0.375, 0.125};

static void restrict_level(const og_grid *g, int lev, const cx *r, cx *rc)
{
    const og_level *F = &g->lev[lev], *C = &g->lev[lev + 1];
    int dim = g->dim;
    int fx = F->n[0], fy = F->n[1], fz = F->n[2];
    int cxn = C->n[0], cyn = C->n[1], czn = C->n[2];
    /* stage 1: x */
    cx *t1 = (cx *)malloc(sizeof(cx) * (size_t)cxn * fy * fz);
#pragma omp parallel for schedule(static) if (F->N > OG_PAR_MIN)
    for (int k = 0; k < fz; ++k)
        for (int j = 0; j < fy; ++j)
            for (int I = 0; I < cxn; ++I) {
                cx s = cx_make(0.0, 0.0);
                for (int q = 0; q < 4; ++q) {
                    int i = 2 * I - 1 + q;
                    cx v = (i >= 0 && i < fx) ? r[(long)i + (long)fx * ((long)j + (long)fy * k)] : cx_make(0.0, 0.0);
                    s = q == 0 ? cx_rscale(RW[q], v) : cx_add(s, cx_rscale(RW[q], v));
                }
                t1[(long)I + (long)cxn * ((long)j + (long)fy * k)] = s;
            }
    if (dim == 1) { memcpy(rc, t1, sizeof(cx) * (size_t)cxn); free(t1); return; }
    /* stage 2: y */
    cx *t2 = (cx *)malloc(sizeof(cx) * (size_t)cxn * cyn * fz);
#pragma omp parallel for schedule(static) if (F->N > OG_PAR_MIN)
    for (int k = 0; k < fz; ++k)
        for (int J = 0; J < cyn; ++J)
            for (int I = 0; I < cxn; ++I) {
                cx s = cx_make(0.0, 0.0);
                for (int q = 0; q < 4; ++q) {
                    int j = 2 * J - 1 + q;
                    cx v = (j >= 0 && j < fy) ? t1[(long)I + (long)cxn * ((long)j + (long)fy * k)] : cx_make(0.0, 0.0);
                    s = q == 0 ? cx_rscale(RW[q], v) : cx_add(s, cx_rscale(RW[q], v));
                }
                t2[(long)I + (long)cxn * ((long)J + (long)cyn * k)] = s;
            }
    free(t1);
    if (dim == 2) { memcpy(rc, t2, sizeof(cx) * (size_t)cxn * cyn); free(t2); return; }
    /* stage 3: z */
#pragma omp parallel for schedule(static) if (F->N > OG_PAR_MIN)
    for (int K = 0; K < czn; ++K)
        for (int J = 0; J < cyn; ++J)
            for (int I = 0; I < cxn; ++I) {
                cx s = cx_make(0.0, 0.0);
                for (int q = 0; q < 4; ++q) {
                    int k = 2 * K - 1 + q;
                    cx v = (k >= 0 && k < fz) ? t2[(long)I + (long)cxn * ((long)J + (long)cyn * k)] : cx_make(0.0, 0.0);
                    s = q == 0 ? cx_rscale(RW[q], v) : cx_add(s, cx_rscale(RW[q], v));
                }
                rc[(long)I + (long)cxn * ((long)J + (long)cyn * K)] = s;
            }
    free(t2);
}

/* Bilinear/trilinear prolongation for cell-centred grids: along each axis the
 * fine cell 2I takes 3/4 of coarse cell I and 1/4 of cell I-1, fine cell
 * 2I+1 takes 3/4 of I and 1/4 of I+1 (zero outside), applied x, then y,
 * then z.  ef = P ec. */
static void prolong_level(const og_grid *g, int lev, const cx *ec, cx *ef)
{
    const og_level *F = &g->lev[lev], *C = &g->lev[lev + 1];
    int dim = g->dim;
    int fx = F->n[0], fy = F->n[1], fz = F->n[2];
    int cxn = C->n[0], cyn = C->n[1], czn = C->n[2];
    const cx zero = cx_make(0.0, 0.0);
    cx *t1 = (cx *)malloc(sizeof(cx) * (size_t)fx * cyn * czn);
#pragma omp parallel for schedule(static) if (F->N > OG_PAR_MIN)
    for (int K = 0; K < czn; ++K)
        for (int J = 0; J < cyn; ++J)
            for (int i = 0; i < fx; ++i) {
                int I = i / 2, Io = (i % 2) ? I + 1 : I - 1;
                long row = (long)cxn * ((long)J + (long)cyn * K);
                cx near = ec[row + I];
                cx far = (Io >= 0 && Io < cxn) ? ec[row + Io] : zero;
                t1[(long)i + (long)fx * ((long)J + (long)cyn * K)] = cx_add(cx_rscale(0.75, near), cx_rscale(0.25, far));
            }
    if (dim == 1) { memcpy(ef, t1, sizeof(cx) * (size_t)fx); free(t1); return; }
    cx *t2 = (cx *)malloc(sizeof(cx) * (size_t)fx * fy * czn);
#pragma omp parallel for schedule(static) if (F->N > OG_PAR_MIN)
    for (int K = 0; K < czn; ++K)
        for (int j = 0; j < fy; ++j)
            for (int i = 0; i < fx; ++i) {
                int J = j / 2, Jo = (j % 2) ? J + 1 : J - 1;
                cx near = t1[(long)i + (long)fx * ((long)J + (long)cyn * K)];
                cx far = (Jo >= 0 && Jo < cyn) ? t1[(long)i + (long)fx * ((long)Jo + (long)cyn * K)] : zero;
                t2[(long)i + (long)fx * ((long)j + (long)fy * K)] = cx_add(cx_rscale(0.75, near), cx_rscale(0.25, far));
            }
    free(t1);
    if (dim == 2) { memcpy(ef, t2, sizeof(cx) * (size_t)fx * fy); free(t2); return; }
#pragma omp parallel for schedule(static) if (F->N > OG_PAR_MIN)
    for (int k = 0; k < fz; ++k)
        for (int j = 0; j < fy; ++j)
            for (int i = 0; i < fx; ++i) {
                int K = k / 2, Ko = (k % 2) ? K + 1 : K - 1;
                cx near = t2[(long)i + (long)fx * ((long)j + (long)fy * K)];
                cx far = (Ko >= 0 && Ko < czn) ? t2[(long)i + (long)fx * ((long)j + (long)fy * Ko)] : zero;
                ef[(long)i + (long)fx * ((long)j + (long)fy * k)] = cx_add(cx_rscale(0.75, near), cx_rscale(0.25, far));
            }
    free(t2);
}

/* Coarsest solve e = Minv f, each row summed pairwise over its Nc terms. */
static void coarse_solve(const og_grid *g, const cx *f, cx *e)
{
    long n = g->Nc;
#pragma omp parallel for schedule(static) if (n * n > OG_PAR_MIN)
    for (long i = 0; i < n; ++i) {
        double *re = (double *)malloc(sizeof(double) * (size_t)n);
        double *im = (double *)malloc(sizeof(double) * (size_t)n);
        for (long j = 0; j < n; ++j) {
            cx t = cx_mul(g->Minv[i * n + j], f[j]);
            re[j] = t.re; im[j] = t.im;
        }
        e[i] = cx_make(pairwise_padded(re, n), pairwise_padded(im, n));
        free(re); free(im);
    }
}

/* One V(nu1,nu2) cycle on level lev from a zero initial guess: u = V(f). */
static void vcycle_level(const og_grid *g, int lev, const cx *f, cx *u)
{
    if (lev == g->nlev - 1) { coarse_solve(g, f, u); return; }
    long N = g->lev[lev].N, Nc = g->lev[lev + 1].N;
    cx *tmp = (cx *)malloc(sizeof(cx) * (size_t)N);
    cx *fc = (cx *)malloc(sizeof(cx) * (size_t)Nc);
    cx *ec = (cx *)malloc(sizeof(cx) * (size_t)Nc);
    memset(u, 0, sizeof(cx) * (size_t)N);
    for (int s = 0; s < g->nu1; ++s) jacobi(g, lev, f, u, tmp);
    apply_level(g, 1, lev, u, tmp);
    for (long p = 0; p < N; ++p) tmp[p] = cx_sub(f[p], tmp[p]);
    restrict_level(g, lev, tmp, fc);
    vcycle_level(g, lev + 1, fc, ec);
    prolong_level(g, lev, ec, tmp);
    for (long p = 0; p < N; ++p) u[p] = cx_add(u[p], tmp[p]);
    for (int s = 0; s < g->nu2; ++s) {
        if (g->smoother == 1) ilu_sweep(g, lev, f, u, tmp);
        else jacobi(g, lev, f, u, tmp);
    }
    free(tmp); free(fc); free(ec);
}

void og_vcycle(const og_grid *g, const double *f, double *u) { vcycle_level(g, 0, (const cx *)f, (cx *)u); }

void og_restrict(const og_grid *g, int lev, const double *r, double *rc) { restrict_level(g, lev, (const cx *)r, (cx *)rc); }

void og_prolong(const og_grid *g, int lev, const double *ec, double *ef) { prolong_level(g, lev, (const cx *)ec, (cx *)ef); }

void og_jacobi(const og_grid *g, int lev, const double *f, double *u)
{
    cx *tmp = (cx *)malloc(sizeof(cx) * (size_t)g->lev[lev].N);
    jacobi(g, lev, (const cx *)f, (cx *)u, tmp);
    free(tmp);
}

void og_coarse_solve(const og_grid *g, const double *f, double *e) { coarse_solve(g, (const cx *)f, (cx *)e); }

int og_ilu_sweep(const og_grid *g, int lev, const double *f, double *u)
{
    if (lev < 0 || lev >= g->nlev || !g->lev[lev].ilu) return OG_ERR_ARG;
    cx *tmp = (cx *)malloc(sizeof(cx) * (size_t)g->lev[lev].N);
    ilu_sweep(g, lev, (const cx *)f, (cx *)u, tmp);
    free(tmp);
    return OG_OK;
}

void og_dotc(const double *x, const double *y, long n, double *out)
{
    cx d = dotc((const cx *)x, (const cx *)y, n);
    out[0] = d.re; out[1] = d.im;
}

double og_nrm2(const double *x, long n) { return nrm2((const cx *)x, n); }

/* ------------------------------------------------------------------------ */
/* Krylov solvers                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int method;             /* 0 Bi-CGSTAB, 1 IDR(s)                       */
    int s;                  /* IDR shadow dimension                        */
    double tol;             /* on ||b - H x|| / ||b||                      */
    int max_matvec;
    int max_restarts;
    int x0_given;
    const double *P;        /* IDR: N x s complex, column-major            */
    double *history;        /* optional: ||r||/||b|| after every matvec    */
    int history_len;
} og_opts;

typedef struct {
    int status, matvecs, iterations, restarts;
    double rel_res_recurrence, rel_res_true;
} og_info;

static void record(const og_opts *o, og_info *info, double rel)
{
    if (o->history && info->matvecs - 1 < o->history_len && info->matvecs >= 1)
        o->history[info->matvecs - 1] = rel;
}

/* r = b - H x, returns ||r|| */
static double residual(const og_grid *g, const cx *b, const cx *x, cx *r, long N)
{
    apply_level(g, 0, 0, x, r);
    for (long p = 0; p < N; ++p) r[p] = cx_sub(b[p], r[p]);
    return nrm2(r, N);
}

/* Right-preconditioned Bi-CGSTAB, preconditioner = one V-cycle on M. */
static int bicgstab(const og_grid *g, const og_opts *o, const cx *b, cx *x, og_info *info)
{
    long N = g->lev[0].N;
    size_t vb = sizeof(cx) * (size_t)N;
    cx *r = (cx *)malloc(vb), *rh = (cx *)malloc(vb), *p = (cx *)malloc(vb), *v = (cx *)malloc(vb);
    cx *ph = (cx *)malloc(vb), *sh = (cx *)malloc(vb), *t = (cx *)malloc(vb);
    double bn = nrm2(b, N);
    int status = OG_ERR_NOCONV;
    if (!o->x0_given) memset(x, 0, vb);
    if (!isfinite(bn)) { status = OG_ERR_NONFINITE; goto done; }
    if (bn == 0.0) { memset(x, 0, vb); info->rel_res_recurrence = 0.0; info->rel_res_true = 0.0; status = OG_OK; goto done; }
    for (;;) {
        residual(g, b, x, r, N);
        memcpy(rh, r, vb);
        memset(p, 0, vb); memset(v, 0, vb);
        cx rho = cx_make(1.0, 0.0), alpha = cx_make(1.0, 0.0), omega = cx_make(1.0, 0.0);
        int stop = 0; /* 1 converged, 2 breakdown, 3 matvec limit, 4 nonfinite */
        while (!stop) {
            cx rho1 = dotc(rh, r, N);
            if (!cx_finite(rho1)) { stop = 4; break; }
            if (rho1.re == 0.0 && rho1.im == 0.0) { stop = 2; break; }
            cx beta = cx_mul(cx_div(rho1, rho), cx_div(alpha, omega));
            rho = rho1;
            for (long q = 0; q < N; ++q) p[q] = cx_add(r[q], cx_mul(beta, cx_sub(p[q], cx_mul(omega, v[q]))));
            vcycle_level(g, 0, p, ph);
            apply_level(g, 0, 0, ph, v);
            info->matvecs++;
            cx rv = dotc(rh, v, N);
            if (!cx_finite(rv)) { stop = 4; break; }
            if (rv.re == 0.0 && rv.im == 0.0) { stop = 2; break; }
            alpha = cx_div(rho, rv);
            for (long q = 0; q < N; ++q) r[q] = cx_sub(r[q], cx_mul(alpha, v[q]));   /* r holds s */
            double rel = nrm2(r, N) / bn;
            record(o, info, rel);
            info->rel_res_recurrence = rel;
            if (!isfinite(rel)) { stop = 4; break; }
            if (rel < o->tol) {
                for (long q = 0; q < N; ++q) x[q] = cx_add(x[q], cx_mul(alpha, ph[q]));
                info->iterations++;
                stop = 1; break;
            }
            if (info->matvecs >= o->max_matvec) {
                for (long q = 0; q < N; ++q) x[q] = cx_add(x[q], cx_mul(alpha, ph[q]));
                info->iterations++;
                stop = 3; break;
            }
            vcycle_level(g, 0, r, sh);
            apply_level(g, 0, 0, sh, t);
            info->matvecs++;
            cx ts = dotc(t, r, N);
            double tt = blocked_sum(2, t, t, N);
            if (!cx_finite(ts) || !isfinite(tt)) { stop = 4; break; }
            if (tt == 0.0) { stop = 2; break; }
            omega = cx_make(ts.re / tt, ts.im / tt);
            for (long q = 0; q < N; ++q) {
                x[q] = cx_add(cx_add(x[q], cx_mul(alpha, ph[q])), cx_mul(omega, sh[q]));
                r[q] = cx_sub(r[q], cx_mul(omega, t[q]));
            }
            info->iterations++;
            rel = nrm2(r, N) / bn;
            record(o, info, rel);
            info->rel_res_recurrence = rel;
            if (!isfinite(rel)) { stop = 4; break; }
            if (rel < o->tol) { stop = 1; break; }
            if (omega.re == 0.0 && omega.im == 0.0) { stop = 2; break; }
            if (info->matvecs >= o->max_matvec) { stop = 3; break; }
        }
        if (stop == 4) { status = OG_ERR_NONFINITE; break; }
        if (stop == 3) { status = OG_ERR_NOCONV; break; }
        double tr = residual(g, b, x, t, N) / bn;
        info->rel_res_true = tr;
        if (stop == 1 && tr < o->tol) { status = OG_OK; break; }
        if (info->restarts >= o->max_restarts) { status = stop == 2 ? OG_ERR_BREAKDOWN : OG_ERR_NOCONV; break; }
        info->restarts++;
    }
done:
    if (status != OG_ERR_NONFINITE && bn > 0.0 && isfinite(bn))
        info->rel_res_true = residual(g, b, x, t, N) / bn;
    free(r); free(rh); free(p); free(v); free(ph); free(sh); free(t);
    return status;
}

/* Small dense solve G c = m (s x s) with the contract LU. */
static int small_solve(const cx *G, int s, const cx *m, cx *c)
{
    cx *A = (cx *)malloc(sizeof(cx) * (size_t)(s * s));
    int *perm = (int *)malloc(sizeof(int) * (size_t)s);
    memcpy(A, G, sizeof(cx) * (size_t)(s * s));
    int rc = lu_factor(A, s, perm);
    if (rc == 0) lu_solve(A, s, perm, m, c);
    free(A); free(perm);
    return rc;
}

/* IDR(s), right preconditioned, x-space form of the prototype algorithm of
 * Sonneveld & van Gijzen: s minimal-residual start-up steps, then cycles of
 * s+1 steps building the G spaces; G = P^H dR (s x s, row major), m = P^H r.
 * Every step is one V-cycle plus one H apply (one matvec). */
static int idrs(const og_grid *g, const og_opts *o, const cx *b, cx *x, og_info *info)
{
    long N = g->lev[0].N;
    int s = o->s;
    size_t vb = sizeof(cx) * (size_t)N;
    const cx *P = (const cx *)o->P;
    cx *r = (cx *)malloc(vb), *v = (cx *)malloc(vb), *w = (cx *)malloc(vb), *t = (cx *)malloc(vb), *q = (cx *)malloc(vb);
    cx *dR = (cx *)malloc(vb * (size_t)s), *dX = (cx *)malloc(vb * (size_t)s);
    cx *G = (cx *)malloc(sizeof(cx) * (size_t)(s * s));
    cx *m = (cx *)malloc(sizeof(cx) * (size_t)s), *c = (cx *)malloc(sizeof(cx) * (size_t)s);
    double bn = nrm2(b, N);
    int status = OG_ERR_NOCONV;
    if (!o->x0_given) memset(x, 0, vb);
    if (s < 1 || !P) { status = OG_ERR_ARG; goto done; }
    if (!isfinite(bn)) { status = OG_ERR_NONFINITE; goto done; }
    if (bn == 0.0) { memset(x, 0, vb); info->rel_res_recurrence = 0.0; info->rel_res_true = 0.0; status = OG_OK; goto done; }
    for (;;) {
        residual(g, b, x, r, N);
        int stop = 0;
        double rel;
        cx om = cx_make(1.0, 0.0);
        /* start-up: s minimal-residual steps */
        for (int k = 0; k < s && !stop; ++k) {
            vcycle_level(g, 0, r, w);
            apply_level(g, 0, 0, w, t);
            info->matvecs++;
            cx tr = dotc(t, r, N);
            double tt = blocked_sum(2, t, t, N);
            if (!cx_finite(tr) || !isfinite(tt)) { stop = 4; break; }
            if (tt == 0.0) { stop = 2; break; }
            om = cx_make(tr.re / tt, tr.im / tt);
            cx *dXk = dX + (size_t)k * N, *dRk = dR + (size_t)k * N;
            for (long e = 0; e < N; ++e) {
                dXk[e] = cx_mul(om, w[e]);
                cx ot = cx_mul(om, t[e]);
                dRk[e] = cx_make(-ot.re, -ot.im);
                x[e] = cx_add(x[e], dXk[e]);
                r[e] = cx_add(r[e], dRk[e]);
            }
            rel = nrm2(r, N) / bn;
            record(o, info, rel);
            info->rel_res_recurrence = rel;
            if (!isfinite(rel)) { stop = 4; break; }
            if (rel < o->tol) { stop = 1; break; }
            if (info->matvecs >= o->max_matvec) { stop = 3; break; }
            for (int i = 0; i < s; ++i) G[i * s + k] = dotc(P + (size_t)i * N, dRk, N);
        }
        int oldest = 0;
        if (!stop)
            for (int i = 0; i < s; ++i) m[i] = dotc(P + (size_t)i * N, r, N);
        while (!stop) {
            for (int k = 0; k <= s && !stop; ++k) {
                if (small_solve(G, s, m, c) != 0) { stop = 2; break; }
                cx *dXo = dX + (size_t)oldest * N, *dRo = dR + (size_t)oldest * N;
                /* q = -dR c ; v = r + q */
                for (long e = 0; e < N; ++e) {
                    cx acc = cx_mul(dR[e], c[0]);
                    for (int j = 1; j < s; ++j) acc = cx_add(acc, cx_mul(dR[(size_t)j * N + e], c[j]));
                    q[e] = cx_make(-acc.re, -acc.im);
                    v[e] = cx_add(r[e], q[e]);
                }
                vcycle_level(g, 0, v, w);
                if (k == 0) {
                    apply_level(g, 0, 0, w, t);
                    info->matvecs++;
                    cx tv = dotc(t, v, N);
                    double tt = blocked_sum(2, t, t, N);
                    if (!cx_finite(tv) || !isfinite(tt)) { stop = 4; break; }
                    if (tt == 0.0) { stop = 2; break; }
                    om = cx_make(tv.re / tt, tv.im / tt);
                    for (long e = 0; e < N; ++e) {
                        cx acc = cx_mul(dX[e], c[0]);
                        for (int j = 1; j < s; ++j) acc = cx_add(acc, cx_mul(dX[(size_t)j * N + e], c[j]));
                        dRo[e] = cx_sub(q[e], cx_mul(om, t[e]));
                        dXo[e] = cx_sub(cx_mul(om, w[e]), acc);
                    }
                } else {
                    for (long e = 0; e < N; ++e) {
                        cx acc = cx_mul(dX[e], c[0]);
                        for (int j = 1; j < s; ++j) acc = cx_add(acc, cx_mul(dX[(size_t)j * N + e], c[j]));
                        dXo[e] = cx_sub(cx_mul(om, w[e]), acc);
                    }
                    apply_level(g, 0, 0, dXo, t);
                    info->matvecs++;
                    for (long e = 0; e < N; ++e) dRo[e] = cx_make(-t[e].re, -t[e].im);
                }
                for (long e = 0; e < N; ++e) {
                    r[e] = cx_add(r[e], dRo[e]);
                    x[e] = cx_add(x[e], dXo[e]);
                }
                info->iterations++;
                rel = nrm2(r, N) / bn;
                record(o, info, rel);
                info->rel_res_recurrence = rel;
                if (!isfinite(rel)) { stop = 4; break; }
                if (rel < o->tol) { stop = 1; break; }
                if (info->matvecs >= o->max_matvec) { stop = 3; break; }
                for (int i = 0; i < s; ++i) {
                    cx dm = dotc(P + (size_t)i * N, dRo, N);
                    G[i * s + oldest] = dm;
                    m[i] = cx_add(m[i], dm);
                }
                oldest = oldest + 1 == s ? 0 : oldest + 1;
            }
        }
        if (stop == 4) { status = OG_ERR_NONFINITE; break; }
        if (stop == 3) { status = OG_ERR_NOCONV; break; }
        double trel = residual(g, b, x, t, N) / bn;
        info->rel_res_true = trel;
        if (stop == 1 && trel < o->tol) { status = OG_OK; break; }
        if (info->restarts >= o->max_restarts) { status = stop == 2 ? OG_ERR_BREAKDOWN : OG_ERR_NOCONV; break; }
        info->restarts++;
    }
done:
    if (status != OG_ERR_NONFINITE && status != OG_ERR_ARG && bn > 0.0 && isfinite(bn))
        info->rel_res_true = residual(g, b, x, t, N) / bn;
    free(r); free(v); free(w); free(t); free(q); free(dR); free(dX); free(G); free(m); free(c);
    return status;
}

int og_solve(const og_grid *g, const og_opts *o, const double *b, double *x, og_info *info)
{
    memset(info, 0, sizeof(*info));
    int st = o->method == 0 ? bicgstab(g, o, (const cx *)b, (cx *)x, info)
                            : idrs(g, o, (const cx *)b, (cx *)x, info);
    info->status = st;
    return st;
}

int og_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
