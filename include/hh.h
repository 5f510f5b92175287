/*
 * hh.h -- C ABI of the MI355X (gfx950) Helmholtz solver with a complex
 * stretched grid (CSG) multigrid preconditioner.
 *
 * The operation follows Reps, Vanroose & bin Zubair, "On the indefinite
 * Helmholtz equation: complex stretched absorbing boundary layers, iterative
 * analysis, and preconditioning":
 *   - the problem  -(Lap + phi(x)) u = chi  (Sec. 4, eq. (Helgen)), phi = k(x)^2,
 *     on a tensor grid whose interior [a,b] per axis is extended by exterior
 *     complex scaled (ECS) layers out to [lo,hi] (Sec. 2, eq. (ecstrans), the
 *     linear map z = r + (x - r) e^{i theta} on the layer), homogeneous
 *     Dirichlet at the contour ends (eq. (lapctuecs));
 *   - Shortley-Weller differences on the complex widths (Sec. 3, eq.
 *     (shortwell)), cell-centred unknowns (Sec. 6);
 *   - the CSG preconditioner M: the same operator on a grid whose widths are
 *     all multiplied by beta = e^{i theta_csg} (uniform mode, Sec. 5.3 and eq.
 *     (CSL-CSG)) or only the interior widths (interior mode, eq.
 *     (lapctucsg));
 *   - one multigrid V(1,1) cycle per preconditioner application (Sec. 6.2)
 *     with weighted Jacobi, full weighting, bilinear/trilinear prolongation,
 *     rediscretised coarse operators and an exact coarsest solve;
 *   - right-preconditioned Bi-CGSTAB or IDR(s) (Sec. 6.2), stopped on the
 *     relative residual ||b - H x|| / ||b|| < tol.
 *
 * Conventions for every call:
 *   - Every call returns an hh_status; nothing aborts or throws across the ABI.
 *     On a non-OK status hh_last_error() gives a thread-local message.
 *   - Complex vectors are interleaved (re, im) pairs: HH_C128 = 2 x double
 *     (16 bytes), HH_C64 = 2 x float (8 bytes); index i + nx*(j + ny*k), x
 *     fastest (the layout of a contiguous torch/numpy complex array indexed
 *     [k][j][i]).  Device vectors must be 16-byte aligned (8 for C64).
 *   - Device pointers are owned by the caller and never retained past the call;
 *     the library owns only hh_grid objects, the solve work space it attaches
 *     to a grid, and the server arena.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue their
 *     work on it; hh_apply_operator and hh_vcycle return without waiting,
 *     hh_solve and hh_solve_batch synchronise the stream before returning.
 *   - The library never falls back to the CPU: without a usable gfx950 device
 *     every compute call returns HH_ERR_HIP.
 */
#ifndef HH_H
#define HH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HH_OK = 0,
    HH_PENDING = 1,          /* hh_poll: request not finished yet                */
    HH_ERR_ARG = -1,         /* invalid argument or description                  */
    HH_ERR_OOM = -2,         /* device allocation failed / footprint over budget */
    HH_ERR_HIP = -3,         /* HIP runtime error, or no usable device           */
    HH_ERR_NOCONV = -4,      /* matvec limit reached (x holds the last iterate)  */
    HH_ERR_BREAKDOWN = -5,   /* Krylov breakdown persisted through the restarts  */
    HH_ERR_NONFINITE = -6,   /* NaN/Inf in the data or the iteration             */
    HH_ERR_BUSY = -7,        /* server queue full                                */
    HH_ERR_TICKET = -8       /* unknown ticket                                   */
} hh_status;

typedef enum { HH_C128 = 0, HH_C64 = 1 } hh_prec;
typedef enum { HH_OP_H = 0, HH_OP_M = 1 } hh_op;
/* The preconditioner M: the complex stretched grid with every width times
 * beta = e^{i theta_csg} (uniform, Sec. 5.3, eq. (CSL-CSG)), with only the
 * interior widths stretched (interior, eq. (lapctucsg)), or the complex
 * shifted Laplacian -(Lap + beta^2 phi) of Sec. 5.2, eq. (helmctucsl), with
 * beta^2 = csl_shift.  The library applies the CSL through eq. (CSL-CSG):
 * M = M_CSL / beta^2, the uniform stretched grid with beta the principal
 * square root of the shift (any modulus); the constant factor does not change
 * the Krylov iterates, and hh_apply_operator(HH_OP_M) returns M_CSL x / beta^2. */
typedef enum { HH_CSG_UNIFORM = 0, HH_CSG_INTERIOR = 1, HH_CSL = 2 } hh_csg_mode;
/* Boundary condition of one side of one axis: homogeneous Dirichlet (at the
 * contour end of a layer, or at the edge), or the first-order Sommerfeld
 * condition du/dn = -i k_bc u (Sec. 2, eq. (sommerfeld1); Sec. 4, eq. (BC)),
 * discretised by a ghost node one cell beyond the last unknown and the
 * centred difference of the condition at the boundary face.  A Sommerfeld
 * side has no layer (a == lo, resp. b == hi) and needs a cell-centred grid;
 * the preconditioner takes the condition in its own stretched coordinate. */
typedef enum { HH_BC_DIRICHLET = 0, HH_BC_SOMMERFELD = 1 } hh_bc;
typedef enum { HH_METHOD_BICGSTAB = 0, HH_METHOD_IDR = 1 } hh_method;
/* Unknowns at cell centres (Sec. 6: the experiments' topology; the Dirichlet
 * ends lo/hi are half a cell beyond the first/last unknown) or at the
 * vertices of a uniform grid (Sec. 3, eq. (ecsgrid): n unknowns between the
 * end nodes lo and hi, width (hi - lo)/(n + 1)). */
typedef enum { HH_CELL = 0, HH_VERTEX = 1 } hh_centering;
/* Coarse-level operators of the V-cycle: rediscretised on the halved grid, or
 * Galerkin M_{l+1} = R M_l P with the cycle's own transfers (Sec. 6.1; 2D,
 * cell-centred; a 25-point stencil per coarse point, since the cell-centred
 * transfers reach two coarse cells). */
typedef enum { HH_COARSE_REDISCRETISED = 0, HH_COARSE_GALERKIN = 1 } hh_coarse_op;
/* Smoother of the V-cycle: weighted Jacobi (omega its weight), or ILU(0), the
 * paper's choice (Sec. 6.1): one sweep u = u + omega (L U)^-1 (f - M u) per
 * level with the incomplete LU factors of the level operator on its nonzero
 * pattern, lexicographic order (omega its relaxation, 1 for the plain
 * sweep).  HH_SMOOTH_ILU0 needs a 2D cell-centred grid, the V(0,1) cycle
 * (nu1 = 0), at least 5 cells per side on every level but the coarsest, and
 * the FP64 V-cycle (HH_C128); it runs single solves and V-cycle calls
 * (batches of more than one problem, hh_submit and hh_profile_vcycle reject
 * it).  Its triangular solves are sequential along anti-diagonals, so a
 * cycle costs about (n_x + n_y) dependent steps per level (rediscretised)
 * or (n_x + 3 n_y) (Galerkin), plus n_x for each further band of rows
 * where a level has more than 1024 (5-point) or 512 (Galerkin) rows.  The
 * device copy of the factors is stored in the solves' step order, padded
 * to whole waves (up to about 2.5 times the 25 N_level entries). */
typedef enum { HH_SMOOTH_JACOBI = 0, HH_SMOOTH_ILU0 = 1 } hh_smoother;

/* Grid description (host memory, read during hh_setup_grid only). */
typedef struct {
    int32_t dim;            /* 2 or 3                                                    */
    int32_t n[3];           /* cells per axis on the finest grid, layers included        */
    double lo[3], hi[3];    /* real coordinates of the outer Dirichlet ends              */
    double a[3], b[3];      /* interior [a,b] per axis (ECS turning points), lo<=a<b<=hi;
                               a == lo (b == hi) means no layer on that side             */
    double theta_ecs;       /* ECS angle theta_gamma of H, in (0, pi/2)                  */
    double theta_csg;       /* CSG angle theta_beta of M, |theta| < pi/2 (negative for
                               Sommerfeld problems, as in the paper's tables); unused
                               for HH_CSL                                                */
    int32_t csg_mode;       /* hh_csg_mode                                               */
    int32_t centering;      /* hh_centering.  HH_VERTEX grids have one level and
                               support hh_apply_operator only (the closed-form
                               eigenpairs of Sec. 3 are on this grid); every
                               multigrid or solve call rejects them with HH_ERR_ARG */
    int32_t levels;         /* multigrid levels; 0 = halve while every side is even and
                               the largest side exceeds 16 (2D) / 8 (3D); HH_VERTEX: 0 or 1 */
    int32_t nu1, nu2;       /* smoothing steps: (1,1), or (0,1), the paper's V(0,1) cycle
                               (Sec. 6.1: no pre-smoothing, one post-smoothing step)     */
    double omega;           /* Jacobi weight, e.g. 0.8                                   */
    const double *phi;      /* host, prod(n) reals: k(x)^2 at the cell centres; NULL ->
                               phi_const everywhere                                      */
    double phi_const;
    int32_t host_only;      /* 1: build the host-side setup only (no device memory);
                               only hh_grid_query / hh_grid_export / hh_free_grid may
                               then be called                                            */
    /* A zero-filled tail keeps the linear contour, Dirichlet sides and no shift. */
    double csl_shift[2];    /* HH_CSL: the complex shift beta^2 = (re, im), nonzero; the
                               paper's tables print -beta^2 (shift -1 - 0.2i is beta^2 =
                               1 + 0.2i)                                                 */
    int32_t contour_steps;  /* 0 or 1: linear ECS contour (eq. (lapctuecs)); m > 1: the
                               contour of each layer turns to theta_ecs in m equal angle
                               steps over m equal parts of the layer (Sec. 6.2, remark on
                               a smooth ECS transition)                                  */
    int32_t bc[3][2];       /* hh_bc per axis, (low side, high side)                     */
    double k_bc;            /* k of the Sommerfeld condition, > 0 when a side uses it    */
    int32_t coarse_op;      /* hh_coarse_op.  HH_COARSE_GALERKIN: 2D cell-centred grids;
                               single solves and every V-cycle call (batched solves with
                               more than one problem, and hh_submit, reject it)          */
    int32_t smoother;       /* hh_smoother (zero: weighted Jacobi)                       */
} hh_grid_desc;

typedef struct hh_grid hh_grid;   /* opaque */

/* Builds node maps, Shortley-Weller coefficients of H and M on every level
 * (Sec. 3, eq. (shortwell); M by Sec. 5.3, eq. (CSL-CSG) / (lapctucsg)),
 * the coarse phi hierarchy (mean of children) and the explicit inverse of
 * the coarsest M (dense LU with partial pivoting), and uploads them.
 * A vertex-centred grid gets the level-0 coefficients and phi only.
 * Errors: HH_ERR_ARG (dim not 2/3; unknown centering; fewer than 2 levels
 * on a cell-centred grid, given or from the automatic rule, more than 1 on a
 * vertex-centred one; side not divisible by 2^(levels-1); coarsest grid above
 * 1024 unknowns; theta outside (0, pi/2); a, b outside
 * [lo, hi]; (nu1, nu2) not (1, 1) or (0, 1); singular coarse matrix), HH_ERR_OOM,
 * HH_ERR_HIP.  *out is set only on HH_OK. */
hh_status hh_setup_grid(const hh_grid_desc *d, hh_grid **out);
hh_status hh_free_grid(hh_grid *g);

typedef struct {
    int32_t dim, levels;
    int32_t n[16][3];        /* per level                                  */
    int64_t unknowns;        /* finest N                                   */
    int32_t coarse_unknowns;
    uint64_t device_bytes;   /* device memory the grid holds right now     */
} hh_grid_info;
hh_status hh_grid_query(const hh_grid *g, hh_grid_info *info);

/* Copies a host-side setup array of the grid (for inspection and tests):
 * what = 0 aH, 1 cH, 2 dH (ECS coefficients, level 0 only), 3 aM, 4 cM, 5 dM
 * (CSG coefficients), complex double per unknown of `axis` on `level`;
 * 6 phi of `level` (N_level doubles); 7 the coarsest inverse (Nc*Nc complex
 * double, row major); 8 the Galerkin stencil of `level` >= 1 (25 * N_level
 * complex double, entry s = (dx+2) + 5(dy+2) of point p at s*N + p, the
 * matrix entry M[p, p + dx + nx*dy]); 9 the ILU(0) factors of a smoothing
 * `level` of an HH_SMOOTH_ILU0 grid (25 * N_level complex double in the same
 * layout: entries below the diagonal hold L, whose unit diagonal is not
 * stored, the diagonal and above hold U, zero off the pattern).  `bytes` must
 * equal the array size. */
hh_status hh_grid_export(const hh_grid *g, int32_t what, int32_t level, int32_t axis, void *host_dst,
                         size_t bytes);

/* y = A x on the finest grid; A = H (the ECS operator of Sec. 3, eq.
 * (shortwell); prec must be HH_C128) or M (the CSG operator of Sec. 5.3;
 * HH_C128 uses FP64 coefficients, HH_C64 the FP32 copies).  x, y: device, N
 * elements of `prec`, must not be the same buffer; the caller owns both.
 * Errors: HH_ERR_ARG (null pointer, host-only grid, x == y, H with HH_C64,
 * unknown op or prec), HH_ERR_HIP (launch failure or no device). */
hh_status hh_apply_operator(const hh_grid *g, hh_op op, hh_prec prec, const void *x, void *y, void *stream);

/* u = V(f): one V(1,1) cycle on M from a zero initial guess (Sec. 6.2: the
 * preconditioner application; weighted Jacobi, full weighting, linear
 * interpolation, exact coarsest solve).
 * prec = HH_C128: f and u are complex double, all levels in FP64.
 * prec = HH_C64 : f is complex double, u is complex float, every level
 *                 computes in FP32 (the mixed-precision preconditioner).
 * f, u: device, N elements, caller-owned, not the same buffer.  The first call
 * per precision builds the grid's launch plan (device memory the grid keeps).
 * Errors: HH_ERR_ARG (null pointer, host-only grid, f == u, unknown prec),
 * HH_ERR_OOM (plan allocation), HH_ERR_HIP. */
hh_status hh_vcycle(const hh_grid *g, hh_prec prec, const void *f, void *u, void *stream);

/* Timing of the preconditioner application (Sec. 6.2: one V-cycle per
 * matvec) and of the two kernels that carry most of its traffic, the fused
 * down-leg and up-leg of the finest level, launched exactly as hh_vcycle and
 * the solves launch them.  Times are averages, from HIP events on `stream`,
 * over `reps` back-to-back cycles and then `reps` back-to-back launches of
 * each leg.  f, u as for hh_vcycle; u is overwritten.  Builds the V-cycle
 * plan like hh_vcycle; creates and destroys six events; synchronises the
 * stream.  Errors: as hh_vcycle, and HH_ERR_ARG for reps < 1 or a null out. */
typedef struct {
    double vcycle_us;               /* one whole V(1,1) cycle                          */
    double down_us, up_us;          /* one launch of the finest down-leg / up-leg      */
    int32_t down_shape, up_shape;   /* tile shapes of those launches (index into the
                                       library's set)                                  */
    int32_t down_groups, up_groups; /* workgroups per launch                           */
} hh_vcycle_profile;
hh_status hh_profile_vcycle(const hh_grid *g, hh_prec prec, const void *f, void *u, int32_t reps,
                            hh_vcycle_profile *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * V-cycle as hh_vcycle, same kernels and results, but the restricted
 * right-hand sides and level solutions of levels >= 1 live in a static
 * device array of the library (32 MiB per device, held until the process
 * ends) instead of memory the grid allocates on first use.  The call
 * allocates nothing, creates no stream or event and times nothing (tile
 * shapes come from earlier hh_vcycle/hh_solve plans of the same level class,
 * else a default; shapes never change results).  Every call on one device
 * shares that array: calls that overlap in time on one device (other
 * streams, other threads) race and give wrong results; calls ordered on one
 * stream are safe.  Nothing in the array needs to start at zero (every value
 * is written before it is read within one cycle).  f: device complex double,
 * u: device, complex double (HH_C128) or complex float (HH_C64), N elements,
 * caller-owned, not the same buffer; the grid must have been set up on the
 * current device.  Errors: HH_ERR_ARG (as hh_vcycle; the coarse levels need
 * more than 32 MiB in this precision -- e.g. 2D 2048^2 in complex double;
 * current device is not the grid's), HH_ERR_HIP (launch failure, or the
 * array's address was not found at grid setup). */
hh_status hh_vcycle_noalloc(const hh_grid *g, hh_prec prec, const void *f, void *u, void *stream);

typedef struct {
    int32_t method;          /* hh_method                                              */
    int32_t s;               /* IDR shadow dimension (1..8)                            */
    double tol;              /* stop when ||b - H x|| / ||b|| < tol                     */
    int32_t max_matvec;      /* one matvec = one V-cycle + one H apply                  */
    int32_t max_restarts;    /* restarts from the true residual after a false stop or
                                a breakdown (e.g. 3)                                    */
    int32_t vcycle_prec;     /* HH_C128 plain FP64, HH_C64 mixed (FP32 V-cycle)         */
    int32_t x0_given;        /* 0: start from x = 0; 1: x holds the initial guess       */
    const void *idr_P;       /* device, N x s complex double, column-major, orthonormal
                                columns; required for IDR                               */
    double *history;         /* optional host buffer: ||r||/||b|| after every matvec    */
    int32_t history_len;
} hh_solve_opts;

typedef struct {
    int32_t status;          /* hh_status of this problem                              */
    int32_t matvecs, iterations, restarts;
    double rel_res_recurrence;  /* last recurrence residual / ||b||                    */
    double rel_res_true;        /* ||b - H x|| / ||b|| in FP64 at exit                 */
    double seconds;             /* wall time inside the call                           */
    int32_t fp64_fallback;      /* 1: a mixed-precision solve drifted (its residual
                                   stalled or rose far above its best) and was
                                   finished from its current iterate with the FP64
                                   V-cycle; matvecs and iterations count both parts */
    int32_t stages;             /* mixed precision: stages run (each restarts from
                                   the FP64 true residual after a fixed reduction;
                                   not counted in `restarts`); 0 in FP64           */
} hh_solve_info;

/* Solves H x = b by right-preconditioned Bi-CGSTAB or IDR(s) with M^{-1}
 * replaced by one V-cycle (Sec. 6.2).  b, x: device complex double, N
 * elements, caller-owned.  Fills *info.  Errors: HH_ERR_ARG (invalid options,
 * host-only grid), HH_ERR_OOM (work space), HH_ERR_HIP, and the solve's own
 * outcome: HH_ERR_NOCONV, HH_ERR_BREAKDOWN, HH_ERR_NONFINITE.
 * HH_ERR_NOCONV / HH_ERR_BREAKDOWN still leave the last iterate in x and a
 * complete info.  A zero b gives x = 0 with 0 matvecs.  The grid keeps its
 * solve work space allocated until hh_free_grid. */
hh_status hh_solve(hh_grid *g, const hh_solve_opts *o, const void *b, void *x, hh_solve_info *info, void *stream);

/* Solves `count` independent problems together: every pass of the method is
 * one launch over the tiles of all problems still running.  All problems must
 * use the same method and vcycle_prec; grids must be distinct.  o, b, x and
 * info are arrays of `count`.  The return value is HH_OK when every problem
 * converged, otherwise the first non-OK per-problem status. */
hh_status hh_solve_batch(hh_grid *const *g, int32_t count, const hh_solve_opts *o, const void *const *b,
                         void *const *x, hh_solve_info *info, void *stream);

/* ---- choosing the preconditioner's stretch or shift --------------------- */
/* Sec. 6.2, remark on choosing the CSL and CSG parameters: starting from a
 * given CSG angle (or CSL imaginary shift), multigrid alone is run on the
 * preconditioner problem M u = f, u_k = u_{k-1} + V(f - M u_{k-1}), u_0 = 0,
 * with the FP64 V-cycle of hh_vcycle, and the parameter is multiplied by
 * `factor` while multigrid still reduces ||f - M u_k|| / ||f|| below
 * `reduction` within `max_cycles` cycles (the paper: "just converges, say in
 * 10-20 cycles"; its tables count cycles to 7 orders).  The result is the
 * last value that converged: the CSG angle theta_csg, or for the CSL the
 * imaginary part eps of the shift beta^2 = 1 + i eps (the paper's tables
 * print -beta^2 = -1 - i eps; a negative start searches negative values).
 * d describes the problem (its own theta_csg / csl_shift / csg_mode are
 * replaced: CSG_ANGLE keeps csg_mode unless it is HH_CSL, which becomes
 * uniform; CSL_SHIFT sets HH_CSL).  f: device, N complex double, nonzero.
 * trace: optional host array of 3 * max_steps doubles, (value, cycles to
 * converge or 0, last relative residual) per candidate.  Norms follow the
 * fixed reduction order of the solves, so the choice is reproducible.
 * Builds and frees one grid per candidate; allocates three work vectors.
 * Errors: HH_ERR_ARG (description or options), HH_ERR_NOCONV (no
 * convergence at the start value), HH_ERR_OOM, HH_ERR_HIP. */
typedef enum { HH_SELECT_CSG_ANGLE = 0, HH_SELECT_CSL_SHIFT = 1 } hh_select_which;
typedef struct {
    int32_t which;          /* hh_select_which                                       */
    double start;           /* first candidate (angle in radians, or eps)            */
    double factor;          /* each next candidate is the previous one times this,
                               0 < factor < 1                                         */
    double min_value;       /* stop before |candidate| falls below this               */
    int32_t max_cycles;     /* e.g. 20                                                */
    double reduction;       /* e.g. 1e-7                                              */
    int32_t max_steps;      /* candidates at most                                     */
} hh_select_opts;
typedef struct {
    double value;           /* chosen angle or eps                                    */
    int32_t cycles;         /* cycles it needed                                       */
    double factor;          /* its average residual reduction per cycle               */
    int32_t tried;          /* candidates run                                         */
    int32_t status;         /* HH_OK or HH_ERR_NOCONV                                 */
} hh_select_result;
hh_status hh_select_preconditioner(const hh_grid_desc *d, const hh_select_opts *o, const void *f,
                                   hh_select_result *res, double *trace, void *stream);

/* ---- serving ---------------------------------------------------------- */
typedef struct {
    uint64_t hbm_budget_bytes;   /* 0: 80% of the free device memory at creation   */
    int32_t max_slots;           /* problems on the device at once                 */
    int32_t device;
} hh_server_opts;

typedef struct {
    hh_grid_desc grid;           /* phi (if non-NULL) is copied at submit            */
    hh_solve_opts opts;          /* history is ignored; IDR needs idr_P_host         */
    const void *b_host;          /* N complex double, copied at submit               */
    void *x_host;                /* N complex double; written before hh_poll returns
                                    HH_OK for this ticket; must stay valid until then */
    const void *idr_P_host;      /* IDR only: N x s complex double, column-major     */
} hh_request;

typedef struct {
    hh_solve_info info;
    double t_submit, t_admit, t_done;   /* seconds on the server's monotonic clock */
} hh_result;

/* Device bytes one request of this description and these options may hold
 * while it is admitted: its hierarchy, solve work space, b, x, the IDR
 * shadow space and its share of the launch lists.  An upper bound; the server
 * admits by it.  HH_ERR_ARG for an invalid description.  Needs no device. */
hh_status hh_request_footprint(const hh_grid_desc *d, const hh_solve_opts *o, uint64_t *bytes);

typedef struct hh_server hh_server;
/* Starts the server's worker and preparation threads on `device`. */
hh_status hh_server_create(const hh_server_opts *o, hh_server **out);
/* Copies the request and queues it.  HH_ERR_OOM if its device footprint
 * exceeds the whole budget, HH_ERR_ARG for an invalid description. */
hh_status hh_submit(hh_server *sv, const hh_request *r, uint64_t *ticket);
/* HH_PENDING until the solve finished; then HH_OK (result filled, x_host
 * written, ticket released) -- the solve's own status is in result.info. */
hh_status hh_poll(hh_server *sv, uint64_t ticket, hh_result *out);
hh_status hh_server_destroy(hh_server *sv);

typedef struct {
    uint64_t submitted, admitted, completed, rejected;
    uint64_t bytes_in_use, bytes_budget, peak_bytes;   /* admission footprints */
    uint64_t actual_in_use, peak_actual;                /* bytes the admitted solves hold */
    int32_t active_slots, queued;
} hh_server_stats;
hh_status hh_server_query(hh_server *sv, hh_server_stats *st);

const char *hh_last_error(void);
const char *hh_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HH_H */
