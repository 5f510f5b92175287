// hh_common.h -- internal types shared by the host setup, the kernels and the
// C-ABI drivers of the gfx950 Helmholtz solver.
//
// Data layout in HBM (one problem):
//   * per level and axis: three complex coefficient arrays of the rediscretised
//     preconditioner M (lower a, upper c, centre d = a + c), FP64 and (for the
//     mixed-precision V-cycle) FP32 copies; level 0 also holds the ECS
//     operator H's arrays (FP64 only).  O(n) per axis, cache resident.
//   * phi_l = k^2 per level (N_l reals), FP64 and FP32.
//   * the explicit inverse of the coarsest M (Nc x Nc, row major), c128/c64.
//   * per level l >= 1: f_l (restricted residual) and e_l (level solution),
//     in the precision of the V-cycle.
//   * solve work space: x, b-copy-free, r, rhat, p, v, t (c128), phat/shat
//     (c128, or c64 in mixed mode), chunk partial sums, a state block.
// Complex values are interleaved (re, im), x fastest.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HH_MAXLEV 16
#define HH_WG 256                 // threads per workgroup (4 wave64)
#define HH_PER_SLOT 1             // elements per thread slot in a reduction chunk (chunk = 256)
#define HH_CHUNK (HH_WG * HH_PER_SLOT)
// Krylov vector passes: a workgroup of HH_GROUP chunks (one unknown per
// thread, chunk s = waves 4s..4s+3) writes one partial per value, the
// group's node of the pairwise tree over chunk partials.  Two chunks per
// workgroup measure fastest (about 1% over one in 2D and 3D; four: 3D 1-3%
// slower).
#define HH_GROUP 2
#define HH_VWG (HH_WG * HH_GROUP)
#define HH_SPAN (HH_CHUNK * HH_GROUP)
#define HH_NPART 40               // reals per chunk partial record (IDR(8) start-up needs 4s+1)
#define HH_MAX_COARSE 1024
#define HH_MAX_S 8
// Coarsest grids above this many unknowns are solved by k_coarse, rows spread
// over many workgroups (one workgroup streaming a 512 x 512 inverse is
// latency bound); smaller ones are solved inside the tail kernel.
#define HH_SPLIT_NC 128

// ---------------------------------------------------------------------------
// complex helpers (fixed operation order: no FMA contraction, the build uses
// -ffp-contract=off)
// ---------------------------------------------------------------------------
template <typename T> struct V2t;
template <> struct V2t<double> { using type = double2; };
template <> struct V2t<float> { using type = float2; };
template <typename T> using V2 = typename V2t<T>::type;

template <typename T> __host__ __device__ inline V2<T> cmk(T re, T im) { V2<T> z; z.x = re; z.y = im; return z; }
template <typename T> __host__ __device__ inline V2<T> cadd(V2<T> a, V2<T> b) { return cmk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __host__ __device__ inline V2<T> csub(V2<T> a, V2<T> b) { return cmk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __host__ __device__ inline V2<T> cmul(V2<T> a, V2<T> b)
{
    return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// FP32 is the V-cycle precision of mixed solves, held to a tolerance against
// FP64 rather than to its operation order: fused multiply-adds
template <> __host__ __device__ inline V2<float> cmul<float>(V2<float> a, V2<float> b)
{
    return cmk<float>(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
template <typename T> __host__ __device__ inline V2<T> cdiv(V2<T> a, V2<T> b)
{
    T d = b.x * b.x + b.y * b.y;
    return cmk<T>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename T> __host__ __device__ inline V2<T> crs(T s, V2<T> a) { return cmk<T>(s * a.x, s * a.y); }

// Multiply-accumulates of the V-cycle kernels: a - b c, a + b c, a + s x and
// s x + t y.  In FP64 they are exactly the separate operations above, in that
// order (the arithmetic contract); FP32 takes fused multiply-adds.
template <typename T> __host__ __device__ inline V2<T> cmsub(V2<T> a, V2<T> b, V2<T> c) { return csub<T>(a, cmul<T>(b, c)); }
template <typename T> __host__ __device__ inline V2<T> cmadd(V2<T> a, V2<T> b, V2<T> c) { return cadd<T>(a, cmul<T>(b, c)); }
template <typename T> __host__ __device__ inline V2<T> crsadd(V2<T> a, T s, V2<T> x) { return cadd<T>(a, crs<T>(s, x)); }
template <typename T> __host__ __device__ inline V2<T> crs2(T s, V2<T> x, T t, V2<T> y) { return cadd<T>(crs<T>(s, x), crs<T>(t, y)); }
template <> __host__ __device__ inline V2<float> cmsub<float>(V2<float> a, V2<float> b, V2<float> c)
{
    return cmk<float>(fmaf(-b.x, c.x, fmaf(b.y, c.y, a.x)), fmaf(-b.x, c.y, fmaf(-b.y, c.x, a.y)));
}
template <> __host__ __device__ inline V2<float> cmadd<float>(V2<float> a, V2<float> b, V2<float> c)
{
    return cmk<float>(fmaf(b.x, c.x, fmaf(-b.y, c.y, a.x)), fmaf(b.x, c.y, fmaf(b.y, c.x, a.y)));
}
template <> __host__ __device__ inline V2<float> crsadd<float>(V2<float> a, float s, V2<float> x)
{
    return cmk<float>(fmaf(s, x.x, a.x), fmaf(s, x.y, a.y));
}
template <> __host__ __device__ inline V2<float> crs2<float>(float s, V2<float> x, float t, V2<float> y)
{
    return cmk<float>(fmaf(s, x.x, t * y.x), fmaf(s, x.y, t * y.y));
}

// Explicit global-address-space accesses: pointers taken from descriptors in
// memory are generic to the compiler, which would otherwise emit flat
// loads/stores; these emit global_load / global_store.
#define HH_GLOBAL __attribute__((address_space(1)))
typedef double hh_dvec2 __attribute__((ext_vector_type(2)));
typedef float hh_fvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double ldg(const double *p, int64_t i) { return ((const HH_GLOBAL double *)p)[i]; }
__device__ __forceinline__ float ldg(const float *p, int64_t i) { return ((const HH_GLOBAL float *)p)[i]; }
__device__ __forceinline__ double2 ldg(const double2 *p, int64_t i)
{
    hh_dvec2 v = ((const HH_GLOBAL hh_dvec2 *)p)[i];
    double2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
__device__ __forceinline__ float2 ldg(const float2 *p, int64_t i)
{
    hh_fvec2 v = ((const HH_GLOBAL hh_fvec2 *)p)[i];
    float2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
typedef unsigned hh_uvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ hh_uvec4 ldg16(const void *p, int64_t i) { return ((const HH_GLOBAL hh_uvec4 *)p)[i]; }
__device__ __forceinline__ void stg(double2 *p, int64_t i, double2 v)
{
    hh_dvec2 w;
    w.x = v.x;
    w.y = v.y;
    ((HH_GLOBAL hh_dvec2 *)p)[i] = w;
}
__device__ __forceinline__ void stg(float2 *p, int64_t i, float2 v)
{
    hh_fvec2 w;
    w.x = v.x;
    w.y = v.y;
    ((HH_GLOBAL hh_fvec2 *)p)[i] = w;
}

// streaming store: output that the next launch does not read past the caches,
// so they keep the inputs (vector store with the non-temporal hint)
__device__ __forceinline__ void stg_nt(double2 *p, int64_t i, double2 v)
{
    hh_dvec2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (HH_GLOBAL hh_dvec2 *)p + i);
}

__device__ __forceinline__ void stg_nt(float2 *p, int64_t i, float2 v)
{
    hh_fvec2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (HH_GLOBAL hh_fvec2 *)p + i);
}
// streaming loads: input that a launch reads once, from HBM when it exceeds
// the caches (vector load with the non-temporal hint, which streams at a
// higher rate than plain loads and leaves the caches to the data that the
// launch's neighbouring tiles share)
__device__ __forceinline__ double2 ldg_nt(const double2 *p, int64_t i)
{
    const hh_dvec2 v = __builtin_nontemporal_load((const HH_GLOBAL hh_dvec2 *)p + i);
    double2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
__device__ __forceinline__ float2 ldg_nt(const float2 *p, int64_t i)
{
    const hh_fvec2 v = __builtin_nontemporal_load((const HH_GLOBAL hh_fvec2 *)p + i);
    float2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
__device__ __forceinline__ float ldg_nt(const float *p, int64_t i) { return __builtin_nontemporal_load((const HH_GLOBAL float *)p + i); }
__device__ __forceinline__ double ldg_nt(const double *p, int64_t i) { return __builtin_nontemporal_load((const HH_GLOBAL double *)p + i); }

// conversions between the two complex precisions
template <typename T, typename S> __device__ inline V2<T> ccvt(S v) { return cmk<T>((T)v.x, (T)v.y); }

// ---------------------------------------------------------------------------
// 32-bit division by a runtime constant (round-up magic number method)
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, l;
};
inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.l = l;
    f.m = d <= 1 ? 0u : (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    return f;
}
__host__ __device__ inline uint32_t fdiv(uint32_t n, FastDiv f)
{
    if (f.d == 1) return n;
#ifdef __HIP_DEVICE_COMPILE__
    uint32_t t = __umulhi(n, f.m);
#else
    uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
    return (t + ((n - t) >> 1)) >> (f.l - 1);
}

// ---------------------------------------------------------------------------
// per-level data of one problem, in one precision
// ---------------------------------------------------------------------------
template <typename T> struct LevelDev {
    int n[3];
    int64_t N;
    FastDiv fx, fxy;                 // linear index -> (i, j, k)
    const V2<T> *a[3], *c[3], *d[3]; // M coefficients per axis
    const T *phi;
    V2<T> *f;                        // restricted right-hand side (levels >= 1)
    V2<T> *e;                        // level solution / correction (levels >= 1)
    const V2<T> *g;                  // Galerkin levels >= 1: the 25 x N stencil, else null
    const V2<T> *ilu;                // ILU(0) smoothing levels (FP64): the 25 x N factors, else null
    V2<T> *w;                        // ILU(0) smoothing levels (FP64): N values of work space
};

// LDS layout of the tail kernel (levels t0 .. L-1 of one problem in one
// workgroup): for each level the byte offsets of f, e, phi and the per-axis
// coefficient arrays, 16-byte rounded and carved level after level; the
// scratch U follows the last level (uoff).  Built on the host (tail_table).
struct TailOff {
    int n[3], N;
    int F, E, PH, A[3], Cc[3], Dd[3];
    int end;
};
struct TailTab {
    TailOff o[HH_MAXLEV];
    FastDiv fx[HH_MAXLEV], fxy[HH_MAXLEV];
    int uoff;
};

// the two levels a V-cycle level kernel works on, passed by value for
// one-problem launches (valid = 0: read them from the problem's descriptor)
template <typename T> struct LvPair {
    LevelDev<T> f, c;
    int valid;
};

// vectors a problem can name in a kernel argument
enum VecSel {
    VS_X = 0, VS_B, VS_R, VS_RH, VS_P, VS_V, VS_T, VS_PH, VS_SH, VS_IN, VS_OUT, VS_W, VS_Q, VS_TMP,
    VS_NVEC
};

// solve phases (first int of every state block)
enum Phase { PH_RUN = 0, PH_HALF = 1, PH_STOP = 2, PH_IDLE = 3 };
// Mixed-precision guard.  With a complex-FP32 V-cycle the preconditioner is
// only accurate to FP32 rounding amplified by the cycle's norm, and on badly
// resolved problems (few points per wavelength) the FP64 outer iteration can
// stall or diverge once its residual nears that level.  A residual far above
// the best one since the last (re)start, or no new best for a long stretch,
// stops the solve so the host continues it from the current iterate with
// the FP64 V-cycle.
// Stage factors of mixed-precision solves (see KBatch): each stage restarts
// from the FP64 true residual once the recurrence residual has dropped by
// this factor.  Measured on 1024^2, a 5.4-points-per-wavelength 512^2 problem,
// MP2/MP3 and 1536^2/2048^2 grids: 1e-1 for Bi-CGSTAB (no FP64 fallback
// left, 1024^2 147 ms against 167 ms unstaged); IDR(4) loses with frequent
// stages (128^3: 497 matvecs at 1e-1 against 396) and takes 1e-4.
#define HH_MIXED_STAGE_BICG 1e-1
#define HH_MIXED_STAGE_IDR 1e-4
#define HH_DRIFT_GROW 1000.0
#define HH_DRIFT_STALL 300           // 0: no stall test

// what a finaliser pass does with the chunk partials of one problem
enum FinKind { FIN_BNORM = 0, FIN_INIT, FIN_ALPHA, FIN_OMEGA, FIN_RHO, FIN_TRUE, FIN_NONE,
               FIN_IDR_OMEGA, FIN_IDR_STEP, FIN_IDR_INIT, FIN_IDR_M };
// stop reasons
enum Reason { RS_NONE = 0, RS_CONV = 1, RS_MAXMV = 2, RS_BREAK = 3, RS_NONFIN = 4, RS_DRIFT = 5 };

struct SolveState {
    int phase, reason, mv, it;
    int max_mv, hist_len;
    unsigned count;                  // blocks of the current reduction done (last one finalises)
    int guard;                       // 1: FP32 V-cycle, drift check on
    double tol, bnorm, rel, true_rel;
    double best_rel;                 // smallest rel since the last (re)start
    int best_mv, drift_stall;        // guard: stop after this many matvecs without a new best
    double drift_grow;               // guard: stop when rel exceeds this multiple of the best
    double2 rho, alpha, omega, beta;
    // IDR(s)
    int s, kstep, oldest, startup;   // kstep in 0..s within a cycle; startup steps left
    double2 om_idr;
    double2 G[HH_MAX_S * HH_MAX_S];  // row major s x s
    double2 m[HH_MAX_S];
    double2 c[HH_MAX_S];
};

// Per-problem control block of a launch plan: the phase and the Krylov
// scalars every pass needs, read by one scalar load from a kernel argument.
struct Ctrl {
    int phase;
    int mode;                        // IDR: 0 start-up step, 1 cycle step k = 0, 2 cycle step k >= 1
    int old;                         // IDR: column of dR/dX this step writes
    int reason;                      // stop reason (host reads it with the phase)
    double2 alpha, beta, omega;      // Bi-CGSTAB
    double2 om_idr;                  // IDR omega
    double2 c[8];                    // IDR: solution of G c = m for this step
};

struct ProbDev {
    int dim, nlev, Nc, ngroup;       // ngroup: chunk groups (partials per value)
    int tail64, tail32;              // first level of the one-workgroup tail kernel, per precision
    int csplit;                      // 1: the coarsest solve runs in k_coarse (many workgroups)
    int n[3];
    int64_t N;
    FastDiv fx, fxy;
    const double2 *aH[3], *cH[3], *dH[3];
    const double *phi;
    const LevelDev<double> *L64;     // device array [nlev]
    const LevelDev<float> *L32;      // device array [nlev] (null if no FP32 set)
    const double2 *Minv64;
    const float2 *Minv32;
    const void *timg64, *timg32;     // LDS image of the tail levels (phi, coefficients), per precision
    const TailTab *ttab64, *ttab32;  // LDS layout of the tail levels, per precision
    int timg_bytes64, timg_bytes32;
    // image segments, one per tail level: LDS offset << 16 | length, in 16-byte units
    uint32_t tseg64[HH_MAXLEV], tseg32[HH_MAXLEV];
    int tnseg64, tnseg32;
    double omega;
    int nu1;                         // pre-smoothing steps of the V-cycle (0 or 1)
    void *vec[VS_NVEC];
    double2 *dR, *dX;                // IDR: s columns of N each
    int nidr;                        // IDR: s
    const double2 *P;                // IDR shadow space, N x s column-major
    double *part;                    // group partials, value-major: part[v * ngroup + g], v < HH_NPART
    SolveState *st;
    Ctrl *ctrl;                      // this problem's slot in the plan's control array
    double *hist;                    // device history (optional)
};

struct Tile {
    int prob, idx;
};

// Launch context passed by value to every kernel.
struct Ctx {
    const ProbDev *P;                // problem descriptors
    const Tile *tiles;               // tile list; null: one problem, tile = blockIdx.x
    const Ctrl *ctrl;                // control blocks; null: every problem runs
    const void *L;                   // one problem: its LevelDev array in the V-cycle precision
    double omega;                    // one problem: Jacobi weight
    int nu1;                         // one problem: pre-smoothing steps (1: V(1,1), 0: V(0,1))
};

// Levels with at most TailCap<T>::N unknowns (and every coarser level) run
// inside one workgroup with all data in LDS.
template <typename T> struct TailCap;
template <> struct TailCap<double> { static constexpr int N = 1024; static constexpr int BYTES = 96 * 1024; static constexpr int WG = 512; };
template <> struct TailCap<float> { static constexpr int N = 1024; static constexpr int BYTES = 64 * 1024; static constexpr int WG = 1024; };

// Tile shapes of the fused V-cycle level kernels (coarse points per axis of
// the down-leg's tile; the up-leg's fine tile is twice it).  The kernels are
// built for every shape of the set and the autotuner picks one per
// (dimension, precision, leg, level class); results do not depend on it.
// In 3D, shapes HH_NBOX and up are z-streaming kernels: a column of X x Y
// coarse points over Z coarse planes, walked plane by plane.
#define HH_NTILE 9
#define HH_NBOX 7
template <int DIM> struct TileSet;
// Fine levels of at least HH_STREAM_MIN unknowns (one problem, 2D, FP32
// cycle) run the legs that stream their per-point inputs and the finest
// output with non-temporal accesses: their fields exceed the 256 MB Infinity
// Cache, so no reuse is lost, and streaming moves this mix of reads and writes
// at a higher rate (4096^2 up-leg 99 -> 88 us).  Smaller levels keep plain
// accesses, which leave f in the cache for the up-leg's second read (2048^2
// legs measured 15% slower streamed).
#define HH_STREAM_MIN (int64_t(8) << 20)

template <> struct TileSet<2> {
    static constexpr int N = HH_NBOX + 1;   // shapes in use (the last a 1024-thread box)
    static constexpr int X[HH_NTILE] = {16, 32, 16, 8, 32, 32, 32, 32, 16};
    static constexpr int Y[HH_NTILE] = {16, 8, 8, 8, 16, 8, 16, 16, 16};
    static constexpr int Z[HH_NTILE] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int T[HH_NTILE] = {256, 256, 256, 256, 256, 512, 512, 1024, 256};   // threads per workgroup
};
template <> struct TileSet<3> {
    static constexpr int N = HH_NTILE;
    static constexpr int X[HH_NTILE] = {4, 8, 8, 4, 8, 8, 8, 16, 8};
    static constexpr int Y[HH_NTILE] = {4, 4, 8, 4, 4, 4, 8, 8, 8};
    static constexpr int Z[HH_NTILE] = {4, 4, 2, 2, 2, 4, 2, 4, 4};
    static constexpr int T[HH_NTILE] = {256, 256, 256, 256, 256, 512, 512, 512, 256};
};
inline int tile_shapes(int dim) { return dim == 2 ? TileSet<2>::N : TileSet<3>::N; }

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
