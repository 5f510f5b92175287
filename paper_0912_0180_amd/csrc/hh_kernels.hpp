// hh_kernels.hpp -- gfx950 kernels of the CSG-preconditioned Helmholtz solver.
//
// Every kernel takes the device array of problem descriptors and a tile list
// (problem id, tile index); one workgroup handles one tile, so one launch
// covers any number of independent problems.  Kernels whose problem is not in
// the running phase return at once.
//
// Arithmetic follows a fixed operation order (no FMA contraction; the build
// passes -ffp-contract=off), so FP64 results are reproducible run to run,
// independent of how problems are batched or tiled, and equal to the
// oracle's value for value:
//   complex multiply (ar*br - ai*bi, ar*bi + ai*br); Jacobi weight
//   g = omega conj(D)/|D|^2 with D = (d_x + d_y + d_z) - phi; stencil
//   y = D u - a_x u_w - c_x u_e - a_y u_s - c_y u_n - a_z u_d - c_z u_u;
//   full weighting (1,3,3,1)/8 applied x, then y, then z; prolongation
//   3/4 near + 1/4 far applied x, then y, then z; reductions over chunks of
//   256 elements (one per thread slot), each chunk a pairwise tree (wave
//   pairs by DPP, then (w0 + w1) + (w2 + w3)), chunk partials by a pairwise
//   tree over their zero-padded power-of-two count.
// The FP32 V-cycle of mixed solves is held to a tolerance against FP64, not
// to this order: its complex products use fused multiply-adds and its
// Jacobi weight the hardware reciprocal.  Every FP32 kernel uses the same
// formulas, so FP32 results are still independent of batching and tiling.
//
// Memory-level parallelism: each thread first issues all of its global loads
// into registers, then computes, then stores, so several HBM requests per
// thread are in flight.  Descriptor fields are copied to registers once per
// workgroup.
#pragma once
#include "hh_common.h"

namespace hh {

// Scale of the Jacobi weight omega / D = (omega / |D|^2) conj(D): the IEEE
// quotient in FP64; FP32 (held to a tolerance) takes the hardware
// reciprocal (1 ulp) and a fused |D|^2.
template <typename T> __device__ inline T jscale(T omega, V2<T> D) { return omega / (D.x * D.x + D.y * D.y); }
template <> __device__ inline float jscale<float>(float omega, V2<float> D)
{
    return omega * __builtin_amdgcn_rcpf(fmaf(D.x, D.x, D.y * D.y));
}
// the Jacobi weight g = omega / D = (D.x q, -(D.y q)), q = jscale(omega, D)
template <typename T> __device__ inline V2<T> jweight(V2<T> D, T omega)
{
    T q = jscale<T>(omega, D);
    return cmk<T>(D.x * q, -(D.y * q));
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Lane exchange by DPP within a row of 16 lanes (CTRL: a quad permute or a
// mirror); every source lane is inside the row, so no lane reads out of range.
template <int CTRL> __device__ inline float dpp_x(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double dpp_x(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline float lane_value(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double lane_value(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l), __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Pairwise tree over the 64 lanes of a wave (all lanes active); every lane
// gets the sum.  Aligned blocks of 1, 2, 4 and 8 lanes are paired with the
// neighbouring block by DPP (xor 1 and xor 2 by quad permutes, then the
// half-row and row mirrors, which pair lane i with the mirror lane of the
// other block; after each step all lanes of a block hold the block sum), then
// the four row sums are combined as (r0 + r1) + (r2 + r3): the tree of the
// xor butterfly, with no LDS traffic.
template <typename T> __device__ inline T wave_sum(T v)
{
    v = v + dpp_x<0xB1>(v);    // quad_perm [1,0,3,2]
    v = v + dpp_x<0x4E>(v);    // quad_perm [2,3,0,1]
    v = v + dpp_x<0x141>(v);   // row_half_mirror
    v = v + dpp_x<0x140>(v);   // row_mirror
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Pairwise tree over the 256 thread slots of a 256-thread workgroup; thread 0
// writes the NV sums to out[q * stride], q < NV.
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], double *out, int64_t stride = 1)
{
    __shared__ double red[4 * NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[w * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q * stride] = (red[q] + red[NV + q]) + (red[2 * NV + q] + red[3 * NV + q]);
}


// Pairwise sum of v[0..n) (stride `stride`; LDS if LOCAL, else global) with
// zero padding to a power of two >= 256, by one 256-thread workgroup; every
// thread gets the sum.  Each thread sums its contiguous segment with the
// iterative (binary counter) form of the pairwise tree, then the slots are
// combined by block_reduce.
template <bool LOCAL>
__device__ inline double pairwise_wg(const double *v, int stride, int n)
{
    int np = 256;
    while (np < n) np <<= 1;
    const int seg = np >> 8;
    const int beg = threadIdx.x * seg;
    double stack[24];
    int top = 0;
    for (int i = 0; i < seg; ++i) {
        int e = beg + i;
        double x = e < n ? (LOCAL ? v[e * stride] : ldg(v, (int64_t)e * stride)) : 0.0;
        for (int c = i; c & 1; c >>= 1) x = stack[--top] + x;
        stack[top++] = x;
    }
    double r[1] = {stack[0]};
    __shared__ double out[1];
    block_reduce<1>(r, out);
    __syncthreads();
    double s = out[0];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// descriptor views (copied to registers once per workgroup)
// ---------------------------------------------------------------------------
struct HView {
    int nx, ny, nz;
    int64_t N;
    FastDiv fx, fxy;
    const double2 *a0, *c0, *d0, *a1, *c1, *d1, *a2, *c2, *d2;
    const double *phi;
};

__host__ __device__ inline HView hview(const ProbDev *pd)
{
    HView h;
    h.nx = pd->n[0];
    h.ny = pd->n[1];
    h.nz = pd->n[2];
    h.N = pd->N;
    h.fx = pd->fx;
    h.fxy = pd->fxy;
    h.a0 = pd->aH[0]; h.c0 = pd->cH[0]; h.d0 = pd->dH[0];
    h.a1 = pd->aH[1]; h.c1 = pd->cH[1]; h.d1 = pd->dH[1];
    h.a2 = pd->aH[2]; h.c2 = pd->cH[2]; h.d2 = pd->dH[2];
    h.phi = pd->phi;
    return h;
}

template <typename T> struct MView {
    int nx, ny, nz;
    int64_t N;
    FastDiv fx, fxy;
    const V2<T> *a0, *c0, *d0, *a1, *c1, *d1, *a2, *c2, *d2;
    const T *phi;
};

template <typename T> __device__ inline MView<T> mview(const LevelDev<T> *L)
{
    MView<T> h;
    h.nx = L->n[0];
    h.ny = L->n[1];
    h.nz = L->n[2];
    h.N = L->N;
    h.fx = L->fx;
    h.fxy = L->fxy;
    h.a0 = L->a[0]; h.c0 = L->c[0]; h.d0 = L->d[0];
    h.a1 = L->a[1]; h.c1 = L->c[1]; h.d1 = L->d[1];
    h.a2 = L->a[2]; h.c2 = L->c[2]; h.d2 = L->d[2];
    h.phi = L->phi;
    return h;
}

template <typename T> __device__ inline const LevelDev<T> *levels(const ProbDev *pd);
template <> __device__ inline const LevelDev<double> *levels<double>(const ProbDev *pd) { return pd->L64; }
template <> __device__ inline const LevelDev<float> *levels<float>(const ProbDev *pd) { return pd->L32; }
template <typename T> __device__ inline int tail_level(const ProbDev *pd);
template <> __device__ inline int tail_level<double>(const ProbDev *pd) { return pd->tail64; }
template <> __device__ inline int tail_level<float>(const ProbDev *pd) { return pd->tail32; }

__device__ inline Tile ldg_tile(const Tile *t, int i)
{
    const HH_GLOBAL int *p = (const HH_GLOBAL int *)(t + i);
    Tile r;
    r.prob = p[0];
    r.idx = p[1];
    return r;
}
// Workgroups are dealt to the eight XCDs round robin (workgroup w runs on
// XCD w mod 8) and every XCD has its own L2.  Renumbering them so that XCD x
// takes one contiguous run of tiles keeps the rows a stencil tile shares with
// its neighbours inside a single L2 instead of fetching them once per XCD.
__device__ inline int xcd_tile_index()
{
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    const int x = b & 7, loc = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
}
__device__ inline Tile tile_of(const Ctx &c)
{
    const int i = xcd_tile_index();
    if (c.tiles) return ldg_tile(c.tiles, i);
    Tile t;
    t.prob = 0;
    t.idx = i;
    return t;
}
__device__ inline int phase_of(const Ctx &c, int prob)
{
    return c.ctrl ? ((const HH_GLOBAL int *)(c.ctrl + prob))[0] : (int)PH_RUN;
}
__device__ inline Ctrl ctrl_of(const Ctx &c, int prob)
{
    const Ctrl *q = c.ctrl + prob;
    Ctrl r;
    const HH_GLOBAL int *qi = (const HH_GLOBAL int *)q;
    r.phase = qi[0];
    r.mode = qi[1];
    r.old = qi[2];
    r.reason = qi[3];
    r.alpha = ldg(&q->alpha, 0);
    r.beta = ldg(&q->beta, 0);
    r.omega = ldg(&q->omega, 0);
    r.om_idr = ldg(&q->om_idr, 0);
#pragma unroll
    for (int i = 0; i < 8; ++i) r.c[i] = ldg(&q->c[i], 0);
    return r;
}
template <typename T> __device__ inline const LevelDev<T> *levels_of(const Ctx &c, const ProbDev *pd)
{
    return c.L ? (const LevelDev<T> *)c.L : levels<T>(pd);
}

template <typename S> __device__ inline double2 ld64(const S *p, int64_t i) { return ccvt<double>(ldg(p, i)); }

__device__ inline void split(int64_t p, int nx, int ny, FastDiv fx, FastDiv fxy, int &i, int &j, int &k)
{
    uint32_t q = fdiv((uint32_t)p, fx);
    i = (int)((uint32_t)p - q * (uint32_t)nx);
    k = (int)fdiv((uint32_t)p, fxy);
    j = (int)(q - (uint32_t)k * (uint32_t)ny);
}

// Stencil of a view V (HView or MView<T>) at point (i,j,k), x of storage S
// converted to precision T.
template <int DIM, typename T, typename VW, typename S>
__device__ inline V2<T> stencil(const VW &h, const S *__restrict__ x, int i, int j, int k, int64_t p)
{
    using C = V2<T>;
    const int64_t sy = h.nx, sz = (int64_t)h.nx * h.ny;
    const C zero = cmk<T>(0, 0);
    C xc = ccvt<T>(ldg(x, p));
    C xw = i > 0 ? ccvt<T>(ldg(x, p - 1)) : zero, xe = i < h.nx - 1 ? ccvt<T>(ldg(x, p + 1)) : zero;
    C xs = j > 0 ? ccvt<T>(ldg(x, p - sy)) : zero, xn = j < h.ny - 1 ? ccvt<T>(ldg(x, p + sy)) : zero;
    C xd = zero, xu = zero;
    if (DIM == 3) {
        xd = k > 0 ? ccvt<T>(ldg(x, p - sz)) : zero;
        xu = k < h.nz - 1 ? ccvt<T>(ldg(x, p + sz)) : zero;
    }
    C d = ldg(h.d0, i);
    d = cadd<T>(d, ldg(h.d1, j));
    if (DIM == 3) d = cadd<T>(d, ldg(h.d2, k));
    C D = cmk<T>(d.x - ldg(h.phi, p), d.y);
    C t = cmul<T>(D, xc);
    t = cmsub<T>(t, ldg(h.a0, i), xw);
    t = cmsub<T>(t, ldg(h.c0, i), xe);
    t = cmsub<T>(t, ldg(h.a1, j), xs);
    t = cmsub<T>(t, ldg(h.c1, j), xn);
    if (DIM == 3) {
        t = cmsub<T>(t, ldg(h.a2, k), xd);
        t = cmsub<T>(t, ldg(h.c2, k), xu);
    }
    return t;
}

// 2D band layout of the operator apply for rows whose length is a multiple of
// 256: a workgroup takes 256 columns of two rows and a thread evaluates its
// column in both rows, loading the x coefficients and the shared centre and
// neighbour values once; every value as in stencil<2, double>.  (The matvec
// kernels of the Krylov iteration keep one chunk per workgroup: their
// per-chunk dot products make the two-row workgroup slower there.)
struct Band {
    int i, j0, nr;
    int64_t p0;
};
__device__ inline Band band_of(const HView &h, int idx)
{
    const int nbx = h.nx >> 8;
    const int bx = idx % nbx, by = idx / nbx;
    Band b;
    b.i = (bx << 8) + (int)threadIdx.x;
    b.j0 = 2 * by;
    b.nr = h.ny - b.j0 < 2 ? h.ny - b.j0 : 2;
    b.p0 = (int64_t)b.j0 * h.nx + b.i;
    return b;
}
template <typename S>
__device__ inline void stencil_band(const HView &h, const S *__restrict__ x, const Band &b, double2 (&y)[2])
{
    using C = double2;
    const C zero = cmk<double>(0, 0);
    const int i = b.i, j0 = b.j0;
    const int64_t sy = h.nx, p0 = b.p0;
    const C a0 = ldg(h.a0, i), c0 = ldg(h.c0, i), d0 = ldg(h.d0, i);
    const C xs = j0 > 0 ? ld64(x, p0 - sy) : zero;
    const C xc = ld64(x, p0);
    const C x1 = j0 < h.ny - 1 ? ld64(x, p0 + sy) : zero;       // row j0 + 1
    const C x2 = j0 + 1 < h.ny - 1 ? ld64(x, p0 + 2 * sy) : zero;
    C w[2], e[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int64_t p = p0 + r * sy;
        const bool in = r < b.nr;
        w[r] = in && i > 0 ? ld64(x, p - 1) : zero;
        e[r] = in && i < h.nx - 1 ? ld64(x, p + 1) : zero;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (r >= b.nr) break;
        const int j = j0 + r;
        const int64_t p = p0 + r * sy;
        const C xcr = r == 0 ? xc : x1, xsr = r == 0 ? xs : xc, xnr = r == 0 ? x1 : x2;
        C d = d0;
        d = cadd<double>(d, ldg(h.d1, j));
        C D = cmk<double>(d.x - ldg(h.phi, p), d.y);
        C t = cmul<double>(D, xcr);
        t = csub<double>(t, cmul<double>(a0, w[r]));
        t = csub<double>(t, cmul<double>(c0, e[r]));
        t = csub<double>(t, cmul<double>(ldg(h.a1, j), xsr));
        t = csub<double>(t, cmul<double>(ldg(h.c1, j), xnr));
        y[r] = t;
    }
}

// ---------------------------------------------------------------------------
// finalisation: one workgroup per problem (k_fin) sums the chunk partials of
// a reducing pass in the fixed pairwise order and advances the scalar state
// ---------------------------------------------------------------------------
#define HH_FIN_STAGE 16384

__device__ inline bool cfin(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__device__ inline void stop(SolveState *st, int reason)
{
    st->phase = PH_STOP;
    st->reason = reason;
}

__device__ inline void record(const ProbDev *pd, SolveState *st, double rel)
{
    st->rel = rel;
    if (pd->hist && st->mv - 1 < st->hist_len && st->mv >= 1) pd->hist[st->mv - 1] = rel;
}

// Sums value first + q (q < nv) of the chunk partials, stored value-major
// (part[v * n + c] for chunk c of n), each by the pairwise tree over the
// zero-padded power-of-two length; results in out[q].  The partials are
// staged in LDS in blocks of HH_FIN_STAGE entries (an aligned power-of-two
// block of a pairwise tree is itself a subtree, so block sums combine
// exactly).
// np = PER * 256 partials of each of G values.  Thread t loads the aligned
// block [t PER, (t+1) PER) of each value (consecutive addresses, zero past
// n) and sums it pairwise in registers; the 256 block sums are combined by
// the wave butterfly and the four-wave sum (block_reduce), which is the same
// tree.  Loading the block directly, rather than coalesced and transposed
// through LDS, saves two barriers per value.
template <int PER, int G>
__device__ inline void reduce_values_blocked(const double *part, int n, int64_t off, int ng, double *out)
{
    const int t = (int)threadIdx.x;
    double r[G][PER];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = t * PER + i;
            r[g][i] = (g < ng && e < n) ? ldg(part, off + (int64_t)g * n + e) : 0.0;
        }
    double sums[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int w = 1; w < PER; w <<= 1)
#pragma unroll
            for (int i = 0; i + w < PER; i += 2 * w) r[g][i] = r[g][i] + r[g][i + w];
        sums[g] = r[g][0];
    }
    __shared__ double tmp[G];
    block_reduce<G>(sums, tmp);
    __syncthreads();
    if (t < ng) out[t] = tmp[t];
}

__device__ void reduce_partials(const double *part, int n, int first, int nv, double *out)
{
    __shared__ double stage[HH_FIN_STAGE];
    __shared__ double bsum[4 * HH_MAX_S + 4][64];
    int np = 1;
    while (np < n) np <<= 1;
    if (np >= HH_WG && np <= 32 * HH_WG) {
        // groups of up to 4 values in flight (1 for the longest blocks); the
        // transpose uses the staging buffer
        const int per = np / HH_WG, G = per <= 16 ? 4 : 1;
        for (int q = 0; q < nv; q += G) {
            const int64_t off = (int64_t)(first + q) * n;
            const int ng = nv - q < G ? nv - q : G;
            switch (per) {
            case 1: reduce_values_blocked<1, 4>(part, n, off, ng, out + q); break;
            case 2: reduce_values_blocked<2, 4>(part, n, off, ng, out + q); break;
            case 4: reduce_values_blocked<4, 4>(part, n, off, ng, out + q); break;
            case 8: reduce_values_blocked<8, 4>(part, n, off, ng, out + q); break;
            case 16: reduce_values_blocked<16, 4>(part, n, off, ng, out + q); break;
            default: reduce_values_blocked<32, 1>(part, n, off, ng, out + q); break;
            }
            __syncthreads();   // block_reduce's LDS is reused by the next group
        }
        return;
    }
    if (np > 32 * HH_WG && np <= 64 * 32 * HH_WG) {
        // longer: aligned blocks of 32 * 256 partials (subtrees) by the
        // blocked path one value at a time, then the block sums pairwise
        constexpr int B = 32 * HH_WG;
        const int nblk = np / B;
        for (int q = 0; q < nv; ++q) {
            for (int b = 0; b < nblk; ++b) {
                const int valid = n - b * B < B ? (n - b * B > 0 ? n - b * B : 0) : B;
                reduce_values_blocked<32, 1>(part, valid, (int64_t)(first + q) * n + (int64_t)b * B, 1, &bsum[q][b]);
                __syncthreads();
            }
        }
        if (threadIdx.x < nv) {
            const int q = threadIdx.x;
            for (int w = 1; w < nblk; w <<= 1)
                for (int i = 0; i + w < nblk; i += 2 * w) bsum[q][i] = bsum[q][i] + bsum[q][i + w];
            out[q] = bsum[q][0];
        }
        __syncthreads();
        return;
    }
    // values per staging pass: all nv at once when they fit
    const int blk = np < HH_FIN_STAGE ? np : HH_FIN_STAGE;
    const int qstep = (HH_FIN_STAGE / blk) < nv ? (HH_FIN_STAGE / blk) : nv;
    const int nblk = np / blk;
    for (int q0 = 0; q0 < nv; q0 += qstep) {
        const int nq = nv - q0 < qstep ? nv - q0 : qstep;
        for (int b = 0; b < nblk; ++b) {
            const int tot = nq * blk;
            for (int e0 = 0; e0 < tot; e0 += 16 * HH_WG) {
                double tmp[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = e0 + threadIdx.x + u * HH_WG;
                    tmp[u] = 0.0;
                    if (e < tot) {
                        const int qq = e / blk, c = b * blk + (e - qq * blk);
                        if (c < n) tmp[u] = ldg(part, (int64_t)(first + q0 + qq) * n + c);
                    }
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int e = e0 + threadIdx.x + u * HH_WG;
                    if (e < tot) stage[e] = tmp[u];
                }
            }
            __syncthreads();
            for (int w = 1; w < blk; w <<= 1) {
                const int pairs = blk / (2 * w);
                for (int e = threadIdx.x; e < nq * pairs; e += HH_WG) {
                    const int qq = e / pairs, i = (e - qq * pairs) * 2 * w;
                    stage[qq * blk + i] = stage[qq * blk + i] + stage[qq * blk + i + w];
                }
                __syncthreads();
            }
            if (threadIdx.x < nq) bsum[q0 + threadIdx.x][b] = stage[threadIdx.x * blk];
            __syncthreads();
        }
    }
    // combine block sums (nblk is a power of two, at most 64 here)
    if (threadIdx.x < nv) {
        const int q = threadIdx.x;
        for (int w = 1; w < nblk; w <<= 1)
            for (int i = 0; i + w < nblk; i += 2 * w) bsum[q][i] = bsum[q][i] + bsum[q][i + w];
        out[q] = bsum[q][0];
    }
    __syncthreads();
}

// copy of the phase and scalars into the plan's control block
__device__ inline void mirror(const ProbDev *pd, const SolveState *st)
{
    if (!pd->ctrl) return;
    Ctrl c;
    c.phase = st->phase;
    c.mode = st->startup >= 0 ? 0 : (st->kstep == 0 ? 1 : 2);
    c.old = st->startup >= 0 ? st->startup : st->oldest;
    c.reason = st->reason;
    c.alpha = st->alpha;
    c.beta = st->beta;
    c.omega = st->omega;
    c.om_idr = st->om_idr;
    for (int i = 0; i < 8; ++i) c.c[i] = i < HH_MAX_S ? st->c[i] : cmk<double>(0.0, 0.0);
    *pd->ctrl = c;
}

// defined with the IDR kernels
__device__ void idr_finalize(const ProbDev *pd, SolveState *st, int kind, const double *s, int phase);
__device__ int idr_nvals(const ProbDev *pd, int kind);

// Scalar state of a Bi-CGSTAB solve, copied to registers before the
// reduction (its loads overlap the partial sums) and written back once.
struct BiLoc {
    int phase, reason, mv, it, max_mv, hist_len, guard, best_mv, drift_stall;
    double tol, bnorm, rel, true_rel, best_rel, drift_grow;
    double2 rho, alpha, omega, beta;
};

// drift check of the mixed-precision guard; updates the best residual
__device__ inline bool drift(double rel, int mv, double &best_rel, int &best_mv, double grow, int stall)
{
    if (rel < best_rel) {
        best_rel = rel;
        best_mv = mv;
        return false;
    }
    return rel > grow * best_rel || (stall > 0 && mv - best_mv > stall);
}

__device__ inline void bi_stop(BiLoc &b, int reason)
{
    b.phase = PH_STOP;
    b.reason = reason;
}

__device__ inline void bi_record(const ProbDev *pd, BiLoc &b, double rel)
{
    b.rel = rel;
    if (pd->hist && b.mv - 1 < b.hist_len && b.mv >= 1) pd->hist[b.mv - 1] = rel;
}

// the phases in which a pass's finalisation advances the state (otherwise the
// problem has stopped, or half-stopped, and the pass is a no-op)
__device__ inline bool fin_runs(int kind, int phase)
{
    if (kind == FIN_RHO) return phase == PH_RUN || phase == PH_HALF;
    if (kind == FIN_ALPHA || kind == FIN_OMEGA) return phase == PH_RUN;
    if (kind >= FIN_IDR_OMEGA && kind != FIN_IDR_INIT) return phase == PH_RUN;
    return true;
}

// gate: skip the update unless fin_runs(kind, phase of the state block),
// decided after the state and the partials are loaded
__device__ __forceinline__ void finalize(const ProbDev *pd, int kind, bool gate)
{
    SolveState *st = pd->st;
    BiLoc b;
    b.phase = st->phase;
    b.reason = st->reason;
    b.mv = st->mv;
    b.it = st->it;
    b.max_mv = st->max_mv;
    b.hist_len = st->hist_len;
    b.tol = st->tol;
    b.bnorm = st->bnorm;
    b.rel = st->rel;
    b.true_rel = st->true_rel;
    b.rho = st->rho;
    b.alpha = st->alpha;
    b.omega = st->omega;
    b.beta = st->beta;
    b.guard = st->guard;
    b.best_rel = st->best_rel;
    b.best_mv = st->best_mv;
    b.drift_stall = st->drift_stall;
    b.drift_grow = st->drift_grow;
    const int phase = b.phase;
    const int nv = kind >= FIN_IDR_OMEGA ? idr_nvals(pd, kind)
                 : (kind == FIN_BNORM || kind == FIN_TRUE) ? 1 : (kind == FIN_ALPHA ? 2 : (kind == FIN_OMEGA ? 4 : 3));
    const int first = (kind == FIN_BNORM || kind == FIN_TRUE) ? 2 : 0;
    __shared__ double res[4 * HH_MAX_S + 4];
    reduce_partials(pd->part, pd->ngroup, first, nv, res);
    const double *s = res;
    if (threadIdx.x != 0) return;
    if (gate && !fin_runs(kind, phase)) return;
    if (kind >= FIN_IDR_OMEGA) {
        idr_finalize(pd, st, kind, s, phase);
        mirror(pd, st);
        return;
    }
    switch (kind) {
    case FIN_BNORM:
        b.bnorm = sqrt(s[0]);
        break;
    case FIN_TRUE:
        b.true_rel = sqrt(s[0]) / b.bnorm;
        break;
    case FIN_INIT: {
        // start (or restart) of Bi-CGSTAB: rho = alpha = omega = 1, then the
        // first beta from rho1 = (rhat, r)
        const double2 one = cmk<double>(1.0, 0.0);
        b.rho = one;
        b.alpha = one;
        b.omega = one;
        b.phase = PH_RUN;
        b.reason = RS_NONE;
        b.best_rel = INFINITY;
        b.best_mv = b.mv;
        double2 rho1 = cmk<double>(s[0], s[1]);
        if (!cfin(rho1)) { bi_stop(b, RS_NONFIN); break; }
        if (rho1.x == 0.0 && rho1.y == 0.0) { bi_stop(b, RS_BREAK); break; }
        b.beta = cmul<double>(cdiv<double>(rho1, b.rho), cdiv<double>(b.alpha, b.omega));
        b.rho = rho1;
        break;
    }
    case FIN_ALPHA: {
        if (phase != PH_RUN) break;
        b.mv += 1;
        double2 rv = cmk<double>(s[0], s[1]);
        if (!cfin(rv)) { bi_stop(b, RS_NONFIN); break; }
        if (rv.x == 0.0 && rv.y == 0.0) { bi_stop(b, RS_BREAK); break; }
        b.alpha = cdiv<double>(b.rho, rv);
        break;
    }
    case FIN_OMEGA: {
        if (phase != PH_RUN) break;
        // half-step check on ||s|| first: when it ends the iteration, t
        // (computed anyway, from the same s) is not used and not counted
        double rel = sqrt(s[3]) / b.bnorm;
        bi_record(pd, b, rel);
        if (!isfinite(rel)) { bi_stop(b, RS_NONFIN); break; }
        if (rel < b.tol) { b.phase = PH_HALF; b.reason = RS_CONV; break; }
        if (b.mv >= b.max_mv) { b.phase = PH_HALF; b.reason = RS_MAXMV; break; }
        if (b.guard && drift(rel, b.mv, b.best_rel, b.best_mv, b.drift_grow, b.drift_stall)) { bi_stop(b, RS_DRIFT); break; }
        b.mv += 1;
        double2 ts = cmk<double>(s[0], s[1]);
        double tt = s[2];
        if (!cfin(ts) || !isfinite(tt)) { bi_stop(b, RS_NONFIN); break; }
        if (tt == 0.0) { bi_stop(b, RS_BREAK); break; }
        b.omega = cmk<double>(ts.x / tt, ts.y / tt);
        break;
    }
    case FIN_RHO: {
        if (phase != PH_RUN && phase != PH_HALF) break;
        b.it += 1;
        if (phase == PH_HALF) { b.phase = PH_STOP; break; }
        double rel = sqrt(s[2]) / b.bnorm;
        bi_record(pd, b, rel);
        if (!isfinite(rel)) { bi_stop(b, RS_NONFIN); break; }
        if (rel < b.tol) { bi_stop(b, RS_CONV); break; }
        if (b.omega.x == 0.0 && b.omega.y == 0.0) { bi_stop(b, RS_BREAK); break; }
        if (b.mv >= b.max_mv) { bi_stop(b, RS_MAXMV); break; }
        if (b.guard && drift(rel, b.mv, b.best_rel, b.best_mv, b.drift_grow, b.drift_stall)) { bi_stop(b, RS_DRIFT); break; }
        double2 rho1 = cmk<double>(s[0], s[1]);
        if (!cfin(rho1)) { bi_stop(b, RS_NONFIN); break; }
        if (rho1.x == 0.0 && rho1.y == 0.0) { bi_stop(b, RS_BREAK); break; }
        b.beta = cmul<double>(cdiv<double>(rho1, b.rho), cdiv<double>(b.alpha, b.omega));
        b.rho = rho1;
        break;
    }
    default:
        break;
    }
    st->phase = b.phase;
    st->reason = b.reason;
    st->mv = b.mv;
    st->it = b.it;
    st->bnorm = b.bnorm;
    st->rel = b.rel;
    st->true_rel = b.true_rel;
    st->rho = b.rho;
    st->alpha = b.alpha;
    st->omega = b.omega;
    st->beta = b.beta;
    st->best_rel = b.best_rel;
    st->best_mv = b.best_mv;
    if (pd->ctrl && kind != FIN_BNORM && kind != FIN_TRUE) {
        Ctrl c;
        c.phase = b.phase;
        c.mode = 0;
        c.old = 0;
        c.reason = b.reason;
        c.alpha = b.alpha;
        c.beta = b.beta;
        c.omega = b.omega;
        c.om_idr = cmk<double>(1.0, 0.0);
        for (int i = 0; i < 8; ++i) c.c[i] = cmk<double>(0.0, 0.0);
        *pd->ctrl = c;
    }
}

// Writes the group partials of a Krylov workgroup (HH_GROUP chunks, chunk s
// held by waves 4s..4s+3, one unknown per thread) as values first .. first +
// NV - 1; the pass's finalisation runs in k_fin.  Each chunk is summed by its
// pairwise tree (wave sums, then (w0 + w1) + (w2 + w3)); the chunk sums are
// then combined pairwise over the first min(HH_GROUP, np) of them, np the
// problem's chunk count rounded up to a power of two.  That is this group's
// node of the pairwise tree over the zero-padded chunk partials, and k_fin
// sums the group partials by the rest of the same tree.
template <int NV>
__device__ inline void group_finish(const ProbDev *pd, int grp, double (&acc)[NV], int first = 0)
{
    static_assert(HH_PER_SLOT == 1 && HH_CHUNK == 256, "a chunk is four waves of one unknown per thread");
    __shared__ double red[HH_VWG / 64][NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = wave_sum(acc[q]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[w][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int q = threadIdx.x;
        const int64_t nch = (pd->N + HH_CHUNK - 1) / HH_CHUNK;
        int width = 1;
        while (width < HH_GROUP && width < nch) width <<= 1;
        double c[HH_GROUP];
#pragma unroll
        for (int s = 0; s < HH_GROUP; ++s) c[s] = (red[4 * s][q] + red[4 * s + 1][q]) + (red[4 * s + 2][q] + red[4 * s + 3][q]);
#pragma unroll
        for (int h = 1; h < HH_GROUP; h <<= 1)
            if (h < width)
#pragma unroll
                for (int i = 0; i + h < HH_GROUP; i += 2 * h) c[i] = c[i] + c[i + h];
        pd->part[(int64_t)(first + q) * pd->ngroup + grp] = c[0];
    }
}

// One workgroup per problem: sums the chunk partials of the pass just run and
// advances the scalar state (kind = FinKind).
__global__ __launch_bounds__(HH_WG) void k_fin(Ctx cx, const int *__restrict__ probs, int kind)
{
    const int prob = probs ? probs[blockIdx.x] : 0;
    const ProbDev *pd = cx.P + prob;
    // the control block mirrors the phase of the state block; one load
    if (!fin_runs(kind, phase_of(cx, prob))) return;
    finalize(pd, kind, false);
}

// k_fin of a one-problem plan: the problem descriptor comes by value, so the
// loads of the state block and of the partials issue together instead of
// behind the control block's phase and the descriptor's pointers (three
// dependent round trips to memory the other XCDs wrote); the phase gate is
// applied after them, on the state block's phase (which the control block
// mirrors).
__global__ __launch_bounds__(HH_WG) void k_fin1(int kind, ProbDev pv)
{
    finalize(&pv, kind, true);
}

// ---------------------------------------------------------------------------
// operator apply (standalone): y = H x or y = M x on the finest level
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(HH_WG) void k_applyH(Ctx cx, const void *xp, void *yp)
{
    const Tile tl = tile_of(cx);
    const HView h = hview(cx.P + tl.prob);
    const double2 *__restrict__ x = (const double2 *)xp;
    double2 *__restrict__ y = (double2 *)yp;
    const int64_t base = (int64_t)tl.idx * HH_CHUNK;
    double2 out[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = base + threadIdx.x + (int64_t)HH_WG * s;
        if (p < h.N) {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            out[s] = stencil<DIM, double>(h, x, i, j, k, p);
        }
    }
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = base + threadIdx.x + (int64_t)HH_WG * s;
        if (p < h.N) stg(y, p, out[s]);
    }
}

// y = H x in the 2D band layout (one problem, no tile list)
// (the operator's view comes by value: no dependent load of the problem
// descriptor ahead of the data loads, every workgroup being resident at once;
// y is written with streaming stores, 20% faster back to back at 1024^2)
__global__ __launch_bounds__(HH_WG) void k_applyH_band(HView h, const void *xp, void *yp)
{
    const Band b = band_of(h, xcd_tile_index());
    double2 y[2];
    stencil_band(h, (const double2 *)xp, b, y);
    double2 *__restrict__ yo = (double2 *)yp;
    stg_nt(yo, b.p0, y[0]);
    if (b.nr > 1) stg_nt(yo, b.p0 + h.nx, y[1]);
}

template <int DIM, typename T>
__global__ __launch_bounds__(HH_WG) void k_applyM(Ctx cx, const void *xp, void *yp)
{
    const Tile tl = tile_of(cx);
    const MView<T> h = mview<T>(levels_of<T>(cx, cx.P + tl.prob));
    const V2<T> *__restrict__ x = (const V2<T> *)xp;
    V2<T> *__restrict__ y = (V2<T> *)yp;
    const int64_t base = (int64_t)tl.idx * HH_CHUNK;
    V2<T> out[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = base + threadIdx.x + (int64_t)HH_WG * s;
        if (p < h.N) {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            out[s] = stencil<DIM, T>(h, x, i, j, k, p);
        }
    }
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = base + threadIdx.x + (int64_t)HH_WG * s;
        if (p < h.N) stg(y, p, out[s]);
    }
}

// ---------------------------------------------------------------------------
// fused V-cycle down-leg on level lev -> lev+1:
//   u1 = g f (one Jacobi sweep from zero), r = f - M u1, f_{lev+1} = R r.
// Only f_{lev+1} is written; u1 is recomputed by the up-leg.
// Tile = a box of coarse points; LDS holds f, phi and u1 on the fine box
// with a halo of 2 (restriction footprint + stencil).
// ---------------------------------------------------------------------------
template <int DIM, typename T, typename TF, int VT>
__device__ __forceinline__ void vdown_box(Ctx cx, int lev, int fsel, const void *fptr, LvPair<T> lp)
{
    using C = V2<T>;
    constexpr int CX = TileSet<DIM>::X[VT], CY = TileSet<DIM>::Y[VT], CZ = DIM == 3 ? TileSet<DIM>::Z[VT] : 1;
    constexpr int NT = TileSet<DIM>::T[VT];   // threads
    constexpr int RX = 2 * CX + 4, RY = 2 * CY + 4, RZ = DIM == 3 ? 2 * CZ + 4 : 1;
    constexpr int RN = RX * RY * RZ;
    constexpr int RM = RX > RY ? (RX > RZ ? RX : RZ) : (RY > RZ ? RY : RZ);
    constexpr int NL = (RN + NT - 1) / NT;
    // u1 and the residual go through LDS (the stencil and the restriction
    // read neighbours); each thread keeps f and the diagonal of the box points
    // it loaded in registers for the residual at the same points
    __shared__ C U[RN];
    __shared__ C R[RN];
    __shared__ C A[3][RM];
    __shared__ C Cc[3][RM];
    __shared__ C Dd[3][RM];

    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    // one problem: the level descriptors come by value and the phase load
    // overlaps the data loads; a batch reads both from memory first
    LevelDev<T> Lf, Lc;
    int run = PH_RUN;
    if (lp.valid) {
        run = phase_of(cx, tl.prob);
        Lf = lp.f;
        Lc = lp.c;
    } else {
        if (phase_of(cx, tl.prob) != PH_RUN) return;
        const LevelDev<T> *Lv = levels_of<T>(cx, pd);
        Lf = Lv[lev];
        Lc = Lv[lev + 1];
    }
    const int nfx = Lf.n[0], nfy = Lf.n[1], nfz = Lf.n[2];
    const int ncx = Lc.n[0], ncy = Lc.n[1], ncz = Lc.n[2];
    const V2<T> *ax0 = Lf.a[0], *cx0 = Lf.c[0], *dx0 = Lf.d[0];
    const V2<T> *ax1 = Lf.a[1], *cx1 = Lf.c[1], *dx1 = Lf.d[1];
    const V2<T> *ax2 = Lf.a[2], *cx2 = Lf.c[2], *dx2 = Lf.d[2];
    const T *__restrict__ phi = Lf.phi;
    C *__restrict__ fout = Lc.f;
    const TF *__restrict__ f = lev == 0 ? (const TF *)(fptr ? fptr : pd->vec[fsel]) : (const TF *)Lf.f;
    const T omega = (T)(cx.L ? cx.omega : pd->omega);
    const bool pre = (cx.L ? cx.nu1 : pd->nu1) != 0;   // V(1,1), or V(0,1) without pre-smoothing
    const int tx = (ncx + CX - 1) / CX, ty = (ncy + CY - 1) / CY;
    int t = tl.idx;
    const int bx = t % tx;
    t /= tx;
    const int by = t % ty, bz = t / ty;
    const int c0x = bx * CX, c0y = by * CY, c0z = DIM == 3 ? bz * CZ : 0;
    const int ox = 2 * c0x - 2, oy = 2 * c0y - 2, oz = DIM == 3 ? 2 * c0z - 2 : 0;
    const C zero = cmk<T>(0, 0);
    const int64_t sy = nfx, sz = (int64_t)nfx * nfy;

    // issue all global loads of the box first
    TF fr[NL];
    T pr[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = threadIdx.x + q * NT;
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        const bool in = l < RN && gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz));
        if (in) {
            const int64_t p = gx + sy * gy + sz * gz;
            fr[q] = ldg(f, p);
            pr[q] = ldg(phi, p);
        }
    }
    for (int l = threadIdx.x; l < RX + RY + RZ; l += NT) {
        const int ax = l < RX ? 0 : (l < RX + RY ? 1 : 2);
        const int q = ax == 0 ? l : (ax == 1 ? l - RX : l - RX - RY);
        const int g = (ax == 0 ? ox : (ax == 1 ? oy : oz)) + q;
        const int nn = ax == 0 ? nfx : (ax == 1 ? nfy : nfz);
        const bool in = (ax < DIM) && g >= 0 && g < nn;
        const V2<T> *pa = ax == 0 ? ax0 : (ax == 1 ? ax1 : ax2);
        const V2<T> *pc = ax == 0 ? cx0 : (ax == 1 ? cx1 : cx2);
        const V2<T> *pdd = ax == 0 ? dx0 : (ax == 1 ? dx1 : dx2);
        A[ax][q] = in ? ldg(pa, g) : zero;
        Cc[ax][q] = in ? ldg(pc, g) : zero;
        Dd[ax][q] = in ? ldg(pdd, g) : zero;
    }
    if (run != PH_RUN) return;   // uniform over the workgroup
    __syncthreads();
    C fk[NL], Dk[NL];
    // step 1: u1 = g f on the whole box
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = threadIdx.x + q * NT;
        if (l >= RN) break;
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        C u1 = zero;
        fk[q] = Dk[q] = zero;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz))) {
            const C fv = ccvt<T>(fr[q]);
            C d = cadd<T>(Dd[0][lx], Dd[1][ly]);
            if (DIM == 3) d = cadd<T>(d, Dd[2][lz]);
            C D = cmk<T>(d.x - pr[q], d.y);
            T qq = jscale<T>(omega, D);
            C gw = cmk<T>(D.x * qq, -(D.y * qq));
            fk[q] = fv;
            Dk[q] = D;
            if (pre) u1 = cmul<T>(gw, fv);
        }
        U[l] = u1;
    }
    __syncthreads();
    // step 2: r = f - M u1 on the box minus its outer ring (the restriction's
    // footprint), zero outside the grid, for the points each thread loaded
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = threadIdx.x + q * NT;
        if (l >= RN) break;
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        if (lx == 0 || lx == RX - 1 || ly == 0 || ly == RY - 1 || (DIM == 3 && (lz == 0 || lz == RZ - 1))) continue;
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        C res = zero;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz))) {
            C mu = cmul<T>(Dk[q], U[l]);
            mu = cmsub<T>(mu, A[0][lx], U[l - 1]);
            mu = cmsub<T>(mu, Cc[0][lx], U[l + 1]);
            mu = cmsub<T>(mu, A[1][ly], U[l - RX]);
            mu = cmsub<T>(mu, Cc[1][ly], U[l + RX]);
            if (DIM == 3) {
                mu = cmsub<T>(mu, A[2][lz], U[l - RX * RY]);
                mu = cmsub<T>(mu, Cc[2][lz], U[l + RX * RY]);
            }
            res = csub<T>(fk[q], mu);
        }
        R[l] = res;
    }
    __syncthreads();
    // step 3: full weighting, x then y then z
    const T w0 = (T)0.125, w1 = (T)0.375;
    for (int cl = threadIdx.x; cl < CX * CY * CZ; cl += NT) {
        const int ix = cl % CX, iy = (cl / CX) % CY, iz = cl / (CX * CY);
        const int I = c0x + ix, J = c0y + iy, K = c0z + iz;
        if (I >= ncx || J >= ncy || (DIM == 3 && K >= ncz)) continue;
        const int bxl = 2 * ix + 1, byl = 2 * iy + 1, bzl = DIM == 3 ? 2 * iz + 1 : 0;
        C acc_z = zero;
        for (int c = 0; c < (DIM == 3 ? 4 : 1); ++c) {
            const T wz = (c == 0 || c == 3) ? w0 : w1;
            C acc_y = zero;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T wy = (b == 0 || b == 3) ? w0 : w1;
                const C *row = &R[bxl + RX * ((byl + b) + RY * (bzl + c))];
                C sx = crs<T>(w0, row[0]);
                sx = crsadd<T>(sx, w1, row[1]);
                sx = crsadd<T>(sx, w1, row[2]);
                sx = crsadd<T>(sx, w0, row[3]);
                acc_y = b == 0 ? crs<T>(wy, sx) : crsadd<T>(acc_y, wy, sx);
            }
            if (DIM == 3) acc_z = c == 0 ? crs<T>(wz, acc_y) : crsadd<T>(acc_z, wz, acc_y);
            else acc_z = acc_y;
        }
        stg(fout, I + (int64_t)ncx * (J + (int64_t)ncy * K), acc_z);
    }
}

// ---------------------------------------------------------------------------
// fused V-cycle up-leg on level lev (coarse correction from lev+1):
//   u2 = g f + P e_{lev+1},  u = u2 + g (f - M u2).
// Output: e_lev (lev >= 1) or the output vector (lev == 0, storage TO).
// ---------------------------------------------------------------------------
template <int DIM, typename T, typename TF, typename TO, int VT>
__device__ __forceinline__ void vup_box(Ctx cx, int lev, int fsel, int osel, const void *fptr, void *optr, LvPair<T> lp)
{
    using C = V2<T>;
    constexpr int CX = TileSet<DIM>::X[VT], CY = TileSet<DIM>::Y[VT], CZ = DIM == 3 ? TileSet<DIM>::Z[VT] : 1;
    constexpr int NT = TileSet<DIM>::T[VT];   // threads
    constexpr int FX = 2 * CX, FY = 2 * CY, FZ = DIM == 3 ? 2 * CZ : 1;
    constexpr int RX = FX + 2, RY = FY + 2, RZ = DIM == 3 ? FZ + 2 : 1;
    constexpr int RN = RX * RY * RZ;
    constexpr int EX = CX + 4, EY = CY + 4, EZ = DIM == 3 ? CZ + 4 : 1;
    constexpr int EN = EX * EY * EZ;
    constexpr int RM = RX > RY ? (RX > RZ ? RX : RZ) : (RY > RZ ? RY : RZ);
    constexpr int NL = (RN + NT - 1) / NT;
    constexpr int NE = (EN + NT - 1) / NT;
    // only u2 goes through LDS (the stencil reads its neighbours); each
    // thread keeps f, the diagonal and the Jacobi weight of the box points it
    // loaded in registers for the post-smoothing of the same points
    __shared__ C U[RN];
    __shared__ C E[EN];
    __shared__ C A[3][RM];
    __shared__ C Cc[3][RM];
    __shared__ C Dd[3][RM];

    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    // one problem: the level descriptors come by value and the phase load
    // overlaps the data loads; a batch reads both from memory first
    LevelDev<T> Lf, Lc;
    int run = PH_RUN;
    if (lp.valid) {
        run = phase_of(cx, tl.prob);
        Lf = lp.f;
        Lc = lp.c;
    } else {
        if (phase_of(cx, tl.prob) != PH_RUN) return;
        const LevelDev<T> *Lv = levels_of<T>(cx, pd);
        Lf = Lv[lev];
        Lc = Lv[lev + 1];
    }
    const int nfx = Lf.n[0], nfy = Lf.n[1], nfz = Lf.n[2];
    const int ncx = Lc.n[0], ncy = Lc.n[1], ncz = Lc.n[2];
    const V2<T> *ax0 = Lf.a[0], *cx0 = Lf.c[0], *dx0 = Lf.d[0];
    const V2<T> *ax1 = Lf.a[1], *cx1 = Lf.c[1], *dx1 = Lf.d[1];
    const V2<T> *ax2 = Lf.a[2], *cx2 = Lf.c[2], *dx2 = Lf.d[2];
    const T *__restrict__ phi = Lf.phi;
    const C *__restrict__ ec = Lc.e;
    C *__restrict__ eout = Lf.e;
    const TF *__restrict__ f = lev == 0 ? (const TF *)(fptr ? fptr : pd->vec[fsel]) : (const TF *)Lf.f;
    TO *__restrict__ outv = lev == 0 ? (TO *)(optr ? optr : pd->vec[osel]) : nullptr;
    const T omega = (T)(cx.L ? cx.omega : pd->omega);
    const bool pre = (cx.L ? cx.nu1 : pd->nu1) != 0;   // V(1,1), or V(0,1) without pre-smoothing
    const int tx = (nfx + FX - 1) / FX, ty = (nfy + FY - 1) / FY;
    int t = tl.idx;
    const int bx = t % tx;
    t /= tx;
    const int by = t % ty, bz = t / ty;
    const int f0x = bx * FX, f0y = by * FY, f0z = DIM == 3 ? bz * FZ : 0;
    const int ox = f0x - 1, oy = f0y - 1, oz = DIM == 3 ? f0z - 1 : 0;
    const int ex0 = (f0x >> 1) - 2, ey0 = (f0y >> 1) - 2, ez0 = DIM == 3 ? (f0z >> 1) - 2 : 0;
    const C zero = cmk<T>(0, 0);
    const int64_t sy = nfx, sz = (int64_t)nfx * nfy;

    // all global loads first: f and phi on the box, e on the coarse box
    TF fr[NL];
    T pr[NL];
    C er[NE];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = threadIdx.x + q * NT;
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        const bool in = l < RN && gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz));
        if (in) {
            const int64_t p = gx + sy * gy + sz * gz;
            fr[q] = ldg(f, p);
            pr[q] = ldg(phi, p);
        }
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int l = threadIdx.x + q * NT;
        const int lx = l % EX, ly = (l / EX) % EY, lz = l / (EX * EY);
        const int gx = ex0 + lx, gy = ey0 + ly, gz = ez0 + lz;
        er[q] = zero;
        if (l < EN && gx >= 0 && gx < ncx && gy >= 0 && gy < ncy && (DIM == 2 || (gz >= 0 && gz < ncz)))
            er[q] = ldg(ec, gx + (int64_t)ncx * (gy + (int64_t)ncy * gz));
    }
    for (int l = threadIdx.x; l < RX + RY + RZ; l += NT) {
        const int ax = l < RX ? 0 : (l < RX + RY ? 1 : 2);
        const int q = ax == 0 ? l : (ax == 1 ? l - RX : l - RX - RY);
        const int g = (ax == 0 ? ox : (ax == 1 ? oy : oz)) + q;
        const int nn = ax == 0 ? nfx : (ax == 1 ? nfy : nfz);
        const bool in = (ax < DIM) && g >= 0 && g < nn;
        const V2<T> *pa = ax == 0 ? ax0 : (ax == 1 ? ax1 : ax2);
        const V2<T> *pc = ax == 0 ? cx0 : (ax == 1 ? cx1 : cx2);
        const V2<T> *pdd = ax == 0 ? dx0 : (ax == 1 ? dx1 : dx2);
        A[ax][q] = in ? ldg(pa, g) : zero;
        Cc[ax][q] = in ? ldg(pc, g) : zero;
        Dd[ax][q] = in ? ldg(pdd, g) : zero;
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int l = threadIdx.x + q * NT;
        if (l < EN) E[l] = er[q];
    }
    if (run != PH_RUN) return;   // uniform over the workgroup
    __syncthreads();
    const T p3 = (T)0.75, p1 = (T)0.25;
    C fk[NL], Dk[NL], gk[NL];
    // step 1: u2 = g f + P e on the tile plus a halo of one
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = threadIdx.x + q * NT;
        if (l >= RN) break;
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        C fv = zero, u2 = zero;
        fk[q] = Dk[q] = gk[q] = zero;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz))) {
            fv = ccvt<T>(fr[q]);
            const T ph = pr[q];
            C d = cadd<T>(Dd[0][lx], Dd[1][ly]);
            if (DIM == 3) d = cadd<T>(d, Dd[2][lz]);
            C D = cmk<T>(d.x - ph, d.y);
            T qq = jscale<T>(omega, D);
            C gw = cmk<T>(D.x * qq, -(D.y * qq));
            fk[q] = fv;
            Dk[q] = D;
            gk[q] = gw;
            C u1 = pre ? cmul<T>(gw, fv) : zero;
            const int Ix = (gx >> 1) - ex0, Iox = ((gx & 1) ? (gx >> 1) + 1 : (gx >> 1) - 1) - ex0;
            const int Iy = (gy >> 1) - ey0, Ioy = ((gy & 1) ? (gy >> 1) + 1 : (gy >> 1) - 1) - ey0;
            C pe;
            if (DIM == 2) {
                C a0 = crs2<T>(p3, E[Ix + EX * Iy], p1, E[Iox + EX * Iy]);
                C a1 = crs2<T>(p3, E[Ix + EX * Ioy], p1, E[Iox + EX * Ioy]);
                pe = crs2<T>(p3, a0, p1, a1);
            } else {
                const int Iz = (gz >> 1) - ez0, Ioz = ((gz & 1) ? (gz >> 1) + 1 : (gz >> 1) - 1) - ez0;
                C pz[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int zz = c == 0 ? Iz : Ioz;
                    C a0 = crs2<T>(p3, E[Ix + EX * (Iy + EY * zz)], p1, E[Iox + EX * (Iy + EY * zz)]);
                    C a1 = crs2<T>(p3, E[Ix + EX * (Ioy + EY * zz)], p1, E[Iox + EX * (Ioy + EY * zz)]);
                    pz[c] = crs2<T>(p3, a0, p1, a1);
                }
                pe = crs2<T>(p3, pz[0], p1, pz[1]);
            }
            u2 = cadd<T>(u1, pe);
        }
        U[l] = u2;
    }
    __syncthreads();
    // step 2: post-smoothing on the tile (the box points this thread owns,
    // the halo left out)
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = threadIdx.x + q * NT;
        if (l >= RN) break;
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const bool halo = lx == 0 || lx == RX - 1 || ly == 0 || ly == RY - 1 || (DIM == 3 && (lz == 0 || lz == RZ - 1));
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        if (halo || gx >= nfx || gy >= nfy || (DIM == 3 && gz >= nfz)) continue;
        const C D = Dk[q], gw = gk[q];
        C mu = cmul<T>(D, U[l]);
        mu = cmsub<T>(mu, A[0][lx], U[l - 1]);
        mu = cmsub<T>(mu, Cc[0][lx], U[l + 1]);
        mu = cmsub<T>(mu, A[1][ly], U[l - RX]);
        mu = cmsub<T>(mu, Cc[1][ly], U[l + RX]);
        if (DIM == 3) {
            mu = cmsub<T>(mu, A[2][lz], U[l - RX * RY]);
            mu = cmsub<T>(mu, Cc[2][lz], U[l + RX * RY]);
        }
        C u = cmadd<T>(U[l], gw, csub<T>(fk[q], mu));
        const int64_t p = gx + sy * gy + sz * gz;
        if (lev == 0) {
            TO o;
            o.x = u.x;
            o.y = u.y;
            stg(outv, p, o);
        } else {
            stg(eout, p, u);
        }
    }
}

// ---------------------------------------------------------------------------
// 2D forms of the fused legs.  A workgroup owns the same coarse tile as the
// box form, and every point's arithmetic is the box form's, operation for
// operation; only the assignment of points to threads differs.  Thread
// (tx, ty) = (t mod FX, t / FX) owns fine column tx of rows ty, ty + PR, ...,
// ty + (NP - 1) PR (FX = 2 CX a power of two, PR = NT / FX), so the row
// offsets of its loads, LDS slots and coarse reads are compile-time
// constants, and its Jacobi data stay in registers between the steps.  The
// halo rings around the owned points go one point per thread.  A tile whose
// fine box lies inside the grid takes a path without bounds checks (the
// choice is uniform over the workgroup).
// ---------------------------------------------------------------------------

// Point h of the ring at distance dist around an FX x FY tile, relative to
// the tile's first point: the two rows (length FX + 2 dist), then the two
// columns without the corners.  The ring has 2 FX + 2 FY + 8 dist - 4 points.
template <int FX, int FY> __device__ __forceinline__ void ring_point(int h, int dist, int &hx, int &hy)
{
    const int W = FX + 2 * dist;
    if (h < 2 * W) {
        hx = (h < W ? h : h - W) - dist;
        hy = h < W ? -dist : FY - 1 + dist;
    } else {
        const int k = h - 2 * W, Hc = FY + 2 * dist - 2;
        hx = k < Hc ? -dist : FX - 1 + dist;
        hy = (k < Hc ? k : k - Hc) - dist + 1;
    }
}

template <typename T, int RM> struct PlaneTables {
    V2<T> A[2][RM], Cc[2][RM], Dd[2][RM];
};
// LDS of the 2D legs: u on the fine box, the residual (down) or the coarse
// box of e (up), and the coefficient tables
template <typename T, int RN, int RM> struct DownLds {
    V2<T> U[RN], R[RN];
    PlaneTables<T, RM> tb;
};
template <typename T, int RN, int EN, int RM> struct UpLds {
    V2<T> U[RN], E[EN];
    PlaneTables<T, RM> tb;
};
template <int VT> struct PlaneDown {
    static constexpr int CX = TileSet<2>::X[VT], CY = TileSet<2>::Y[VT];
    static constexpr int RX = 2 * CX + 4, RY = 2 * CY + 4, RN = RX * RY, RM = RX > RY ? RX : RY;
};
template <int VT> struct PlaneUp {
    static constexpr int CX = TileSet<2>::X[VT], CY = TileSet<2>::Y[VT];
    static constexpr int RX = 2 * CX + 2, RY = 2 * CY + 2, RN = RX * RY, RM = RX > RY ? RX : RY;
    static constexpr int EN = (CX + 4) * (CY + 4);
};

// x and y coefficient tables of the fine box [ox, ox + RX) x [oy, oy + RY)
// (zero outside the grid).  The axis is chosen by selects, not by indexing
// the descriptor's arrays, which would move the descriptor to scratch memory.
template <typename T, int RX, int RY, int RM, int NT>
__device__ __forceinline__ void plane_tables(PlaneTables<T, RM> &tb, const LevelDev<T> &Lf, int ox, int oy)
{
    for (int l = threadIdx.x; l < RX + RY; l += NT) {
        const bool ya = l >= RX;
        const int q = ya ? l - RX : l;
        const int g = (ya ? oy : ox) + q;
        const bool in = g >= 0 && g < (ya ? Lf.n[1] : Lf.n[0]);
        const V2<T> z = cmk<T>(0, 0);
        const V2<T> *pa = ya ? Lf.a[1] : Lf.a[0], *pc = ya ? Lf.c[1] : Lf.c[0], *pd = ya ? Lf.d[1] : Lf.d[0];
        const int ax = ya ? 1 : 0;
        tb.A[ax][q] = in ? ldg(pa, g) : z;
        tb.Cc[ax][q] = in ? ldg(pc, g) : z;
        tb.Dd[ax][q] = in ? ldg(pd, g) : z;
    }
}

// the diagonal D = d_x + d_y - phi and the Jacobi weight g = omega / D
template <typename T>
__device__ __forceinline__ void plane_jacobi(V2<T> dx, V2<T> dy, T ph, T omega, V2<T> &D, V2<T> &gw)
{
    const V2<T> d = cadd<T>(dx, dy);
    D = cmk<T>(d.x - ph, d.y);
    const T qq = jscale<T>(omega, D);
    gw = cmk<T>(D.x * qq, -(D.y * qq));
}

// r = f - M u at box slot l (stencil in LDS)
template <typename T, int RX>
__device__ __forceinline__ V2<T> plane_resid(const V2<T> *U, int l, V2<T> D, V2<T> f, V2<T> ax, V2<T> cxx, V2<T> ay,
                                             V2<T> cy)
{
    V2<T> mu = cmul<T>(D, U[l]);
    mu = cmsub<T>(mu, ax, U[l - 1]);
    mu = cmsub<T>(mu, cxx, U[l + 1]);
    mu = cmsub<T>(mu, ay, U[l - RX]);
    mu = cmsub<T>(mu, cy, U[l + RX]);
    return csub<T>(f, mu);
}

// bilinear prolongation of the coarse box E at fine point (gx, gy)
template <typename T, int EX>
__device__ __forceinline__ V2<T> plane_prolong(const V2<T> *E, int Ix, int Iox, int Iy, int Ioy)
{
    const T p3 = (T)0.75, p1 = (T)0.25;
    const V2<T> a0 = crs2<T>(p3, E[Ix + EX * Iy], p1, E[Iox + EX * Iy]);
    const V2<T> a1 = crs2<T>(p3, E[Ix + EX * Ioy], p1, E[Iox + EX * Ioy]);
    return crs2<T>(p3, a0, p1, a1);
}

// 2D down-leg of the tile at coarse (c0x, c0y): u1 = g f on the fine box
// (owned points plus two rings), r = f - M u1 on the owned points and the
// first ring, full weighting onto the coarse tile.
template <typename T, typename TF, int VT, bool EDGE, bool STREAM>
__device__ __forceinline__ void vdown_plane_tile(DownLds<T, PlaneDown<VT>::RN, PlaneDown<VT>::RM> &sm,
                                                 const LevelDev<T> &Lf, const LevelDev<T> &Lc, const TF *__restrict__ f,
                                                 T omega, bool pre, int c0x, int c0y, bool run)
{
    using C = V2<T>;
    constexpr int CX = TileSet<2>::X[VT], CY = TileSet<2>::Y[VT], NT = TileSet<2>::T[VT];
    constexpr int FX = 2 * CX, FY = 2 * CY;
    constexpr int RX = FX + 4, RY = FY + 4, RN = RX * RY, RM = RX > RY ? RX : RY;
    constexpr int PR = NT / FX, NP = FY / PR;
    constexpr int N1 = 2 * FX + 2 * FY + 4, N2 = 2 * FX + 2 * FY + 12;
    static_assert((FX & (FX - 1)) == 0 && NT % FX == 0 && FY % PR == 0 && N1 <= NT && N2 <= NT, "2D down-leg tile");
    static_assert(RN == PlaneDown<VT>::RN && RM == PlaneDown<VT>::RM, "2D down-leg LDS");
    C *U = sm.U, *R = sm.R;
    PlaneTables<T, RM> &tb = sm.tb;

    const int nfx = Lf.n[0], nfy = Lf.n[1], ncx = Lc.n[0], ncy = Lc.n[1];
    const T *__restrict__ phi = Lf.phi;
    const int64_t sy = nfx;
    const int f0x = 2 * c0x, f0y = 2 * c0y, ox = f0x - 2, oy = f0y - 2;
    const int tx = threadIdx.x & (FX - 1), ty = threadIdx.x / FX;
    const int gx = f0x + tx;
    const int64_t p0 = (int64_t)(f0y + ty) * sy + gx, dq = (int64_t)PR * sy;
    const C zero = cmk<T>(0, 0);

    // loads: owned points, one point of each ring, the coefficient tables
    TF fr[NP];
    T pr[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        if (!EDGE || (gx < nfx && f0y + ty + q * PR < nfy)) {
            fr[q] = STREAM ? ldg_nt(f, p0 + q * dq) : ldg(f, p0 + q * dq);
            pr[q] = STREAM ? ldg_nt(phi, p0 + q * dq) : ldg(phi, p0 + q * dq);
        }
    }
    const int t1 = threadIdx.x, t2 = NT - 1 - (int)threadIdx.x;   // ring slots (ring 2 from the last thread)
    int h1x = 0, h1y = 0, h2x = 0, h2y = 0;
    if (t1 < N1) ring_point<FX, FY>(t1, 1, h1x, h1y);
    if (t2 < N2) ring_point<FX, FY>(t2, 2, h2x, h2y);
    const int g1x = f0x + h1x, g1y = f0y + h1y, g2x = f0x + h2x, g2y = f0y + h2y;
    const bool in1 = t1 < N1 && (!EDGE || (g1x >= 0 && g1x < nfx && g1y >= 0 && g1y < nfy));
    const bool in2 = t2 < N2 && (!EDGE || (g2x >= 0 && g2x < nfx && g2y >= 0 && g2y < nfy));
    TF f1, f2;
    T ph1 = 0, ph2 = 0;
    if (in1) {
        f1 = ldg(f, g1x + sy * g1y);
        ph1 = ldg(phi, g1x + sy * g1y);
    }
    if (in2) {
        f2 = ldg(f, g2x + sy * g2y);
        ph2 = ldg(phi, g2x + sy * g2y);
    }
    plane_tables<T, RX, RY, RM, NT>(tb, Lf, ox, oy);
    if (!run) return;   // uniform over the workgroup
    __syncthreads();

    // step 1: u1 = g f on the box
    const int lx = tx + 2;
    const C dxo = tb.Dd[0][lx];
    C fk[NP], Dk[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int ly = ty + q * PR + 2;
        C u1 = zero;
        fk[q] = Dk[q] = zero;
        if (!EDGE || (gx < nfx && f0y + ly - 2 < nfy)) {
            C gw;
            fk[q] = ccvt<T>(fr[q]);
            plane_jacobi<T>(dxo, tb.Dd[1][ly], pr[q], omega, Dk[q], gw);
            if (pre) u1 = cmul<T>(gw, fk[q]);
        }
        U[lx + RX * ly] = u1;
    }
    C fr1 = zero, D1 = zero;
    if (t1 < N1) {
        C u1 = zero;
        if (in1) {
            C gw;
            fr1 = ccvt<T>(f1);
            plane_jacobi<T>(tb.Dd[0][h1x + 2], tb.Dd[1][h1y + 2], ph1, omega, D1, gw);
            if (pre) u1 = cmul<T>(gw, fr1);
        }
        U[(h1x + 2) + RX * (h1y + 2)] = u1;
    }
    if (t2 < N2) {
        C u1 = zero;
        if (in2) {
            C D, gw;
            const C fv = ccvt<T>(f2);
            plane_jacobi<T>(tb.Dd[0][h2x + 2], tb.Dd[1][h2y + 2], ph2, omega, D, gw);
            if (pre) u1 = cmul<T>(gw, fv);
        }
        U[(h2x + 2) + RX * (h2y + 2)] = u1;
    }
    __syncthreads();

    // step 2: r = f - M u1 on the owned points and the first ring (zero
    // outside the grid)
    const C axo = tb.A[0][lx], cxo = tb.Cc[0][lx];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int ly = ty + q * PR + 2;
        const int l = lx + RX * ly;
        C res = zero;
        if (!EDGE || (gx < nfx && f0y + ly - 2 < nfy))
            res = plane_resid<T, RX>(U, l, Dk[q], fk[q], axo, cxo, tb.A[1][ly], tb.Cc[1][ly]);
        R[l] = res;
    }
    if (t1 < N1) {
        const int x = h1x + 2, y = h1y + 2, l = x + RX * y;
        C res = zero;
        if (in1) res = plane_resid<T, RX>(U, l, D1, fr1, tb.A[0][x], tb.Cc[0][x], tb.A[1][y], tb.Cc[1][y]);
        R[l] = res;
    }
    __syncthreads();

    // step 3: full weighting, x then y
    C *__restrict__ fout = Lc.f;
    const T w0 = (T)0.125, w1 = (T)0.375;
    for (int cl = threadIdx.x; cl < CX * CY; cl += NT) {
        const int ix = cl % CX, iy = cl / CX;
        const int I = c0x + ix, J = c0y + iy;
        if (I >= ncx || J >= ncy) continue;
        const int bxl = 2 * ix + 1, byl = 2 * iy + 1;
        C acc = zero;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T wy = (b == 0 || b == 3) ? w0 : w1;
            const C *row = &R[bxl + RX * (byl + b)];
            C sx = crs<T>(w0, row[0]);
            sx = crsadd<T>(sx, w1, row[1]);
            sx = crsadd<T>(sx, w1, row[2]);
            sx = crsadd<T>(sx, w0, row[3]);
            acc = b == 0 ? crs<T>(wy, sx) : crsadd<T>(acc, wy, sx);
        }
        stg(fout, I + (int64_t)ncx * J, acc);
    }
}

template <typename T, typename TF, int VT, bool ST>
__device__ __forceinline__ void vdown_plane(Ctx cx, int lev, int fsel, const void *fptr, LvPair<T> lp)
{
    constexpr int CX = TileSet<2>::X[VT], CY = TileSet<2>::Y[VT];
    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    LevelDev<T> Lf, Lc;
    int run = PH_RUN;
    if (lp.valid) {
        run = phase_of(cx, tl.prob);
        Lf = lp.f;
        Lc = lp.c;
    } else {
        if (phase_of(cx, tl.prob) != PH_RUN) return;
        const LevelDev<T> *Lv = levels_of<T>(cx, pd);
        Lf = Lv[lev];
        Lc = Lv[lev + 1];
    }
    const TF *f = lev == 0 ? (const TF *)(fptr ? fptr : pd->vec[fsel]) : (const TF *)Lf.f;
    const T omega = (T)(cx.L ? cx.omega : pd->omega);
    const bool pre = (cx.L ? cx.nu1 : pd->nu1) != 0;   // V(1,1), or V(0,1) without pre-smoothing
    const int ntx = (Lc.n[0] + CX - 1) / CX;
    const int c0x = (tl.idx % ntx) * CX, c0y = (tl.idx / ntx) * CY;
    // the fine box [2 c0x - 2, 2 c0x + 2 CX + 2) (and in y) inside the grid
    const bool edge = c0x == 0 || c0y == 0 || 2 * c0x + 2 * CX + 2 > Lf.n[0] || 2 * c0y + 2 * CY + 2 > Lf.n[1];
    __shared__ DownLds<T, PlaneDown<VT>::RN, PlaneDown<VT>::RM> sm;
    if (edge) vdown_plane_tile<T, TF, VT, true, false>(sm, Lf, Lc, f, omega, pre, c0x, c0y, run == PH_RUN);
    else vdown_plane_tile<T, TF, VT, false, ST>(sm, Lf, Lc, f, omega, pre, c0x, c0y, run == PH_RUN);
}

// 2D up-leg of the fine tile at (f0x, f0y): u2 = g f + P e on the owned
// points and the ring of one around them, then u = u2 + g (f - M u2) on the
// owned points.
template <typename T, typename TF, typename TO, int VT, bool EDGE, bool STREAM>
__device__ __forceinline__ void vup_plane_tile(UpLds<T, PlaneUp<VT>::RN, PlaneUp<VT>::EN, PlaneUp<VT>::RM> &sm,
                                               const LevelDev<T> &Lf, const LevelDev<T> &Lc, const TF *__restrict__ f,
                                               TO *__restrict__ outv, int lev, T omega, bool pre, int f0x, int f0y,
                                               bool run)
{
    using C = V2<T>;
    constexpr int CX = TileSet<2>::X[VT], CY = TileSet<2>::Y[VT], NT = TileSet<2>::T[VT];
    constexpr int FX = 2 * CX, FY = 2 * CY;
    constexpr int RX = FX + 2, RY = FY + 2, RN = RX * RY, RM = RX > RY ? RX : RY;
    constexpr int EX = CX + 4, EY = CY + 4, EN = EX * EY;
    constexpr int PR = NT / FX, NP = FY / PR;
    constexpr int NH = 2 * FX + 2 * FY + 4;
    static_assert((FX & (FX - 1)) == 0 && NT % FX == 0 && FY % PR == 0 && PR % 2 == 0 && NH <= NT, "2D up-leg tile");
    // the coarse box is loaded as rows of EXP lanes (EXP a power of two >= EX)
    constexpr int EXP = EX <= 16 ? 16 : (EX <= 32 ? 32 : 64);
    static_assert(EX <= EXP && NT % EXP == 0, "2D up-leg coarse box");
    constexpr int ER = NT / EXP, NE = (EY + ER - 1) / ER;
    static_assert(RN == PlaneUp<VT>::RN && EN == PlaneUp<VT>::EN && RM == PlaneUp<VT>::RM, "2D up-leg LDS");
    C *U = sm.U, *E = sm.E;
    PlaneTables<T, RM> &tb = sm.tb;

    const int nfx = Lf.n[0], nfy = Lf.n[1], ncx = Lc.n[0], ncy = Lc.n[1];
    const T *__restrict__ phi = Lf.phi;
    const C *__restrict__ ec = Lc.e;
    const int64_t sy = nfx;
    const int ox = f0x - 1, oy = f0y - 1;
    const int ex0 = (f0x >> 1) - 2, ey0 = (f0y >> 1) - 2;
    const int tx = threadIdx.x & (FX - 1), ty = threadIdx.x / FX;
    const int gx = f0x + tx;
    const int64_t p0 = (int64_t)(f0y + ty) * sy + gx, dq = (int64_t)PR * sy;
    const C zero = cmk<T>(0, 0);

    // loads: owned points, the ring point, the coarse box, the tables
    TF fr[NP];
    T pr[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        if (!EDGE || (gx < nfx && f0y + ty + q * PR < nfy)) {
            fr[q] = STREAM ? ldg_nt(f, p0 + q * dq) : ldg(f, p0 + q * dq);
            pr[q] = STREAM ? ldg_nt(phi, p0 + q * dq) : ldg(phi, p0 + q * dq);
        }
    }
    const bool hr = (int)threadIdx.x < NH;
    int hx = 0, hy = 0;
    if (hr) ring_point<FX, FY>(threadIdx.x, 1, hx, hy);
    const int hgx = f0x + hx, hgy = f0y + hy;
    const bool hin = hr && (!EDGE || (hgx >= 0 && hgx < nfx && hgy >= 0 && hgy < nfy));
    TF hf;
    T hph = 0;
    if (hin) {
        hf = ldg(f, hgx + sy * hgy);
        hph = ldg(phi, hgx + sy * hgy);
    }
    const int ex = threadIdx.x & (EXP - 1), ey = threadIdx.x / EXP;
    C er[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int yy = ey + q * ER, gxe = ex0 + ex, gye = ey0 + yy;
        er[q] = zero;
        if (ex < EX && yy < EY && gxe >= 0 && gxe < ncx && gye >= 0 && gye < ncy) er[q] = ldg(ec, gxe + (int64_t)ncx * gye);
    }
    plane_tables<T, RX, RY, RM, NT>(tb, Lf, ox, oy);
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int yy = ey + q * ER;
        if (ex < EX && yy < EY) E[ex + EX * yy] = er[q];
    }
    if (!run) return;   // uniform over the workgroup
    __syncthreads();

    // step 1: u2 = g f + P e.  Owned fine column gx = f0x + tx has coarse
    // neighbours (tx >> 1) + 2 and one to the side of its parity in the
    // coarse box (f0x is even); likewise in y, and PR is even, so the rows
    // of this thread keep their parity.
    const int lx = tx + 1;
    const int Ix = (tx >> 1) + 2, Iox = Ix + ((tx & 1) ? 1 : -1);
    const int Iy0 = (ty >> 1) + 2, Ioy0 = Iy0 + ((ty & 1) ? 1 : -1);
    const C dxo = tb.Dd[0][lx];
    C fk[NP], Dk[NP], gk[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int ly = ty + q * PR + 1;
        C u2 = zero;
        fk[q] = Dk[q] = gk[q] = zero;
        if (!EDGE || (gx < nfx && f0y + ly - 1 < nfy)) {
            fk[q] = ccvt<T>(fr[q]);
            plane_jacobi<T>(dxo, tb.Dd[1][ly], pr[q], omega, Dk[q], gk[q]);
            const C u1 = pre ? cmul<T>(gk[q], fk[q]) : zero;
            const C pe = plane_prolong<T, EX>(E, Ix, Iox, Iy0 + q * (PR / 2), Ioy0 + q * (PR / 2));
            u2 = cadd<T>(u1, pe);
        }
        U[lx + RX * ly] = u2;
    }
    if (hr) {
        C u2 = zero;
        if (hin) {
            C D, gw;
            const C fv = ccvt<T>(hf);
            plane_jacobi<T>(tb.Dd[0][hx + 1], tb.Dd[1][hy + 1], hph, omega, D, gw);
            const C u1 = pre ? cmul<T>(gw, fv) : zero;
            const int Jx = (hgx >> 1) - ex0, Jox = ((hgx & 1) ? (hgx >> 1) + 1 : (hgx >> 1) - 1) - ex0;
            const int Jy = (hgy >> 1) - ey0, Joy = ((hgy & 1) ? (hgy >> 1) + 1 : (hgy >> 1) - 1) - ey0;
            u2 = cadd<T>(u1, plane_prolong<T, EX>(E, Jx, Jox, Jy, Joy));
        }
        U[(hx + 1) + RX * (hy + 1)] = u2;
    }
    __syncthreads();

    // step 2: post-smoothing of the owned points
    const C axo = tb.A[0][lx], cxo = tb.Cc[0][lx];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int ly = ty + q * PR + 1;
        if (EDGE && (gx >= nfx || f0y + ly - 1 >= nfy)) continue;
        const int l = lx + RX * ly;
        const C r = plane_resid<T, RX>(U, l, Dk[q], fk[q], axo, cxo, tb.A[1][ly], tb.Cc[1][ly]);
        const C u = cmadd<T>(U[l], gk[q], r);
        if (lev == 0) {
            TO o;
            o.x = u.x;
            o.y = u.y;
            if (STREAM) stg_nt(outv, p0 + q * dq, o);
            else stg(outv, p0 + q * dq, o);
        } else {
            stg(Lf.e, p0 + q * dq, u);
        }
    }
}

template <typename T, typename TF, typename TO, int VT, bool ST>
__device__ __forceinline__ void vup_plane(Ctx cx, int lev, int fsel, int osel, const void *fptr, void *optr, LvPair<T> lp)
{
    constexpr int FX = 2 * TileSet<2>::X[VT], FY = 2 * TileSet<2>::Y[VT];
    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    LevelDev<T> Lf, Lc;
    int run = PH_RUN;
    if (lp.valid) {
        run = phase_of(cx, tl.prob);
        Lf = lp.f;
        Lc = lp.c;
    } else {
        if (phase_of(cx, tl.prob) != PH_RUN) return;
        const LevelDev<T> *Lv = levels_of<T>(cx, pd);
        Lf = Lv[lev];
        Lc = Lv[lev + 1];
    }
    const TF *f = lev == 0 ? (const TF *)(fptr ? fptr : pd->vec[fsel]) : (const TF *)Lf.f;
    TO *outv = lev == 0 ? (TO *)(optr ? optr : pd->vec[osel]) : nullptr;
    const T omega = (T)(cx.L ? cx.omega : pd->omega);
    const bool pre = (cx.L ? cx.nu1 : pd->nu1) != 0;   // V(1,1), or V(0,1) without pre-smoothing
    const int ntx = (Lf.n[0] + FX - 1) / FX;
    const int f0x = (tl.idx % ntx) * FX, f0y = (tl.idx / ntx) * FY;
    // the fine box [f0x - 1, f0x + FX + 1) (and in y) inside the grid
    const bool edge = f0x == 0 || f0y == 0 || f0x + FX + 1 > Lf.n[0] || f0y + FY + 1 > Lf.n[1];
    __shared__ UpLds<T, PlaneUp<VT>::RN, PlaneUp<VT>::EN, PlaneUp<VT>::RM> sm;
    if (edge) vup_plane_tile<T, TF, TO, VT, true, false>(sm, Lf, Lc, f, outv, lev, omega, pre, f0x, f0y, run == PH_RUN);
    else vup_plane_tile<T, TF, TO, VT, false, ST>(sm, Lf, Lc, f, outv, lev, omega, pre, f0x, f0y, run == PH_RUN);
}

// The fused legs: the plane form in 2D, the box form in 3D.  ST: the 2D
// interior tiles stream their per-point inputs and the finest output with
// non-temporal accesses (the host takes it for levels of at least
// HH_STREAM_MIN points).
template <int DIM, typename T, typename TF, int VT, bool ST = false>
__global__ __launch_bounds__(TileSet<DIM>::T[VT]) void k_vdown(Ctx cx, int lev, int fsel, const void *fptr, LvPair<T> lp)
{
    if constexpr (DIM == 2) vdown_plane<T, TF, VT, ST>(cx, lev, fsel, fptr, lp);
    else vdown_box<DIM, T, TF, VT>(cx, lev, fsel, fptr, lp);
}
template <int DIM, typename T, typename TF, typename TO, int VT, bool ST = false>
__global__ __launch_bounds__(TileSet<DIM>::T[VT]) void k_vup(Ctx cx, int lev, int fsel, int osel, const void *fptr, void *optr,
                                                LvPair<T> lp)
{
    if constexpr (DIM == 2) vup_plane<T, TF, TO, VT, ST>(cx, lev, fsel, osel, fptr, optr, lp);
    else vup_box<DIM, T, TF, TO, VT>(cx, lev, fsel, osel, fptr, optr, lp);
}

// ---------------------------------------------------------------------------
// Fused legs of a Galerkin level l >= 1 (2D): the level's operator is its
// stored 25-point stencil G (entry s = (dx+2) + 5(dy+2) of point p at s*N + p,
// the matrix entry M[p, p + dx + nx*dy]), applied as G_12 u_p and then + G_s u_q
// for s ascending, s != 12, with u = 0 outside the grid; the Jacobi weight is
// taken from G_12.  Transfers and the order of every other operation are those
// of the rediscretised legs.  One problem; descriptors by value.
// ---------------------------------------------------------------------------
template <typename T> struct GalArgs {
    const V2<T> *G;      // stencil of the leg's fine level
    const V2<T> *f;      // f of the fine level
    V2<T> *e;            // up-leg output: e of the fine level
    V2<T> *fc;           // down-leg output: f of the coarse level
    const V2<T> *ec;     // up-leg input: e of the coarse level
    int nfx, nfy, ncx, ncy;
    T omega;
    int pre;             // pre-smoothing (V(1,1)) or none (V(0,1))
};
constexpr int GAL_C = 16;    // down-leg: coarse tile side; up-leg: fine tile side 2 GAL_C
constexpr int GAL_NT = 256;

// Down-leg: u1 = g f on the fine box (the owned 2C x 2C cells and a ring of
// three: the residual's stencil reaches two cells beyond the restriction's
// footprint), r = f - G u1 on the footprint (owned cells and a ring of one),
// full weighting onto the C x C coarse tile.
template <typename T>
__global__ __launch_bounds__(GAL_NT) void k_gdown(Ctx cx, GalArgs<T> ga)
{
    using C = V2<T>;
    constexpr int FX = 2 * GAL_C, BX = FX + 6, RX = FX + 2;   // u1 box, residual box
    __shared__ C U[BX * BX];
    __shared__ C R[RX * RX];
    if (phase_of(cx, 0) != PH_RUN) return;
    const int nfx = ga.nfx, nfy = ga.nfy;
    const int tiles_x = (ga.ncx + GAL_C - 1) / GAL_C;
    const int c0x = (blockIdx.x % tiles_x) * GAL_C, c0y = (blockIdx.x / tiles_x) * GAL_C;
    const int f0x = 2 * c0x, f0y = 2 * c0y;
    const int64_t N = (int64_t)nfx * nfy;
    const C zero = cmk<T>(0, 0);
    for (int l = threadIdx.x; l < BX * BX; l += GAL_NT) {
        const int gx = f0x - 3 + l % BX, gy = f0y - 3 + l / BX;
        C u1 = zero;
        if (ga.pre && gx >= 0 && gx < nfx && gy >= 0 && gy < nfy) {
            const int64_t p = gx + (int64_t)nfx * gy;
            u1 = cmul<T>(jweight<T>(ldg(ga.G, 12 * N + p), ga.omega), ldg(ga.f, p));
        }
        U[l] = u1;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < RX * RX; l += GAL_NT) {
        const int rx = l % RX, ry = l / RX;
        const int gx = f0x - 1 + rx, gy = f0y - 1 + ry;
        C res = zero;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy) {
            const int64_t p = gx + (int64_t)nfx * gy;
            const int c = (rx + 2) + BX * (ry + 2);
            C mu = cmul<T>(ldg(ga.G, 12 * N + p), U[c]);
#pragma unroll
            for (int s = 0; s < 25; ++s) {
                if (s == 12) continue;
                mu = cmadd<T>(mu, ldg(ga.G, s * N + p), U[c + (s % 5 - 2) + BX * (s / 5 - 2)]);
            }
            res = csub<T>(ldg(ga.f, p), mu);
        }
        R[l] = res;
    }
    __syncthreads();
    const T w0 = (T)0.125, w1 = (T)0.375;
    for (int cl = threadIdx.x; cl < GAL_C * GAL_C; cl += GAL_NT) {
        const int ix = cl % GAL_C, iy = cl / GAL_C;
        const int I = c0x + ix, J = c0y + iy;
        if (I >= ga.ncx || J >= ga.ncy) continue;
        C acc = zero;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T wy = (b == 0 || b == 3) ? w0 : w1;
            const C *row = &R[2 * ix + RX * (2 * iy + b)];
            C sx = crs<T>(w0, row[0]);
            sx = crsadd<T>(sx, w1, row[1]);
            sx = crsadd<T>(sx, w1, row[2]);
            sx = crsadd<T>(sx, w0, row[3]);
            acc = b == 0 ? crs<T>(wy, sx) : crsadd<T>(acc, wy, sx);
        }
        stg(ga.fc, I + (int64_t)ga.ncx * J, acc);
    }
}

// Up-leg: u2 = g f + P e on the owned 2C x 2C fine cells and a ring of two
// (the stencil's reach), then u = u2 + g (f - G u2) on the owned cells.
template <typename T>
__global__ __launch_bounds__(GAL_NT) void k_gup(Ctx cx, GalArgs<T> ga)
{
    using C = V2<T>;
    constexpr int FX = 2 * GAL_C, BX = FX + 4, EX = GAL_C + 4;   // u2 box, coarse box
    __shared__ C U[BX * BX];
    __shared__ C E[EX * EX];
    if (phase_of(cx, 0) != PH_RUN) return;
    const int nfx = ga.nfx, nfy = ga.nfy;
    const int tiles_x = (nfx + FX - 1) / FX;
    const int f0x = (blockIdx.x % tiles_x) * FX, f0y = (blockIdx.x / tiles_x) * FX;
    const int ex0 = (f0x >> 1) - 2, ey0 = (f0y >> 1) - 2;
    const int64_t N = (int64_t)nfx * nfy;
    const C zero = cmk<T>(0, 0);
    for (int l = threadIdx.x; l < EX * EX; l += GAL_NT) {
        const int gx = ex0 + l % EX, gy = ey0 + l / EX;
        E[l] = (gx >= 0 && gx < ga.ncx && gy >= 0 && gy < ga.ncy) ? ldg(ga.ec, gx + (int64_t)ga.ncx * gy) : zero;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < BX * BX; l += GAL_NT) {
        const int gx = f0x - 2 + l % BX, gy = f0y - 2 + l / BX;
        C u2 = zero;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy) {
            const int64_t p = gx + (int64_t)nfx * gy;
            const C fv = ldg(ga.f, p);
            const C u1 = ga.pre ? cmul<T>(jweight<T>(ldg(ga.G, 12 * N + p), ga.omega), fv) : zero;
            const int Ix = (gx >> 1) - ex0, Iox = ((gx & 1) ? (gx >> 1) + 1 : (gx >> 1) - 1) - ex0;
            const int Iy = (gy >> 1) - ey0, Ioy = ((gy & 1) ? (gy >> 1) + 1 : (gy >> 1) - 1) - ey0;
            u2 = cadd<T>(u1, plane_prolong<T, EX>(E, Ix, Iox, Iy, Ioy));
        }
        U[l] = u2;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < FX * FX; l += GAL_NT) {
        const int gx = f0x + l % FX, gy = f0y + l / FX;
        if (gx >= nfx || gy >= nfy) continue;
        const int64_t p = gx + (int64_t)nfx * gy;
        const int c = (l % FX + 2) + BX * (l / FX + 2);
        const C D = ldg(ga.G, 12 * N + p);
        C mu = cmul<T>(D, U[c]);
#pragma unroll
        for (int s = 0; s < 25; ++s) {
            if (s == 12) continue;
            mu = cmadd<T>(mu, ldg(ga.G, s * N + p), U[c + (s % 5 - 2) + BX * (s / 5 - 2)]);
        }
        stg(ga.e, p, cmadd<T>(U[c], jweight<T>(D, ga.omega), csub<T>(ldg(ga.f, p), mu)));
    }
}

// ---------------------------------------------------------------------------
// ILU(0) up-leg (2D, FP64): the paper's smoother (Sec. 6.1) in its V(0,1)
// cycle.  Level l's up-leg is u = P e_{l+1} (no pre-smoothing: the down-legs
// only restrict), then one sweep u = u + omega (L U)^-1 (f - M u) with the
// level's ILU(0) factors (lexicographic order, set up on the host).  The
// triangular solves are the exact lexicographic ones: point (i, j) depends
// on its stencil neighbours below (resp. above) the diagonal only, so the
// anti-diagonals d = i + m j (m = 1 for the 5-point set, whose lower
// neighbours are (i-1, j) and (i, j-1); m = 3 for the 25-point set, whose
// lower neighbours reach (i+2, j-1) and (i-2, j)) are sets of independent
// points, taken in order with a barrier between them.  That is n_x + m n_y
// dependent steps per solve, so one workgroup runs the level and the leg is
// latency-bound by construction; every per-point operation is the oracle's,
// in its order.  Every side of a smoothing level has at least 5 cells (the
// 25-point offsets are then in column order).
// ---------------------------------------------------------------------------
#define HH_ILU_WG 1024
// the pointwise phases (prolongation, residual, update) of a level with more
// points than this run as grid-wide launches of HH_ILU_PW threads per
// workgroup: in one workgroup they would take N / 1024 dependent load
// round trips per thread
#define HH_ILU_PW 256
#define HH_ILU_INNER_MAX (int64_t(1) << 10)
struct IluArgs {
    LevelDev<double> fl, cl;          // level l and the coarser level l + 1
    const double2 *f;                 // right-hand side of level l (the cycle's input on level 0)
    double2 *u;                       // result of level l (e_l, or the cycle's output on level 0)
    double omega;                     // relaxation of the ILU(0) update
    int inner;                        // 1: the sweep kernel runs the pointwise phases too;
                                      // 0: k_ilu_prolong, k_ilu_resid, k_ilu_update run them
    int diag;                         // 1: w in the row form's step order (IluLayout position
                                      // dd TS + t of each point); 0: w by point
};

// entry s (offset (s % 5 - 2, s / 5 - 2)) of row p of M_l applied to u, with
// the neighbour outside the grid taken as zero: the Galerkin stencil, or the
// 5-point set of the rediscretised stencil; y = M u in the contract's order
__device__ __forceinline__ double2 ilu_Mu(const LevelDev<double> &L, const double2 *u, int i, int j, int64_t p)
{
    const int nx = L.n[0], ny = L.n[1];
    const double2 zero = cmk<double>(0.0, 0.0);
    if (L.g) {
        const int64_t N = L.N;
        double2 t = cmul<double>(ldg(L.g, 12 * N + p), ldg(u, p));
        for (int s = 0; s < 25; ++s) {
            if (s == 12) continue;
            const int ii = i + s % 5 - 2, jj = j + s / 5 - 2;
            const double2 uq = (ii >= 0 && ii < nx && jj >= 0 && jj < ny) ? ldg(u, ii + (int64_t)nx * jj) : zero;
            t = cadd<double>(t, cmul<double>(ldg(L.g, s * N + p), uq));
        }
        return t;
    }
    double2 d = cadd<double>(ldg(L.d[0], i), ldg(L.d[1], j));
    const double2 D = cmk<double>(d.x - ldg(L.phi, p), d.y);
    double2 t = cmul<double>(D, ldg(u, p));
    t = csub<double>(t, cmul<double>(ldg(L.a[0], i), i > 0 ? ldg(u, p - 1) : zero));
    t = csub<double>(t, cmul<double>(ldg(L.c[0], i), i < nx - 1 ? ldg(u, p + 1) : zero));
    t = csub<double>(t, cmul<double>(ldg(L.a[1], j), j > 0 ? ldg(u, p - nx) : zero));
    t = csub<double>(t, cmul<double>(ldg(L.c[1], j), j < ny - 1 ? ldg(u, p + nx) : zero));
    return t;
}

// The entry sets of the triangular solves (NLO entries on each side of the
// diagonal), the anti-diagonal step m, and the workgroup size NT of the row
// form (k_ilu_up_rows) for the 25-point (Galerkin) and the 5-point stencils.
template <bool GAL> struct IluSet;
template <> struct IluSet<true> {
    static constexpr int M = 3, NLO = 12, NT = 512, RING = 9, HR = 2, HMAX = 2048, PF = 3;
    __host__ __device__ static constexpr int lo(int k) { return k; }          // s = 0 .. 11
    __host__ __device__ static constexpr int up(int k) { return 13 + k; }     // s = 13 .. 24
};
template <> struct IluSet<false> {
    static constexpr int M = 1, NLO = 2, NT = 1024, RING = 2, HR = 1, HMAX = 4096, PF = 4;
    __host__ __device__ static constexpr int lo(int k) { return k == 0 ? 7 : 11; }
    __host__ __device__ static constexpr int up(int k) { return k == 0 ? 13 : 17; }
};

// Device layout of a level's ILU(0) factors, in the order the row form reads
// them.  Where nx <= m NT all rows form one band, thread t solving rows t,
// t + NT, ... (a row ends before the one NT below it starts); otherwise the
// rows are split into nb bands of at most NT rows (sizes base or base + 1,
// the first `extra` bands the larger).  Row offset r of band b is solved by
// thread lane(r) = r mod NT, point (i, j0(b) + r) at the band's step d = i +
// m r, and the bands' steps are numbered on from one band to the next
// (global step dd = d0(b) + d).  The entries of one step are stored
// lane-contiguous: entry k of lane t at (dd NLO + k) TS + t for the lower
// set, and the diagonal (k = 0) and upper entries (k = 1 .. NLO) at (DT NLO
// + dd (NLO + 1) + k) TS + t, where TS is the largest band rounded up to 64
// lanes (at most NT) and DT the total step count; positions without a point,
// and the entries of a point's neighbours outside the grid, are +0.  A wave's loads of one
// entry are then one contiguous 1 KB block.
template <bool GAL> struct IluLayout {
    using S = IluSet<GAL>;
    int nx, ny, nb, base, extra, TS;
    int64_t DT;
    __host__ __device__ IluLayout(int nx_, int ny_) : nx(nx_), ny(ny_)
    {
        // one band when a thread finishes a row before the row NT below it
        // starts (nx <= m NT): thread t then owns rows t, t + NT, ...
        nb = nx <= S::M * S::NT ? 1 : (ny + S::NT - 1) / S::NT;
        base = ny / nb;
        extra = ny % nb;
        const int rmax = base + (extra > 0 ? 1 : 0);
        TS = rmax > S::NT ? S::NT : (rmax + 63) / 64 * 64;
        DT = (int64_t)nb * (nx - S::M) + (int64_t)S::M * ny;
    }
    // lane of row offset r within its band
    __host__ __device__ static int lane(int r) { return r % S::NT; }
    __host__ __device__ int j0(int b) const { return b * base + (b < extra ? b : extra); }
    __host__ __device__ int band_of(int j) const
    {
        const int c = extra * (base + 1);
        return j < c ? j / (base + 1) : extra + (j - c) / base;
    }
    // steps of the bands before b: sum of (nx - 1) + m (R - 1) + 1
    __host__ __device__ int64_t d0(int b) const { return (int64_t)b * (nx - S::M) + (int64_t)S::M * j0(b); }
    __host__ __device__ int64_t lo(int64_t dd, int k, int t) const { return (dd * S::NLO + k) * TS + t; }
    __host__ __device__ int64_t up(int64_t dd, int k, int t) const { return (DT * S::NLO + dd * (S::NLO + 1) + k) * TS + t; }
    __host__ __device__ int64_t size() const { return DT * (2 * S::NLO + 1) * TS; }
};

// position of point p in w: p, or with the row form the point's layout
// position (the level's set: the 25-point one on Galerkin levels)
__device__ __forceinline__ int64_t ilu_wpos(const IluArgs &a, int64_t p)
{
    if (!a.diag) return p;
    const int nx = a.fl.n[0], ny = a.fl.n[1];
    const int i = (int)(p % nx), j = (int)(p / nx);
    if (a.fl.g) {
        const IluLayout<true> lay(nx, ny);
        const int b = lay.band_of(j), r = j - lay.j0(b);
        return (lay.d0(b) + i + 3 * r) * lay.TS + lay.lane(r);
    }
    const IluLayout<false> lay(nx, ny);
    const int b = lay.band_of(j), r = j - lay.j0(b);
    return (lay.d0(b) + i + r) * lay.TS + lay.lane(r);
}

// the pointwise phases of the up-leg at point p: u = 0 + P e_{l+1} (bilinear,
// x then y; coarse values outside are zero), r = f - M u (into w, once every
// u is written), and after the solves u = u + omega z
__device__ __forceinline__ void ilu_prolong_at(const IluArgs &a, int64_t p)
{
    const int nx = a.fl.n[0], ncx = a.cl.n[0], ncy = a.cl.n[1];
    const double2 *__restrict__ ec = a.cl.e;
    const double2 zero = cmk<double>(0.0, 0.0);
    const int i = (int)(p % nx), j = (int)(p / nx);
    const int Ix = i >> 1, Iox = (i & 1) ? Ix + 1 : Ix - 1;
    const int Iy = j >> 1, Ioy = (j & 1) ? Iy + 1 : Iy - 1;
    auto ev = [&](int x, int y) -> double2 {
        return (x >= 0 && x < ncx && y >= 0 && y < ncy) ? ldg(ec, x + (int64_t)ncx * y) : zero;
    };
    const double2 a0 = crs2<double>(0.75, ev(Ix, Iy), 0.25, ev(Iox, Iy));
    const double2 a1 = crs2<double>(0.75, ev(Ix, Ioy), 0.25, ev(Iox, Ioy));
    stg(a.u, p, cadd<double>(zero, crs2<double>(0.75, a0, 0.25, a1)));
}
__device__ __forceinline__ void ilu_resid_at(const IluArgs &a, int64_t p)
{
    const int nx = a.fl.n[0];
    const int i = (int)(p % nx), j = (int)(p / nx);
    stg(a.fl.w, ilu_wpos(a, p), csub<double>(ldg(a.f, p), ilu_Mu(a.fl, a.u, i, j, p)));
}
__device__ __forceinline__ void ilu_update_at(const IluArgs &a, int64_t p)
{
    stg(a.u, p, crsadd<double>(ldg(a.u, p), a.omega, ldg(a.fl.w, ilu_wpos(a, p))));
}

// the pointwise phases as grid-wide launches, for levels whose points are
// too many for one workgroup's loops (same values: one point per thread)
__global__ __launch_bounds__(HH_ILU_PW) void k_ilu_prolong(Ctx cx, IluArgs a)
{
    if (phase_of(cx, 0) != PH_RUN) return;
    const int64_t p = blockIdx.x * (int64_t)HH_ILU_PW + threadIdx.x;
    if (p < a.fl.N) ilu_prolong_at(a, p);
}
__global__ __launch_bounds__(HH_ILU_PW) void k_ilu_resid(Ctx cx, IluArgs a)
{
    if (phase_of(cx, 0) != PH_RUN) return;
    const int64_t p = blockIdx.x * (int64_t)HH_ILU_PW + threadIdx.x;
    if (p < a.fl.N) ilu_resid_at(a, p);
}
__global__ __launch_bounds__(HH_ILU_PW) void k_ilu_update(Ctx cx, IluArgs a)
{
    if (phase_of(cx, 0) != PH_RUN) return;
    const int64_t p = blockIdx.x * (int64_t)HH_ILU_PW + threadIdx.x;
    if (p < a.fl.N) ilu_update_at(a, p);
}

__global__ __launch_bounds__(HH_ILU_WG) void k_ilu_up(Ctx cx, IluArgs a)
{
    if (phase_of(cx, 0) != PH_RUN) return;
    const LevelDev<double> L = a.fl;
    const int nx = L.n[0], ny = L.n[1];
    const int64_t N = L.N;
    const double2 *__restrict__ F = L.ilu;
    double2 *w = L.w;
    const bool gal = L.g != nullptr;
    const int tid = threadIdx.x;
    if (a.inner) {
        for (int64_t p = tid; p < N; p += HH_ILU_WG) ilu_prolong_at(a, p);
        __syncthreads();
        for (int64_t p = tid; p < N; p += HH_ILU_WG) ilu_resid_at(a, p);
        __syncthreads();
    }
    const int m = gal ? 3 : 1;
    const int nd = (nx - 1) + m * (ny - 1) + 1;
    const IluLayout<true> lg(nx, ny);
    const IluLayout<false> l5(nx, ny);
    // the layout position (global step, thread) of point (i, j)
    auto pos = [&](int i, int j, int64_t &dd, int &t) {
        if (gal) {
            const int b = lg.band_of(j), r = j - lg.j0(b);
            t = lg.lane(r);
            dd = lg.d0(b) + i + 3 * r;
        } else {
            const int b = l5.band_of(j), r = j - l5.j0(b);
            t = l5.lane(r);
            dd = l5.d0(b) + i + r;
        }
    };
    // forward: y = r - sum of l_s y_q over the neighbours below, columns ascending
    for (int d = 0; d < nd; ++d) {
        const int jlo = d - (nx - 1) > 0 ? (d - (nx - 1) + m - 1) / m : 0, jhi = min(ny - 1, d / m);
        for (int j = jlo + tid; j <= jhi; j += HH_ILU_WG) {
            const int i = d - m * j;
            const int64_t p = i + (int64_t)nx * j;
            int64_t dd;
            int t;
            pos(i, j, dd, t);
            double2 y = ldg(w, p);
            if (gal) {
                for (int s = 0; s < 12; ++s) {
                    const int ii = i + s % 5 - 2, jj = j + s / 5 - 2;
                    if (ii >= 0 && ii < nx && jj >= 0) y = csub<double>(y, cmul<double>(ldg(F, lg.lo(dd, s, t)), ldg(w, ii + (int64_t)nx * jj)));
                }
            } else {
                if (j > 0) y = csub<double>(y, cmul<double>(ldg(F, l5.lo(dd, 0, t)), ldg(w, p - nx)));
                if (i > 0) y = csub<double>(y, cmul<double>(ldg(F, l5.lo(dd, 1, t)), ldg(w, p - 1)));
            }
            stg(w, p, y);
        }
        __syncthreads();
    }
    // backward: z = (y - sum of u_s z_c over the neighbours above, columns ascending) / u_12
    for (int d = nd - 1; d >= 0; --d) {
        const int jlo = d - (nx - 1) > 0 ? (d - (nx - 1) + m - 1) / m : 0, jhi = min(ny - 1, d / m);
        for (int j = jlo + tid; j <= jhi; j += HH_ILU_WG) {
            const int i = d - m * j;
            const int64_t p = i + (int64_t)nx * j;
            int64_t dd;
            int t;
            pos(i, j, dd, t);
            double2 z = ldg(w, p);
            if (gal) {
                for (int s = 13; s < 25; ++s) {
                    const int ii = i + s % 5 - 2, jj = j + s / 5 - 2;
                    if (ii >= 0 && ii < nx && jj < ny) z = csub<double>(z, cmul<double>(ldg(F, lg.up(dd, 1 + (s - 13), t)), ldg(w, ii + (int64_t)nx * jj)));
                }
                stg(w, p, cdiv<double>(z, ldg(F, lg.up(dd, 0, t))));
            } else {
                if (i < nx - 1) z = csub<double>(z, cmul<double>(ldg(F, l5.up(dd, 1, t)), ldg(w, p + 1)));
                if (j < ny - 1) z = csub<double>(z, cmul<double>(ldg(F, l5.up(dd, 2, t)), ldg(w, p + nx)));
                stg(w, p, cdiv<double>(z, ldg(F, l5.up(dd, 0, t))));
            }
        }
        __syncthreads();
    }
    if (a.inner)
        for (int64_t p = tid; p < N; p += HH_ILU_WG) ilu_update_at(a, p);
}

// The same up-leg with the triangular solves in the pipelined row form
// (NT = 1024 threads for the 5-point set; 512 for the 25-point one, whose
// 2 x 12 factors in flight need the registers of a 512-thread workgroup).
// Thread t owns row t, and on anti-diagonal d it solves point (d - m t, t),
// so its points come left to right (right to left in the backward solve) one
// step after another.  A level of more rows than threads runs as one pass
// with thread t owning rows t, t + NT, ... where a row ends before the row NT
// below it starts (nx <= m NT), and otherwise in bands of at most NT rows.
// The values of the last RING diagonals sit in LDS (slot d mod RING, entry
// lane t of the thread that solved the point): the neighbours below a point
// lie on the 8 diagonals before it (m = 3) or the one before (m = 1), in the
// same or the two lanes before (wrapping from lane 0 to NT - 1 in the one
// pass), and those above on as many after it, so no neighbour value is read
// from global memory, and a slot is rewritten only after every read of its
// previous diagonal.  Bands run one after
// another (bottom up forward, top down backward); the rows a band reads from
// the band before it (two with m = 3, one with m = 1) are kept in an LDS halo
// by column, each entry rewritten by the band's own boundary rows only after
// its last read (bands have at least 3 rows).  The factors and the
// right-hand side of a thread's points are loaded PF steps before they are
// needed (3 with m = 3, 4 with m = 1), behind the barriers of the steps in
// between.  Values and operation order are k_ilu_up's.
template <bool GAL, int NT, bool MULTI>
__global__ __launch_bounds__(NT) void k_ilu_up_rows(Ctx cx, IluArgs a)
{
    using S = IluSet<GAL>;
    // NT below the layout's S::NT serves levels of at most NT rows (one band,
    // whose layout does not depend on the workgroup size); MULTI (one band of
    // more rows than threads) needs the layout's NT
    static_assert(NT <= S::NT && NT % 64 == 0 && (!MULTI || NT == S::NT), "the factor layout's workgroup size");
    constexpr int M = S::M, NK = S::NLO, RG = S::RING, HR = S::HR, HM = S::HMAX;
    // the ring of the last RG diagonals (slot d mod RG, entry t), then the
    // halo, then one entry holding +0 (the value of a neighbour outside the
    // grid)
    __shared__ double2 lds[RG * NT + HR * HM + 1];
    constexpr int HB = RG * NT, Z0 = RG * NT + HR * HM;
    if (phase_of(cx, 0) != PH_RUN) return;
    const LevelDev<double> L = a.fl;
    const int nx = L.n[0], ny = L.n[1];
    const int64_t N = L.N;
    const double2 *__restrict__ F = L.ilu;
    double2 *w = L.w;
    const double2 zero = cmk<double>(0.0, 0.0);
    const int t = threadIdx.x;
    if (t == 0) lds[Z0] = zero;
    if (a.inner) {
        for (int64_t p = t; p < N; p += NT) ilu_prolong_at(a, p);
        __syncthreads();
        for (int64_t p = t; p < N; p += NT) ilu_resid_at(a, p);
    }
    __syncthreads();
    // nb bands of ny / nb or ny / nb + 1 rows (the layout's); the halo is used
    // (and nx <= HM holds) only when nb > 1
    const IluLayout<GAL> lay(nx, ny);
    const int nb = lay.nb;
    const bool banded = nb > 1;
    auto band0 = [&](int bi) { return lay.j0(bi); };
    auto slot = [&](int d, int tt) -> int { return (d % RG) * NT + tt; };
    // the factors and the right-hand side (and, backward, the diagonal) of
    // a thread's points are prefetched PF steps ahead into PF buffers with
    // fixed roles: step d uses buffer d mod PF, and refills it with the point
    // the thread solves at step d + PF.  Every thread loads on every step, a
    // thread without a point there (before its row's first point, after its
    // last, or beyond the band) from point 0 and layout position 0, so the
    // same number of loads follows each refill on every path and the wait
    // before a use is for that buffer's loads only, while idle lanes add one
    // cache line per load; the active lanes of a wave read lane-contiguous
    // factors (IluLayout); a factor of a neighbour outside the grid is loaded
    // but never used.  The loops start PF steps early (loads only), so no
    // buffer needs filling before them.
    constexpr int PF = S::PF, G = GAL ? 4 : 2;   // G divides NK
    double2 fq[PF][NK], rq[PF], dq[PF];
    auto fetch = [&](bool act, int64_t dd, bool lower, double2(&fv)[NK], double2 &rv, double2 &dv) {
        const int64_t dc = act ? dd : 0;
        const int tc = act ? t : 0;
        rv = ldg(w, dc * lay.TS + tc);
        if (lower) {
#pragma unroll
            for (int k = 0; k < NK; ++k) fv[k] = ldg(F, lay.lo(dc, k, tc));
        } else {
            dv = ldg(F, lay.up(dc, 0, tc));
#pragma unroll
            for (int k = 0; k < NK; ++k) fv[k] = ldg(F, lay.up(dc, 1 + k, tc));
        }
    };
    // forward: y = r - sum over the neighbours below, columns ascending
    for (int bi = 0; bi < nb; ++bi) {
        const int j0 = band0(bi), R = band0(bi + 1) - j0;
        const int nd = (nx - 1) + M * (R - 1) + 1;
        const int64_t D0 = lay.d0(bi);
        // the row offset r and column i the thread solves at step d: row t,
        // or with more rows than threads (MULTI: one band, nx <= M NT) the
        // row t + k NT whose steps contain d
        auto locate = [&](int d, int &r, int &i) -> bool {
            const int q = d - M * t;
            const int k = MULTI && q >= 0 ? q / (M * NT) : 0;
            r = t + k * NT;
            i = q - k * (M * NT);
            return r < R && i >= 0 && i < nx;
        };
        auto fwd = [&](int d, double2(&fv)[NK], double2 &rv, double2 &dv) {
            int r, i;
            if (locate(d, r, i)) {
                const int j = j0 + r;
                // the neighbour values are read G at a time, then their terms
                // are taken in order; for a neighbour outside the grid both
                // factors are +0 (the layout stores its entry as +0, and it
                // reads the +0 entry of LDS), and subtracting their product
                // (+0, +0) leaves y as it is
                double2 y = rv;
#pragma unroll
                for (int g = 0; g < NK; g += G) {
                    double2 q[G];
                    bool in[G];
                    int ix[G];
#pragma unroll
                    for (int k = g; k < g + G; ++k) {
                        const int sk = S::lo(k), dx = sk % 5 - 2, dy = sk / 5 - 2;
                        in[k - g] = i + dx >= 0 && i + dx < nx && j + dy >= 0;
                        const int ir = ((d + dx + M * dy + RG) % RG) * NT + (MULTI ? (t + dy + NT) % NT : t + dy);
                        const int ih = HB + (HR + r + dy) * HM + i + dx;
                        ix[k - g] = in[k - g] ? (dy >= 0 || r + dy >= 0 ? ir : ih) : Z0;
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) q[k] = lds[ix[k]];
#pragma unroll
                    for (int k = g; k < g + G; ++k) y = csub<double>(y, cmul<double>(fv[k], q[k - g]));
                }
                lds[slot(d, t)] = y;
                if (banded && r >= R - HR) lds[HB + (r - (R - HR)) * HM + i] = y;
                stg(w, (D0 + d) * lay.TS + t, y);
            }
            int rn, in_;
            const bool an = locate(d + PF, rn, in_);
            fetch(an, D0 + d + PF, true, fv, rv, dv);
            __syncthreads();
        };
        for (int d0 = -PF; d0 < nd; d0 += PF) {
#pragma unroll
            for (int b = 0; b < PF; ++b) fwd(d0 + b, fq[b], rq[b], dq[b]);
        }
    }
    // backward: z = (y - sum over the neighbours above, columns ascending) / u_12
    for (int bi = nb - 1; bi >= 0; --bi) {
        const int j0 = band0(bi), R = band0(bi + 1) - j0;
        const int nd = (nx - 1) + M * (R - 1) + 1;
        const int64_t D0 = lay.d0(bi);
        auto locate = [&](int d, int &r, int &i) -> bool {
            const int q = d - M * t;
            const int k = MULTI && q >= 0 ? q / (M * NT) : 0;
            r = t + k * NT;
            i = q - k * (M * NT);
            return r < R && i >= 0 && i < nx;
        };
        auto bwd = [&](int d, double2(&fv)[NK], double2 &rv, double2 &dv) {
            int r, i;
            if (locate(d, r, i)) {
                const int j = j0 + r;
                double2 z = rv;
#pragma unroll
                for (int g = 0; g < NK; g += G) {
                    double2 q[G];
                    bool in[G];
                    int ix[G];
#pragma unroll
                    for (int k = g; k < g + G; ++k) {
                        const int sk = S::up(k), dx = sk % 5 - 2, dy = sk / 5 - 2;
                        in[k - g] = i + dx >= 0 && i + dx < nx && j + dy < ny;
                        const int ir = ((d + dx + M * dy) % RG) * NT + (MULTI ? (t + dy) % NT : t + dy);
                        const int ih = HB + (r + dy - R) * HM + i + dx;
                        ix[k - g] = in[k - g] ? (dy <= 0 || r + dy < R ? ir : ih) : Z0;
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k) q[k] = lds[ix[k]];
#pragma unroll
                    for (int k = g; k < g + G; ++k) z = csub<double>(z, cmul<double>(fv[k], q[k - g]));
                }
                z = cdiv<double>(z, dv);
                lds[slot(d, t)] = z;
                if (banded && r < HR) lds[HB + r * HM + i] = z;
                stg(w, (D0 + d) * lay.TS + t, z);
            }
            int rn, in_;
            const bool an = locate(d - PF, rn, in_);
            fetch(an, D0 + d - PF, false, fv, rv, dv);
            __syncthreads();
        };
        // the first block (from nd rounded up to a multiple of PF) only loads
        for (int d0 = (nd + PF - 1) / PF * PF; d0 >= 0; d0 -= PF) {
#pragma unroll
            for (int b = PF - 1; b >= 0; --b) bwd(d0 + b, fq[b], rq[b], dq[b]);
        }
    }
    if (a.inner)
        for (int64_t p = t; p < N; p += NT) ilu_update_at(a, p);
}

// ---------------------------------------------------------------------------
// Merged 2D legs of K consecutive coarse levels lev0 .. lev0 + K - 1 (ending
// at the tail's first level lev0 + K), one launch per leg instead of K.  On
// these small levels a launch costs its latency, not its work.
//
// Down: the smoothing from zero is pointwise, so a coarse point's restricted
// residual depends only on the finer level within two points of its
// footprint.  A workgroup owning a C x C tile of level lev0 + K computes every
// level from lev0 on the region its tile depends on (width W_K = C,
// W_k = 2 W_{k+1} + 4, origin O_k = 2 O_{k+1} - 2), all in LDS, with the
// arithmetic of k_vdown point for point.  It writes f of each coarser level
// on its own part of the region (the up-legs read them).
//
// Up: a workgroup owning a UT x UT tile of level lev0 computes, from level
// lev0 + K - 1 up, u2 = g f + P e and the post-smoothing on the region its
// tile depends on (each coarser region is the prolongation footprint of the
// finer region plus its halo of one), with the arithmetic of k_vup point for
// point; only e of level lev0 is written.
// ---------------------------------------------------------------------------
template <typename T, int K> struct LvChain {
    LevelDev<T> L[K + 1];
};
// (no recursion: the sizes fold to constants once the level loops unroll)
template <int K, int C> struct MergeDown {
    // W_K = C, W_k = 2 W_{k+1} + 4, for 0 <= k <= K
    static constexpr int width(int k) { return (C + 4) * (1 << (K - k)) - 4; }
    static constexpr int area(int k0, int k1)
    {
        int a = 0;
        for (int k = k0; k < k1; ++k) a += width(k) * width(k);
        return a;
    }
};
template <int K, int UT> struct MergeUp {
    // bound on the width of level k's e region; the fine range adds a halo of one
    static constexpr int width(int k)
    {
        int w = UT;
        for (int i = 0; i < k; ++i) w = w / 2 + 4;
        return w;
    }
    static constexpr int rw(int k) { return width(k) + 2; }
    static constexpr int rarea(int k0, int k1)
    {
        int a = 0;
        for (int k = k0; k < k1; ++k) a += rw(k) * rw(k);
        return a;
    }
    static constexpr int earea(int k0, int k1)
    {
        int a = 0;
        for (int k = k0; k < k1; ++k) a += width(k) * width(k);
        return a;
    }
    static constexpr int rpos(int k0, int k1)
    {
        int a = 0;
        for (int k = k0; k < k1; ++k) a += 2 * rw(k);
        return a;
    }
};

// origin on level k of the down region whose level-K tile starts at c0:
// O_K = c0, O_k = 2 O_{k+1} - 2
template <int K> __device__ __forceinline__ int mdown_origin(int c0, int k)
{
    return (c0 << (K - k)) - 2 * ((1 << (K - k)) - 1);
}

template <typename T, int K, int C, int NT>
__global__ __launch_bounds__(NT) void k_vdown_m(Ctx cx, LvChain<T, K> lc)
{
    using Cx = V2<T>;
    using MD = MergeDown<K, C>;
    constexpr int W0 = MD::width(0), N0 = W0 * W0, NL = (N0 + NT - 1) / NT;
    constexpr int W1 = MD::width(1), NQ = (W1 * W1 + NT - 1) / NT;
    constexpr int NF = MD::area(1, K + 1);      // f of levels 1 .. K
    constexpr int NP = MD::area(1, K) + 1;      // phi of levels 1 .. K-1
    static_assert(K >= 2 && 2 * W0 <= NT, "one coefficient position per thread and level");
    __shared__ Cx U[N0];
    __shared__ Cx F0[N0];
    __shared__ T PH0[N0];
    __shared__ Cx FK[NF];
    __shared__ T PK[NP];
    __shared__ Cx CA[K][2 * W0], CC[K][2 * W0], CD[K][2 * W0];   // [k][axis * W_k + i]

    const Cx zero = cmk<T>(0, 0);
    const int tid = threadIdx.x;
    const int run = phase_of(cx, 0);
    const T omega = (T)(cx.L ? cx.omega : cx.P->omega);
    const bool pre = (cx.L ? cx.nu1 : cx.P->nu1) != 0;
    const int tx = (lc.L[K].n[0] + C - 1) / C;
    const int b = tile_of(cx).idx;
    const int cx0 = (b % tx) * C, cy0 = (b / tx) * C;
    // all global loads first: f and phi of level lev0 on its region, phi of
    // levels 1 .. K-1 on theirs, the coefficients of levels 0 .. K-1
    Cx fr[NL];
    T pr[NL];
    {
        const int nx = lc.L[0].n[0], ny = lc.L[0].n[1];
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int l = tid + q * NT;
            const int gx = mdown_origin<K>(cx0, 0) + l % W0, gy = mdown_origin<K>(cy0, 0) + l / W0;
            fr[q] = zero;
            pr[q] = 0;
            if (l < N0 && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int64_t p = gx + (int64_t)nx * gy;
                fr[q] = ldg(lc.L[0].f, p);
                pr[q] = ldg(lc.L[0].phi, p);
            }
        }
    }
    T pk[K][NQ];
#pragma unroll
    for (int k = 1; k < K; ++k) {
        const int Wk = MD::width(k), nx = lc.L[k].n[0], ny = lc.L[k].n[1];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int l = tid + q * NT;
            const int gx = mdown_origin<K>(cx0, k) + l % Wk, gy = mdown_origin<K>(cy0, k) + l / Wk;
            pk[k][q] = 0;
            if (l < Wk * Wk && gx >= 0 && gx < nx && gy >= 0 && gy < ny) pk[k][q] = ldg(lc.L[k].phi, gx + (int64_t)nx * gy);
        }
    }
    Cx qa[K], qc[K], qd[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int Wk = MD::width(k);
        const int ax = tid >= Wk, i = tid - ax * Wk;
        const int g = (ax ? mdown_origin<K>(cy0, k) : mdown_origin<K>(cx0, k)) + i, n = ax ? lc.L[k].n[1] : lc.L[k].n[0];
        qa[k] = qc[k] = qd[k] = zero;
        if (tid < 2 * Wk && g >= 0 && g < n) {
            qa[k] = ldg(ax ? lc.L[k].a[1] : lc.L[k].a[0], g);
            qc[k] = ldg(ax ? lc.L[k].c[1] : lc.L[k].c[0], g);
            qd[k] = ldg(ax ? lc.L[k].d[1] : lc.L[k].d[0], g);
        }
    }
    {
        int off = 0;
#pragma unroll
        for (int k = 1; k < K; ++k) {
            const int Wk = MD::width(k);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int l = tid + q * NT;
                if (l < Wk * Wk) PK[off + l] = pk[k][q];
            }
            off += Wk * Wk;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (tid < 2 * MD::width(k)) {
            CA[k][tid] = qa[k];
            CC[k][tid] = qc[k];
            CD[k][tid] = qd[k];
        }
    if (run != PH_RUN) return;   // uniform over the workgroup
    __syncthreads();
    // level lev0: u1 = g f on the region
    {
        const int nx = lc.L[0].n[0], ny = lc.L[0].n[1];
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int l = tid + q * NT;
            if (l >= N0) break;
            const int lx = l % W0, ly = l / W0;
            const int gx = mdown_origin<K>(cx0, 0) + lx, gy = mdown_origin<K>(cy0, 0) + ly;
            Cx u1 = zero;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                Cx d = cadd<T>(CD[0][lx], CD[0][W0 + ly]);
                Cx D = cmk<T>(d.x - pr[q], d.y);
                T qq = jscale<T>(omega, D);
                Cx gw = cmk<T>(D.x * qq, -(D.y * qq));
                if (pre) u1 = cmul<T>(gw, fr[q]);
            }
            U[l] = u1;
            F0[l] = fr[q];
            PH0[l] = pr[q];
        }
    }
    __syncthreads();
    const T w0 = (T)0.125, w1 = (T)0.375;
    int foff = 0, poff = 0;   // level k's f and phi in FK / PK (k >= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int Wk = MD::width(k), Wn = MD::width(k + 1);
        const int nx = lc.L[k].n[0], ny = lc.L[k].n[1];
        Cx *Fk = k == 0 ? F0 : FK + foff;
        const T *Pk = k == 0 ? PH0 : PK + poff;
        Cx *Fn = FK + (k == 0 ? 0 : foff + Wk * Wk);
        if (k > 0) {
            // u1 = g f on the region
            for (int l = tid; l < Wk * Wk; l += NT) {
                const int lx = l % Wk, ly = l / Wk;
                const int gx = mdown_origin<K>(cx0, k) + lx, gy = mdown_origin<K>(cy0, k) + ly;
                Cx u1 = zero;
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                    Cx d = cadd<T>(CD[k][lx], CD[k][Wk + ly]);
                    Cx D = cmk<T>(d.x - Pk[l], d.y);
                    T qq = jscale<T>(omega, D);
                    Cx gw = cmk<T>(D.x * qq, -(D.y * qq));
                    if (pre) u1 = cmul<T>(gw, Fk[l]);
                }
                U[l] = u1;
            }
            __syncthreads();
        }
        // r = f - M u1 on the region minus its outer ring, in place
        for (int r = tid; r < (Wk - 2) * (Wk - 2); r += NT) {
            const int lx = 1 + r % (Wk - 2), ly = 1 + r / (Wk - 2);
            const int gx = mdown_origin<K>(cx0, k) + lx, gy = mdown_origin<K>(cy0, k) + ly;
            const int l = lx + Wk * ly;
            Cx res = zero;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                Cx d = cadd<T>(CD[k][lx], CD[k][Wk + ly]);
                Cx D = cmk<T>(d.x - Pk[l], d.y);
                Cx mu = cmul<T>(D, U[l]);
                mu = cmsub<T>(mu, CA[k][lx], U[l - 1]);
                mu = cmsub<T>(mu, CC[k][lx], U[l + 1]);
                mu = cmsub<T>(mu, CA[k][Wk + ly], U[l - Wk]);
                mu = cmsub<T>(mu, CC[k][Wk + ly], U[l + Wk]);
                res = csub<T>(Fk[l], mu);
            }
            Fk[l] = res;
        }
        __syncthreads();
        // full weighting onto level k + 1's region (zero outside the grid);
        // the workgroup's own part goes to memory
        {
            const int ncx = lc.L[k + 1].n[0], ncy = lc.L[k + 1].n[1];
            const int own = 2 * ((1 << (K - k - 1)) - 1), ownw = C << (K - k - 1);
            Cx *__restrict__ fout = lc.L[k + 1].f;
            for (int cl = tid; cl < Wn * Wn; cl += NT) {
                const int ix = cl % Wn, iy = cl / Wn;
                const int I = mdown_origin<K>(cx0, k + 1) + ix, J = mdown_origin<K>(cy0, k + 1) + iy;
                Cx acc_y = zero;
                if (I >= 0 && I < ncx && J >= 0 && J < ncy) {
                    const int bxl = 2 * ix + 1, byl = 2 * iy + 1;
#pragma unroll
                    for (int bb = 0; bb < 4; ++bb) {
                        const T wy = (bb == 0 || bb == 3) ? w0 : w1;
                        const Cx *row = &Fk[bxl + Wk * (byl + bb)];
                        Cx sx = crs<T>(w0, row[0]);
                        sx = crsadd<T>(sx, w1, row[1]);
                        sx = crsadd<T>(sx, w1, row[2]);
                        sx = crsadd<T>(sx, w0, row[3]);
                        acc_y = bb == 0 ? crs<T>(wy, sx) : crsadd<T>(acc_y, wy, sx);
                    }
                    if (ix >= own && ix < own + ownw && iy >= own && iy < own + ownw)
                        stg(fout, I + (int64_t)ncx * J, acc_y);
                }
                Fn[cl] = acc_y;
            }
        }
        __syncthreads();
        if (k > 0) {
            foff += Wk * Wk;
            poff += Wk * Wk;
        }
    }
}

template <typename T, int K, int UT, int NT>
__global__ __launch_bounds__(NT) void k_vup_m(Ctx cx, LvChain<T, K> lc)
{
    using Cx = V2<T>;
    using MU = MergeUp<K, UT>;
    constexpr int RW0 = MU::rw(0), NR = MU::rarea(0, K), NE = MU::earea(1, K + 1), NPOS = MU::rpos(0, K);
    constexpr int RQ = (RW0 * RW0 + NT - 1) / NT;   // loads per thread and level (level 0 is the largest)
    constexpr int WK = MU::width(K), EQ = (WK * WK + NT - 1) / NT;
    static_assert(K >= 2 && 2 * RW0 <= NT, "one coefficient position per thread and level");
    __shared__ Cx U[RW0 * RW0];
    __shared__ Cx F[NR];
    __shared__ T PH[NR];
    __shared__ Cx E[NE];                  // e of levels 1 .. K
    __shared__ Cx CA[NPOS], CC[NPOS], CD[NPOS];

    const Cx zero = cmk<T>(0, 0);
    const int tid = threadIdx.x;
    const int run = phase_of(cx, 0);
    const T omega = (T)(cx.L ? cx.omega : cx.P->omega);
    const bool pre = (cx.L ? cx.nu1 : cx.P->nu1) != 0;
    const int tx = (lc.L[0].n[0] + UT - 1) / UT;
    const int b = tile_of(cx).idx;
    // e regions: level 0 is the tile; level k + 1's covers the prolongation
    // footprint of level k's region plus its halo of one
    int ox[K + 1], oy[K + 1], wx[K + 1], wy[K + 1];
    ox[0] = (b % tx) * UT;
    oy[0] = (b / tx) * UT;
    wx[0] = wy[0] = UT;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int lx = ox[k] - 1, hx = ox[k] + wx[k], ly = oy[k] - 1, hy = oy[k] + wy[k];
        ox[k + 1] = (lx >> 1) - ((lx & 1) ? 0 : 1);
        oy[k + 1] = (ly >> 1) - ((ly & 1) ? 0 : 1);
        wx[k + 1] = (hx >> 1) + ((hx & 1) ? 1 : 0) - ox[k + 1] + 1;
        wy[k + 1] = (hy >> 1) + ((hy & 1) ? 1 : 0) - oy[k + 1] + 1;
    }
    // all global loads first: f and phi of levels 0 .. K-1 on their regions
    // with the halo, e of level K, the coefficients
    Cx fr[K][RQ];
    T pr[K][RQ];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int R = MU::rw(k), nx = lc.L[k].n[0], ny = lc.L[k].n[1];
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const int l = tid + q * NT;
            const int lx = l % R, ly = l / R;
            const int gx = ox[k] - 1 + lx, gy = oy[k] - 1 + ly;
            fr[k][q] = zero;
            pr[k][q] = 0;
            if (l < R * R && lx < wx[k] + 2 && ly < wy[k] + 2 && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int64_t p = gx + (int64_t)nx * gy;
                fr[k][q] = ldg(lc.L[k].f, p);
                pr[k][q] = ldg(lc.L[k].phi, p);
            }
        }
    }
    Cx er[EQ];
    {
        const int nx = lc.L[K].n[0], ny = lc.L[K].n[1];
#pragma unroll
        for (int q = 0; q < EQ; ++q) {
            const int l = tid + q * NT;
            const int lx = l % WK, ly = l / WK;
            const int gx = ox[K] + lx, gy = oy[K] + ly;
            er[q] = zero;
            if (l < WK * WK && lx < wx[K] && ly < wy[K] && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
                er[q] = ldg(lc.L[K].e, gx + (int64_t)nx * gy);
        }
    }
    Cx qa[K], qc[K], qd[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int R = MU::rw(k);
        const int ax = tid >= R, i = tid - ax * R;
        const int g = (ax ? oy[k] : ox[k]) - 1 + i, n = ax ? lc.L[k].n[1] : lc.L[k].n[0];
        qa[k] = qc[k] = qd[k] = zero;
        if (tid < 2 * R && g >= 0 && g < n) {
            qa[k] = ldg(ax ? lc.L[k].a[1] : lc.L[k].a[0], g);
            qc[k] = ldg(ax ? lc.L[k].c[1] : lc.L[k].c[0], g);
            qd[k] = ldg(ax ? lc.L[k].d[1] : lc.L[k].d[0], g);
        }
    }
    {
        int roff = 0, coff = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int R = MU::rw(k);
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int l = tid + q * NT;
                if (l < R * R) {
                    F[roff + l] = fr[k][q];
                    PH[roff + l] = pr[k][q];
                }
            }
            if (tid < 2 * R) {
                CA[coff + tid] = qa[k];
                CC[coff + tid] = qc[k];
                CD[coff + tid] = qd[k];
            }
            roff += R * R;
            coff += 2 * R;
        }
        Cx *EK = E + MU::earea(1, K);
#pragma unroll
        for (int q = 0; q < EQ; ++q) {
            const int l = tid + q * NT;
            if (l < WK * WK) EK[l] = er[q];
        }
    }
    if (run != PH_RUN) return;   // uniform over the workgroup
    __syncthreads();
    const T p3 = (T)0.75, p1 = (T)0.25;
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
        const int R = MU::rw(k), WE = MU::width(k + 1), WO = MU::width(k);
        const int roff = MU::rarea(0, k), coff = MU::rpos(0, k);
        const Cx *Fk = F + roff;
        const T *Pk = PH + roff;
        const Cx *Ak = CA + coff, *Ck = CC + coff, *Dk = CD + coff;
        const Cx *Ec = E + MU::earea(1, k + 1);   // e of level k + 1
        Cx *Eo = E + (k > 0 ? MU::earea(1, k) : 0);
        const int nx = lc.L[k].n[0], ny = lc.L[k].n[1];
        const int x0 = ox[k] - 1, y0 = oy[k] - 1;
        // u2 = g f + P e on the region with its halo
        for (int l = tid; l < R * R; l += NT) {
            const int lx = l % R, ly = l / R;
            const int gx = x0 + lx, gy = y0 + ly;
            Cx u2 = zero;
            if (lx < wx[k] + 2 && ly < wy[k] + 2 && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                Cx d = cadd<T>(Dk[lx], Dk[R + ly]);
                Cx D = cmk<T>(d.x - Pk[l], d.y);
                T qq = jscale<T>(omega, D);
                Cx gw = cmk<T>(D.x * qq, -(D.y * qq));
                Cx u1 = pre ? cmul<T>(gw, Fk[l]) : zero;
                const int Ix = (gx >> 1) - ox[k + 1], Iox = ((gx & 1) ? (gx >> 1) + 1 : (gx >> 1) - 1) - ox[k + 1];
                const int Iy = (gy >> 1) - oy[k + 1], Ioy = ((gy & 1) ? (gy >> 1) + 1 : (gy >> 1) - 1) - oy[k + 1];
                Cx a0 = crs2<T>(p3, Ec[Ix + WE * Iy], p1, Ec[Iox + WE * Iy]);
                Cx a1 = crs2<T>(p3, Ec[Ix + WE * Ioy], p1, Ec[Iox + WE * Ioy]);
                Cx pe = crs2<T>(p3, a0, p1, a1);
                u2 = cadd<T>(u1, pe);
            }
            U[l] = u2;
        }
        __syncthreads();
        // post-smoothing on the region; level lev0's goes to memory
        for (int r = tid; r < WO * WO; r += NT) {
            const int ix = r % WO, iy = r / WO;
            if (ix >= wx[k] || iy >= wy[k]) continue;
            const int lx = ix + 1, ly = iy + 1;
            const int gx = x0 + lx, gy = y0 + ly;
            const int l = lx + R * ly;
            Cx u = zero;
            const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            if (in) {
                Cx d = cadd<T>(Dk[lx], Dk[R + ly]);
                Cx D = cmk<T>(d.x - Pk[l], d.y);
                T qq = jscale<T>(omega, D);
                Cx gw = cmk<T>(D.x * qq, -(D.y * qq));
                Cx mu = cmul<T>(D, U[l]);
                mu = cmsub<T>(mu, Ak[lx], U[l - 1]);
                mu = cmsub<T>(mu, Ck[lx], U[l + 1]);
                mu = cmsub<T>(mu, Ak[R + ly], U[l - R]);
                mu = cmsub<T>(mu, Ck[R + ly], U[l + R]);
                u = cmadd<T>(U[l], gw, csub<T>(Fk[l], mu));
            }
            if (k == 0) {
                if (in) stg(lc.L[0].e, gx + (int64_t)nx * gy, u);
            } else {
                Eo[ix + WO * iy] = u;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3D down-leg, z-streaming form (same results as k_vdown, value for value).
// A workgroup owns a CX x CY column of coarse points over ZC coarse planes
// and walks its fine planes upwards: the fine xy box (halo 2) of each plane
// is computed once, four u1 planes and two residual planes stay in LDS, and
// each coarse plane's full weighting is accumulated in registers as its four
// fine planes go by (z terms in the same order as k_vdown).  One barrier per
// fine plane; the loads of f and phi run PD planes ahead in registers.
// Step j of the walk:  phase 1: u1 on plane j, restriction of residual plane
// j - 3;  barrier;  phase 2: residual on plane j - 1.
// ---------------------------------------------------------------------------
template <typename T, int VT> struct ZTile {
    static constexpr int CX = TileSet<3>::X[VT], CY = TileSet<3>::Y[VT], ZC = TileSet<3>::Z[VT];
    static constexpr int NT = TileSet<3>::T[VT];
    static constexpr int PD = 2;        // planes of f and phi loaded ahead
    static constexpr int RS = PD + 1;   // register ring of planes
};

template <typename T, typename TF, int VT>
__global__ __launch_bounds__(TileSet<3>::T[VT]) void k_vdown_z(Ctx cx, int lev, int fsel, const void *fptr, LvPair<T> lp)
{
    using C = V2<T>;
    constexpr int CX = ZTile<T, VT>::CX, CY = ZTile<T, VT>::CY, ZC = ZTile<T, VT>::ZC, NT = ZTile<T, VT>::NT;
    constexpr int RX = 2 * CX + 4, RY = 2 * CY + 4, RP = RX * RY;   // fine xy box, halo 2
    constexpr int NZ = 2 * ZC + 4;                                  // fine planes of u1
    constexpr int NL = (RP + NT - 1) / NT;                          // box points per thread
    constexpr int RM = RX > RY ? RX : RY;
    static_assert(CX * CY <= NT, "one thread per coarse column");
    __shared__ C U[4][RP];
    __shared__ C R[2][RP];
    __shared__ C A[2][RM], Cc[2][RM], Dd[2][RM];   // x and y coefficients of the box
    __shared__ C Az[NZ], Cz[NZ], Dz[NZ];           // z coefficients of the chunk's fine planes

    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    LevelDev<T> Lf, Lc;
    int run = PH_RUN;
    if (lp.valid) {
        run = phase_of(cx, tl.prob);
        Lf = lp.f;
        Lc = lp.c;
    } else {
        if (phase_of(cx, tl.prob) != PH_RUN) return;
        const LevelDev<T> *Lv = levels_of<T>(cx, pd);
        Lf = Lv[lev];
        Lc = Lv[lev + 1];
    }
    const int nfx = Lf.n[0], nfy = Lf.n[1], nfz = Lf.n[2];
    const int ncx = Lc.n[0], ncy = Lc.n[1], ncz = Lc.n[2];
    const T *__restrict__ phi = Lf.phi;
    C *__restrict__ fout = Lc.f;
    const TF *__restrict__ f = lev == 0 ? (const TF *)(fptr ? fptr : pd->vec[fsel]) : (const TF *)Lf.f;
    const T omega = (T)(cx.L ? cx.omega : pd->omega);
    const bool pre = (cx.L ? cx.nu1 : pd->nu1) != 0;   // V(1,1), or V(0,1) without pre-smoothing
    const int tx = (ncx + CX - 1) / CX, ty = (ncy + CY - 1) / CY;
    int t = tl.idx;
    const int bx = t % tx;
    t /= tx;
    const int by = t % ty, bz = t / ty;
    const int c0x = bx * CX, c0y = by * CY, c0z = bz * ZC;
    const int ox = 2 * c0x - 2, oy = 2 * c0y - 2, oz = 2 * c0z - 2;
    const C zero = cmk<T>(0, 0);
    const int64_t sy = nfx, sz = (int64_t)nfx * nfy;
    const int tid = threadIdx.x;

    // this thread's box points (the same in every plane)
    int64_t pxy[NL];
    bool inxy[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = tid + q * NT;
        const int gx = ox + l % RX, gy = oy + l / RX;
        inxy[q] = l < RP && gx >= 0 && gx < nfx && gy >= 0 && gy < nfy;
        pxy[q] = inxy[q] ? gx + sy * gy : 0;
    }
    // register ring of f and phi: plane j in slot j % RS
    constexpr int PD = ZTile<T, VT>::PD, RS = ZTile<T, VT>::RS;
    TF fr[RS][NL];
    T pr[RS][NL];
    auto load = [&](int j, TF(&fd)[NL], T(&pdst)[NL]) {
        const int gz = oz + j;
        const bool zin = j < NZ && gz >= 0 && gz < nfz;
#pragma unroll
        for (int q = 0; q < NL; ++q)
            if (zin && inxy[q]) {
                fd[q] = ldg(f, pxy[q] + sz * gz);
                pdst[q] = ldg(phi, pxy[q] + sz * gz);
            }
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) load(u, fr[u], pr[u]);
    // coefficients of the box and of the chunk's planes
    {
        const V2<T> *ax0 = Lf.a[0], *cx0 = Lf.c[0], *dx0 = Lf.d[0];
        const V2<T> *ax1 = Lf.a[1], *cx1 = Lf.c[1], *dx1 = Lf.d[1];
        const V2<T> *ax2 = Lf.a[2], *cx2 = Lf.c[2], *dx2 = Lf.d[2];
        for (int l = tid; l < RX + RY + NZ; l += NT) {
            const int ax = l < RX ? 0 : (l < RX + RY ? 1 : 2);
            const int q = ax == 0 ? l : (ax == 1 ? l - RX : l - RX - RY);
            const int g = (ax == 0 ? ox : (ax == 1 ? oy : oz)) + q;
            const int nn = ax == 0 ? nfx : (ax == 1 ? nfy : nfz);
            const bool in = g >= 0 && g < nn;
            const V2<T> *pa = ax == 0 ? ax0 : (ax == 1 ? ax1 : ax2);
            const V2<T> *pc = ax == 0 ? cx0 : (ax == 1 ? cx1 : cx2);
            const V2<T> *pdd = ax == 0 ? dx0 : (ax == 1 ? dx1 : dx2);
            const C va = in ? ldg(pa, g) : zero, vc = in ? ldg(pc, g) : zero, vd = in ? ldg(pdd, g) : zero;
            if (ax < 2) {
                A[ax][q] = va;
                Cc[ax][q] = vc;
                Dd[ax][q] = vd;
            } else {
                Az[q] = va;
                Cz[q] = vc;
                Dz[q] = vd;
            }
        }
    }
    if (run != PH_RUN) return;   // uniform over the workgroup
    __syncthreads();

    // this thread's box columns: x and y coefficients and d_x + d_y, the
    // same in every plane
    int lxq[NL], lyq[NL];
    C dxy[NL], a0q[NL], c0q[NL], a1q[NL], c1q[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = tid + q * NT < RP ? tid + q * NT : 0;
        lxq[q] = l % RX;
        lyq[q] = l / RX;
        dxy[q] = cadd<T>(Dd[0][lxq[q]], Dd[1][lyq[q]]);
        a0q[q] = A[0][lxq[q]];
        c0q[q] = Cc[0][lxq[q]];
        a1q[q] = A[1][lyq[q]];
        c1q[q] = Cc[1][lyq[q]];
    }
    const T w0 = (T)0.125, w1 = (T)0.375;
    // restriction: thread tid < CX * CY owns coarse column (ix, iy)
    const int ix = tid % CX, iy = tid / CX;
    const bool cown = tid < CX * CY && c0x + ix < ncx && c0y + iy < ncy;
    C accOld = zero, accNew = zero;

    // step j uses plane j (slot fj) and plane j - 1 (slot fm), then loads
    // plane j + PD into the slot plane j - 1 leaves
    auto step = [&](int j, TF(&fj)[NL], T(&pj)[NL], TF(&fm)[NL], T(&pm)[NL]) {
        // phase 1a: u1 on plane j
        if (j < NZ) {
            const int gz = oz + j;
            const bool zin = gz >= 0 && gz < nfz;
            C *Uj = U[j & 3];
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int l = tid + q * NT;
                if (l < RP) {
                    C u1 = zero;
                    if (zin && inxy[q]) {
                        const C fv = ccvt<T>(fj[q]);
                        const C d = cadd<T>(dxy[q], Dz[j]);
                        C D = cmk<T>(d.x - pj[q], d.y);
                        T qq = jscale<T>(omega, D);
                        C gw = cmk<T>(D.x * qq, -(D.y * qq));
                        if (pre) u1 = cmul<T>(gw, fv);
                    }
                    Uj[l] = u1;
                }
            }
        }
        // phase 1b: restriction of residual plane m = j - 3 (box planes 1 .. NZ - 2)
        const int m = j - 3;
        if (m >= 1 && m <= NZ - 2 && cown) {
            const C *Rm = R[m & 1];
            const int bxl = 2 * ix + 1, byl = 2 * iy + 1;
            C acc_y = zero;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T wy = (b == 0 || b == 3) ? w0 : w1;
                const C *row = &Rm[bxl + RX * (byl + b)];
                C sx = crs<T>(w0, row[0]);
                sx = crsadd<T>(sx, w1, row[1]);
                sx = crsadd<T>(sx, w1, row[2]);
                sx = crsadd<T>(sx, w0, row[3]);
                acc_y = b == 0 ? crs<T>(wy, sx) : crsadd<T>(acc_y, wy, sx);
            }
            // plane m is term c = 0 of coarse plane (m - 1) / 2 and term
            // c = 2 of the one below (m odd), or terms c = 1 and c = 3 (m even)
            if (m & 1) {
                const int i = (m - 1) >> 1;
                if (i >= 1) accOld = crsadd<T>(accOld, w1, acc_y);
                accNew = crs<T>(w0, acc_y);
            } else {
                const int i = (m - 2) >> 1;
                accNew = crsadd<T>(accNew, w1, acc_y);
                if (i >= 1) {
                    accOld = crsadd<T>(accOld, w0, acc_y);
                    const int K = c0z + i - 1;
                    if (K < ncz) stg(fout, (c0x + ix) + (int64_t)ncx * ((c0y + iy) + (int64_t)ncy * K), accOld);
                }
                accOld = accNew;
            }
        }
        __syncthreads();
        // phase 2: residual r = f - M u1 on plane j - 1 (inner box points)
        const int r = j - 1;
        if (r >= 1 && r <= NZ - 2) {
            const int gzr = oz + r;
            const bool zin = gzr >= 0 && gzr < nfz;
            const C *Ub = U[(r - 1) & 3], *Uc = U[r & 3], *Ut = U[(r + 1) & 3];
            C *Rr = R[r & 1];
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int l = tid + q * NT;
                const int lx = lxq[q], ly = lyq[q];
                if (l < RP && lx >= 1 && lx <= RX - 2 && ly >= 1 && ly <= RY - 2) {
                    C res = zero;
                    if (zin && inxy[q]) {
                        const C d = cadd<T>(dxy[q], Dz[r]);
                        C D = cmk<T>(d.x - pm[q], d.y);
                        C mu = cmul<T>(D, Uc[l]);
                        mu = cmsub<T>(mu, a0q[q], Uc[l - 1]);
                        mu = cmsub<T>(mu, c0q[q], Uc[l + 1]);
                        mu = cmsub<T>(mu, a1q[q], Uc[l - RX]);
                        mu = cmsub<T>(mu, c1q[q], Uc[l + RX]);
                        mu = cmsub<T>(mu, Az[r], Ub[l]);
                        mu = cmsub<T>(mu, Cz[r], Ut[l]);
                        res = csub<T>(ccvt<T>(fm[q]), mu);
                    }
                    Rr[l] = res;
                }
            }
        }
        load(j + PD, fm, pm);
    };
    constexpr int NS = NZ + 2;   // steps 0 .. NZ + 1
    for (int j0 = 0; j0 < NS; j0 += RS) {
#pragma unroll
        for (int u = 0; u < RS; ++u)
            if (j0 + u < NS) step(j0 + u, fr[u], pr[u], fr[(u + RS - 1) % RS], pr[(u + RS - 1) % RS]);
    }
}

// ---------------------------------------------------------------------------
// 3D up-leg, z-streaming form (same results as k_vup, value for value).
// A workgroup owns a 2CX x 2CY column of fine points over 2ZC fine planes;
// e of the coarse box it needs is staged in LDS first.  Step j: u2 = g f + P e
// on plane j of the box (halo 1);  barrier;  smoothing of plane j - 1 and its
// store.  Four u2 planes stay in LDS; f and phi run PD planes ahead in
// registers.
// ---------------------------------------------------------------------------
template <typename T, typename TF, typename TO, int VT>
__global__ __launch_bounds__(TileSet<3>::T[VT]) void k_vup_z(Ctx cx, int lev, int fsel, int osel, const void *fptr,
                                                             void *optr, LvPair<T> lp)
{
    using C = V2<T>;
    constexpr int CX = ZTile<T, VT>::CX, CY = ZTile<T, VT>::CY, ZC = ZTile<T, VT>::ZC, NT = ZTile<T, VT>::NT;
    constexpr int FX = 2 * CX, FY = 2 * CY, FZ = 2 * ZC;
    constexpr int RX = FX + 2, RY = FY + 2, RP = RX * RY;   // fine xy box, halo 1
    constexpr int NZ = FZ + 2;                             // fine planes of u2
    constexpr int EX = CX + 4, EY = CY + 4, EZ = ZC + 4, EN = EX * EY * EZ;
    constexpr int NL = (RP + NT - 1) / NT;
    constexpr int NE = (EN + NT - 1) / NT;
    constexpr int RM = RX > RY ? RX : RY;
    __shared__ C U[4][RP];
    __shared__ C E[EN];
    __shared__ C A[2][RM], Cc[2][RM], Dd[2][RM];
    __shared__ C Az[NZ], Cz[NZ], Dz[NZ];

    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    LevelDev<T> Lf, Lc;
    int run = PH_RUN;
    if (lp.valid) {
        run = phase_of(cx, tl.prob);
        Lf = lp.f;
        Lc = lp.c;
    } else {
        if (phase_of(cx, tl.prob) != PH_RUN) return;
        const LevelDev<T> *Lv = levels_of<T>(cx, pd);
        Lf = Lv[lev];
        Lc = Lv[lev + 1];
    }
    const int nfx = Lf.n[0], nfy = Lf.n[1], nfz = Lf.n[2];
    const int ncx = Lc.n[0], ncy = Lc.n[1], ncz = Lc.n[2];
    const T *__restrict__ phi = Lf.phi;
    const C *__restrict__ ec = Lc.e;
    C *__restrict__ eout = Lf.e;
    const TF *__restrict__ f = lev == 0 ? (const TF *)(fptr ? fptr : pd->vec[fsel]) : (const TF *)Lf.f;
    TO *__restrict__ outv = lev == 0 ? (TO *)(optr ? optr : pd->vec[osel]) : nullptr;
    const T omega = (T)(cx.L ? cx.omega : pd->omega);
    const bool pre = (cx.L ? cx.nu1 : pd->nu1) != 0;   // V(1,1), or V(0,1) without pre-smoothing
    const int tx = (nfx + FX - 1) / FX, ty = (nfy + FY - 1) / FY;
    int t = tl.idx;
    const int bx = t % tx;
    t /= tx;
    const int by = t % ty, bz = t / ty;
    const int f0x = bx * FX, f0y = by * FY, f0z = bz * FZ;
    const int ox = f0x - 1, oy = f0y - 1, oz = f0z - 1;
    const int ex0 = (f0x >> 1) - 2, ey0 = (f0y >> 1) - 2, ez0 = (f0z >> 1) - 2;
    const C zero = cmk<T>(0, 0);
    const int64_t sy = nfx, sz = (int64_t)nfx * nfy;
    const int tid = threadIdx.x;

    int64_t pxy[NL];
    bool inxy[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = tid + q * NT;
        const int gx = ox + l % RX, gy = oy + l / RX;
        inxy[q] = l < RP && gx >= 0 && gx < nfx && gy >= 0 && gy < nfy;
        pxy[q] = inxy[q] ? gx + sy * gy : 0;
    }
    constexpr int PD = ZTile<T, VT>::PD, RS = ZTile<T, VT>::RS;
    TF fr[RS][NL];
    T pr[RS][NL];
    auto load = [&](int j, TF(&fd)[NL], T(&pdst)[NL]) {
        const int gz = oz + j;
        const bool zin = j < NZ && gz >= 0 && gz < nfz;
#pragma unroll
        for (int q = 0; q < NL; ++q)
            if (zin && inxy[q]) {
                fd[q] = ldg(f, pxy[q] + sz * gz);
                pdst[q] = ldg(phi, pxy[q] + sz * gz);
            }
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) load(u, fr[u], pr[u]);
    // e on the coarse box
    {
        C er[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int l = tid + q * NT;
            const int lx = l % EX, ly = (l / EX) % EY, lz = l / (EX * EY);
            const int gx = ex0 + lx, gy = ey0 + ly, gz = ez0 + lz;
            er[q] = zero;
            if (l < EN && gx >= 0 && gx < ncx && gy >= 0 && gy < ncy && gz >= 0 && gz < ncz)
                er[q] = ldg(ec, gx + (int64_t)ncx * (gy + (int64_t)ncy * gz));
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int l = tid + q * NT;
            if (l < EN) E[l] = er[q];
        }
    }
    {
        const V2<T> *ax0 = Lf.a[0], *cx0 = Lf.c[0], *dx0 = Lf.d[0];
        const V2<T> *ax1 = Lf.a[1], *cx1 = Lf.c[1], *dx1 = Lf.d[1];
        const V2<T> *ax2 = Lf.a[2], *cx2 = Lf.c[2], *dx2 = Lf.d[2];
        for (int l = tid; l < RX + RY + NZ; l += NT) {
            const int ax = l < RX ? 0 : (l < RX + RY ? 1 : 2);
            const int q = ax == 0 ? l : (ax == 1 ? l - RX : l - RX - RY);
            const int g = (ax == 0 ? ox : (ax == 1 ? oy : oz)) + q;
            const int nn = ax == 0 ? nfx : (ax == 1 ? nfy : nfz);
            const bool in = g >= 0 && g < nn;
            const V2<T> *pa = ax == 0 ? ax0 : (ax == 1 ? ax1 : ax2);
            const V2<T> *pc = ax == 0 ? cx0 : (ax == 1 ? cx1 : cx2);
            const V2<T> *pdd = ax == 0 ? dx0 : (ax == 1 ? dx1 : dx2);
            const C va = in ? ldg(pa, g) : zero, vc = in ? ldg(pc, g) : zero, vd = in ? ldg(pdd, g) : zero;
            if (ax < 2) {
                A[ax][q] = va;
                Cc[ax][q] = vc;
                Dd[ax][q] = vd;
            } else {
                Az[q] = va;
                Cz[q] = vc;
                Dz[q] = vd;
            }
        }
    }
    if (run != PH_RUN) return;   // uniform over the workgroup
    __syncthreads();
    const T p3 = (T)0.75, p1 = (T)0.25;
    // this thread's box columns: x and y coefficients, d_x + d_y and the
    // prolongation columns, the same in every plane
    int lxq[NL], lyq[NL], ixq[NL], ioxq[NL], iyq[NL], ioyq[NL];
    C dxy[NL], a0q[NL], c0q[NL], a1q[NL], c1q[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int l = tid + q * NT < RP ? tid + q * NT : 0;
        lxq[q] = l % RX;
        lyq[q] = l / RX;
        const int gx = ox + lxq[q], gy = oy + lyq[q];
        ixq[q] = (gx >> 1) - ex0;
        ioxq[q] = ((gx & 1) ? (gx >> 1) + 1 : (gx >> 1) - 1) - ex0;
        iyq[q] = (gy >> 1) - ey0;
        ioyq[q] = ((gy & 1) ? (gy >> 1) + 1 : (gy >> 1) - 1) - ey0;
        dxy[q] = cadd<T>(Dd[0][lxq[q]], Dd[1][lyq[q]]);
        a0q[q] = A[0][lxq[q]];
        c0q[q] = Cc[0][lxq[q]];
        a1q[q] = A[1][lyq[q]];
        c1q[q] = Cc[1][lyq[q]];
    }

    auto step = [&](int j, TF(&fj)[NL], T(&pj)[NL], TF(&fm)[NL], T(&pm)[NL]) {
        // phase 1: u2 = g f + P e on plane j
        if (j < NZ) {
            const int gz = oz + j;
            const bool zin = gz >= 0 && gz < nfz;
            const int Iz = (gz >> 1) - ez0, Ioz = ((gz & 1) ? (gz >> 1) + 1 : (gz >> 1) - 1) - ez0;
            C *Uj = U[j & 3];
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int l = tid + q * NT;
                if (l < RP) {
                    C u2 = zero;
                    if (zin && inxy[q]) {
                        const C fv = ccvt<T>(fj[q]);
                        const C d = cadd<T>(dxy[q], Dz[j]);
                        C D = cmk<T>(d.x - pj[q], d.y);
                        T qq = jscale<T>(omega, D);
                        C gw = cmk<T>(D.x * qq, -(D.y * qq));
                        C u1 = pre ? cmul<T>(gw, fv) : zero;
                        const int Ix = ixq[q], Iox = ioxq[q], Iy = iyq[q], Ioy = ioyq[q];
                        C pz[2];
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const int zz = c == 0 ? Iz : Ioz;
                            C a0 = crs2<T>(p3, E[Ix + EX * (Iy + EY * zz)], p1, E[Iox + EX * (Iy + EY * zz)]);
                            C a1 = crs2<T>(p3, E[Ix + EX * (Ioy + EY * zz)], p1, E[Iox + EX * (Ioy + EY * zz)]);
                            pz[c] = crs2<T>(p3, a0, p1, a1);
                        }
                        const C pe = crs2<T>(p3, pz[0], p1, pz[1]);
                        u2 = cadd<T>(u1, pe);
                    }
                    Uj[l] = u2;
                }
            }
        }
        __syncthreads();
        // phase 2: smoothing of plane j - 1 on the tile, and its store
        const int r = j - 1;
        if (r >= 1 && r <= NZ - 2) {
            const int gz = oz + r;
            const C *Ub = U[(r - 1) & 3], *Uc = U[r & 3], *Ut = U[(r + 1) & 3];
            if (gz < nfz) {
#pragma unroll
                for (int q = 0; q < NL; ++q) {
                    const int l = tid + q * NT;
                    const int lx = lxq[q], ly = lyq[q];
                    if (l < RP && lx >= 1 && lx <= FX && ly >= 1 && ly <= FY && ox + lx < nfx && oy + ly < nfy) {
                        const C d = cadd<T>(dxy[q], Dz[r]);
                        C D = cmk<T>(d.x - pm[q], d.y);
                        T qq = jscale<T>(omega, D);
                        C gw = cmk<T>(D.x * qq, -(D.y * qq));
                        C mu = cmul<T>(D, Uc[l]);
                        mu = cmsub<T>(mu, a0q[q], Uc[l - 1]);
                        mu = cmsub<T>(mu, c0q[q], Uc[l + 1]);
                        mu = cmsub<T>(mu, a1q[q], Uc[l - RX]);
                        mu = cmsub<T>(mu, c1q[q], Uc[l + RX]);
                        mu = cmsub<T>(mu, Az[r], Ub[l]);
                        mu = cmsub<T>(mu, Cz[r], Ut[l]);
                        C u = cmadd<T>(Uc[l], gw, csub<T>(ccvt<T>(fm[q]), mu));
                        const int64_t p = pxy[q] + sz * gz;
                        if (lev == 0) {
                            TO o;
                            o.x = u.x;
                            o.y = u.y;
                            stg(outv, p, o);
                        } else {
                            stg(eout, p, u);
                        }
                    }
                }
            }
        }
        load(j + PD, fm, pm);
    };
    constexpr int NS = NZ;   // steps 0 .. NZ - 1
    for (int j0 = 0; j0 < NS; j0 += RS) {
#pragma unroll
        for (int u = 0; u < RS; ++u)
            if (j0 + u < NS) step(j0 + u, fr[u], pr[u], fr[(u + RS - 1) % RS], pr[(u + RS - 1) % RS]);
    }
}

// ---------------------------------------------------------------------------
// tail of the V-cycle: every level from `tail` down to the coarsest inside
// one workgroup, all fields in LDS.  Reads f_tail, writes e_tail.  Same
// arithmetic as the tiled kernels; the coarsest solve applies the explicit
// inverse with a pairwise sum per row.
// ---------------------------------------------------------------------------
// Slots per lane and batch of the coarse solve (rows per batch = slots / seg);
// fewer for FP64 to stay within the register file.
template <typename T> __host__ __device__ constexpr int coarse_slots(int seg)
{
    return sizeof(T) == 8 ? (seg > 8 ? seg : 8) : 16;
}

// (always inlined: LDS operands then keep their address space)
template <typename T, int SEG>
__device__ __forceinline__ void coarse_rows_seg(const V2<T> *__restrict__ Minv, const V2<T> *f, V2<T> *e, int n, int row0, int rstep)
{
    constexpr int NS = coarse_slots<T>(SEG);
    constexpr int RPB = NS / SEG;  // rows per batch
    const int lane = threadIdx.x & 63;
    // the entries of f this lane multiplies (reads clamped into f, masked
    // by the column test below)
    V2<T> fv[SEG];
#pragma unroll
    for (int c = 0; c < SEG; ++c) {
        const int col = lane * SEG + c;
        fv[c] = f[col < n ? col : n - 1];
    }
    for (int rb = row0; rb < n; rb += RPB * rstep) {
        T re[NS], im[NS];
        // inverse entries in groups of 8 loads in flight together (unused
        // slots read entry 0); the products of unused slots are replaced by
        // zero
#pragma unroll
        for (int h = 0; h < NS; h += 8) {
            V2<T> mv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int row = rb + ((h + q) / SEG) * rstep, col = lane * SEG + (h + q) % SEG;
                const int64_t idx = (row < n && col < n) ? (int64_t)row * n + col : 0;
                mv[q] = ldg(Minv, idx);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int row = rb + ((h + q) / SEG) * rstep, col = lane * SEG + (h + q) % SEG;
                const V2<T> pr = cmul<T>(mv[q], fv[(h + q) % SEG]);
                const bool in = row < n && col < n;
                re[h + q] = in ? pr.x : (T)0;
                im[h + q] = in ? pr.y : (T)0;
            }
        }
        // in-lane pairwise over each row's segment (aligned power-of-two
        // blocks of the slots); row r's partial ends in slot r * SEG
#pragma unroll
        for (int w = 1; w < SEG; w <<= 1) {
#pragma unroll
            for (int i = 0; i + w < NS; i += 2 * w) {
                re[i] = re[i] + re[i + w];
                im[i] = im[i] + im[i + w];
            }
        }
        // pairwise across the wave, up to 4 rows of the batch together
        constexpr int RG = RPB < 4 ? RPB : 4;
#pragma unroll
        for (int r0 = 0; r0 < RPB; r0 += RG) {
            if (rb + r0 * rstep >= n) break;   // rest of the batch past the last row (uniform)
#pragma unroll
            for (int r = r0; r < r0 + RG; ++r) {
                re[r * SEG] = wave_sum(re[r * SEG]);
                im[r * SEG] = wave_sum(im[r * SEG]);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < RPB; ++r) {
                const int row = rb + r * rstep;
                if (row < n) e[row] = cmk<T>(re[r * SEG], im[r * SEG]);
            }
        }
    }
}

// Coarsest solve by one wave: rows row0, row0 + rstep, ... (16 / seg rows
// per batch, loads issued together) of Minv applied to f; each row is summed
// pairwise over its zero-padded length np = max(64, 2^ceil(log2 n)) (lane
// segments of seg = np/64 terms, then a butterfly).  Lane 0 writes e[row].
// Inside the tail kernel n <= HH_SPLIT_NC, so seg is 1 or 2.
__host__ __device__ inline int coarse_seg(int n)
{
    int np = 64;
    while (np < n) np <<= 1;
    return np >> 6;
}
// Coarsest solve from registers, at most 64 unknowns: lane l of wave w holds
// m[k] = Minv[(w + k W) n + l] (W waves); each row summed pairwise over the 64
// lanes with zeros past n, as in coarse_rows_seg with one-term segments.
template <typename T, int MR>
__device__ __forceinline__ void coarse_rows_reg(const V2<T> (&m)[MR], const V2<T> *f, V2<T> *e, int n, int w, int W)
{
    const int lane = threadIdx.x & 63;
    const V2<T> fv = f[lane < n ? lane : n - 1];
    T re[MR], im[MR];
#pragma unroll
    for (int k = 0; k < MR; ++k) {
        const V2<T> pr = cmul<T>(m[k], fv);
        const bool in = w + W * k < n && lane < n;
        re[k] = in ? pr.x : (T)0;
        im[k] = in ? pr.y : (T)0;
    }
#pragma unroll
    for (int k = 0; k < MR; ++k)
        if (w + W * k < n) {   // uniform over the wave
            re[k] = wave_sum(re[k]);
            im[k] = wave_sum(im[k]);
        }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < MR; ++k)
            if (w + W * k < n) e[w + W * k] = cmk<T>(re[k], im[k]);
}

template <typename T>
__device__ __forceinline__ void coarse_rows_tail(const V2<T> *__restrict__ Minv, const V2<T> *f, V2<T> *e, int n, int row0, int rstep)
{
    static_assert(HH_SPLIT_NC <= 128, "tail coarse solve handles seg 1 and 2");
    if (coarse_seg(n) == 1) coarse_rows_seg<T, 1>(Minv, f, e, n, row0, rstep);
    else coarse_rows_seg<T, 2>(Minv, f, e, n, row0, rstep);
}


// What the tail kernel of a one-problem plan takes by value (see k_vtail).
template <typename T> struct TailArgs {
    const LevelDev<T> *Lv;           // level descriptors (device array)
    const V2<T> *f_top;              // f of the tail's first level
    V2<T> *e_top;                    // e of the tail's first level
    const V2<T> *Minv;               // coarsest inverse
    const void *img;                 // tail image (see tail_image)
    int n16, nseg;                   // image length in 16-byte units, segments
    const TailTab *tab;              // level table (see tail_table)
    int t0, L, Nc, split, nu1;
    T omega;
    uint32_t seg[HH_MAXLEV];         // image segments
};

// pointers of one tail level into the LDS block
template <typename T> struct TailPtr {
    int nx, ny, nz, N;
    FastDiv fx, fxy;
    V2<T> *F, *E, *A0, *A1, *A2, *C0, *C1, *C2, *D0, *D1, *D2;
    T *PH;
};

template <int DIM, typename T>
__device__ inline TailPtr<T> tail_ptr(char *lds, const TailTab &tab, int l)
{
    const TailOff &o = tab.o[l];
    TailPtr<T> q;
    q.nx = o.n[0];
    q.ny = o.n[1];
    q.nz = o.n[2];
    q.N = o.N;
    q.fx = tab.fx[l];
    q.fxy = tab.fxy[l];
    q.F = (V2<T> *)(lds + o.F);
    q.E = (V2<T> *)(lds + o.E);
    q.PH = (T *)(lds + o.PH);
    q.A0 = (V2<T> *)(lds + o.A[0]); q.A1 = (V2<T> *)(lds + o.A[1]); q.A2 = (V2<T> *)(lds + o.A[2]);
    q.C0 = (V2<T> *)(lds + o.Cc[0]); q.C1 = (V2<T> *)(lds + o.Cc[1]); q.C2 = (V2<T> *)(lds + o.Cc[2]);
    q.D0 = (V2<T> *)(lds + o.Dd[0]); q.D1 = (V2<T> *)(lds + o.Dd[1]); q.D2 = (V2<T> *)(lds + o.Dd[2]);
    return q;
}

template <int DIM, typename T>
__device__ inline V2<T> tail_diag(const TailPtr<T> &Q, int i, int j, int k, int p)
{
    V2<T> d = cadd<T>(Q.D0[i], Q.D1[j]);
    if (DIM == 3) d = cadd<T>(d, Q.D2[k]);
    return cmk<T>(d.x - Q.PH[p], d.y);
}

template <int DIM, typename T>
__device__ inline V2<T> tail_Mu(const TailPtr<T> &Q, const V2<T> *U, V2<T> D, int i, int j, int k, int p)
{
    using C = V2<T>;
    const C zero = cmk<T>(0, 0);
    const int sy = Q.nx, sz = Q.nx * Q.ny;
    // neighbours outside the level are zero: every read stays inside the
    // level (clamped to p) and is masked, so the reads issue together
    const C uw = U[i > 0 ? p - 1 : p], ue = U[i < Q.nx - 1 ? p + 1 : p];
    const C us = U[j > 0 ? p - sy : p], un = U[j < Q.ny - 1 ? p + sy : p];
    C mu = cmul<T>(D, U[p]);
    mu = cmsub<T>(mu, Q.A0[i], i > 0 ? uw : zero);
    mu = cmsub<T>(mu, Q.C0[i], i < Q.nx - 1 ? ue : zero);
    mu = cmsub<T>(mu, Q.A1[j], j > 0 ? us : zero);
    mu = cmsub<T>(mu, Q.C1[j], j < Q.ny - 1 ? un : zero);
    if (DIM == 3) {
        const C ub = U[k > 0 ? p - sz : p], ut = U[k < Q.nz - 1 ? p + sz : p];
        mu = cmsub<T>(mu, Q.A2[k], k > 0 ? ub : zero);
        mu = cmsub<T>(mu, Q.C2[k], k < Q.nz - 1 ? ut : zero);
    }
    return mu;
}

template <typename T>
__device__ inline void tail_ijk(const TailPtr<T> &Q, int p, int &i, int &j, int &k)
{
    split(p, Q.nx, Q.ny, Q.fx, Q.fxy, i, j, k);
}

// ---------------------------------------------------------------------------
// tail of the V-cycle: every level from `tail` down to the coarsest inside
// one workgroup, all fields in LDS.  Reads f_tail, writes e_tail.  Same
// arithmetic as the tiled kernels; the coarsest solve applies the explicit
// inverse with a pairwise sum per row.
// ---------------------------------------------------------------------------
// up = 0: the whole tail (down-legs, coarsest solve, up-legs), or, for a
// problem whose coarsest solve runs in k_coarse, the down-legs only (the
// restricted right-hand sides of the tail levels go to global memory).
// up = 1: the up-legs of such a problem, from those right-hand sides and the
// coarsest solution k_coarse left in global memory.
// BV (one problem): every value read before the first barrier comes by
// value in ta, so the loads of f, the image and the inverse issue at once,
// next to the phase load, instead of after a chain of dependent descriptor
// loads; the phase decides only at that barrier.  Batches (BV false) read
// the problem descriptor.
template <int DIM, typename T, bool BV>
__global__ __launch_bounds__(TailCap<T>::WG) void k_vtail(Ctx cx, const int *__restrict__ probs, int up, TailArgs<T> ta)
{
    using C = V2<T>;
    __shared__ __attribute__((aligned(16))) char lds[TailCap<T>::BYTES];
    const int prob = !BV && probs ? probs[blockIdx.x] : 0;
    int run = PH_RUN;
    if constexpr (BV) run = phase_of(cx, prob);
    else if (phase_of(cx, prob) != PH_RUN) return;
    const ProbDev *pd = cx.P + prob;
    const int split = BV ? ta.split : pd->csplit;
    if (up && !split) return;
    const LevelDev<T> *Lv = BV ? ta.Lv : levels_of<T>(cx, pd);
    const int t0 = BV ? ta.t0 : tail_level<T>(pd), L = BV ? ta.L : pd->nlev;
    const T omega = BV ? ta.omega : (T)pd->omega;
    const bool pre = (BV ? ta.nu1 : pd->nu1) != 0;
    const C zero = cmk<T>(0, 0);
    const int tid = threadIdx.x, nth = TailCap<T>::WG;
    __shared__ TailTab tab;
    // FP32 with a coarsest grid of at most 64 unknowns: the coarsest inverse
    // is loaded with the image straight into the registers of the lanes that
    // use it (lane l of wave w: row w + k W, column l, W waves) and stays there
    // until the coarse solve, so its latency overlaps the image, f and the
    // down-legs
    constexpr int MR = sizeof(T) == 4 ? 64 / (TailCap<T>::WG / 64) : 1;   // rows per lane
    const int nc = BV ? ta.Nc : pd->Nc;
    const bool mreg = sizeof(T) == 4 && !up && !split && nc <= 64;
    C mt[MR];
    const C *fg_top = BV ? ta.f_top : Lv[t0].f;
    C *eg_top = BV ? ta.e_top : Lv[t0].e;
    const C *__restrict__ Minv =
        BV ? ta.Minv : (const C *)(sizeof(T) == 8 ? (const void *)pd->Minv64 : (const void *)pd->Minv32);
    // the tail image (phi and coefficients of every tail level, see
    // tail_image), the coarsest inverse when it goes to LDS, and f of the top
    // level, all loads in flight together while the level table is built
    {
        const void *img = BV ? ta.img : (sizeof(T) == 8 ? pd->timg64 : pd->timg32);
        const int n16 = BV ? ta.n16 : (sizeof(T) == 8 ? pd->timg_bytes64 : pd->timg_bytes32) / 16;
        const uint32_t *seg = BV ? ta.seg : (sizeof(T) == 8 ? pd->tseg64 : pd->tseg32);
        const int nseg = BV ? ta.nseg : (sizeof(T) == 8 ? pd->tnseg64 : pd->tnseg32);
        // the level table, one 32-bit word per thread
        constexpr int TW = sizeof(TailTab) / 4;
        static_assert(sizeof(TailTab) % 4 == 0 && TW <= TailCap<T>::WG, "tail table words");
        const uint32_t *tabg = (const uint32_t *)(BV ? ta.tab : (sizeof(T) == 8 ? pd->ttab64 : pd->ttab32));
        const uint32_t tw = tid < TW ? ((const HH_GLOBAL uint32_t *)tabg)[tid] : 0u;
        hh_uvec4 *l16 = (hh_uvec4 *)lds;
        if (mreg) {
            const int w = tid >> 6, lane = tid & 63;
#pragma unroll
            for (int k = 0; k < MR; ++k) {
                const int row = w + (nth >> 6) * k;
                mt[k] = (row < nc && lane < nc) ? ldg(Minv, (int64_t)row * nc + lane) : zero;
            }
        }
        // f of the top level leads the LDS block (offset 0)
        constexpr int FT = (TailCap<T>::N + TailCap<T>::WG - 1) / TailCap<T>::WG;
        const int ntop = up ? 0 : (int)Lv[t0].N;
        C ft[FT];
#pragma unroll
        for (int q = 0; q < FT; ++q) {
            const int i = tid + q * nth;
            if (i < ntop) ft[q] = ldg(fg_top, i);
        }
        for (int b = 0; b < n16; b += 8 * nth) {
            hh_uvec4 tmp[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = b + tid + q * nth;
                if (i < n16) tmp[q] = ldg16(img, i);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = b + tid + q * nth;
                if (i < n16) {
                    // segment of entry i (one per level, in order)
                    int k = 0, s0 = 0;
                    for (; k < nseg - 1; ++k) {
                        const int len = (int)(seg[k] & 0xffffu);
                        if (i < s0 + len) break;
                        s0 += len;
                    }
                    l16[(int)(seg[k] >> 16) + (i - s0)] = tmp[q];
                }
            }
        }
        if (tid < TW) ((uint32_t *)&tab)[tid] = tw;
#pragma unroll
        for (int q = 0; q < FT; ++q) {
            const int i = tid + q * nth;
            if (i < ntop) ((C *)lds)[i] = ft[q];
        }
        if (run != PH_RUN) return;   // uniform over the workgroup
        __syncthreads();
        // for the up-legs of a split tail: f of every tail level and e of the
        // coarsest
        for (int l = t0; l < (up ? L - 1 : t0); ++l) {
            const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, l);
            const C *__restrict__ fg = l == t0 ? fg_top : Lv[l].f;
            for (int b = 0; b < Q.N; b += 4 * nth) {
                C tmp[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (b + tid + q * nth < Q.N) tmp[q] = ldg(fg, b + tid + q * nth);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (b + tid + q * nth < Q.N) Q.F[b + tid + q * nth] = tmp[q];
            }
        }
        if (up) {
            const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, L - 1);
            const C *__restrict__ eg = Lv[L - 1].e;
            for (int p = tid; p < Q.N; p += nth) Q.E[p] = ldg(eg, p);
        }
    }
    if (up) __syncthreads();   // uniform
    C *U = (C *)(lds + tab.uoff);
    const T w0 = (T)0.125, w1 = (T)0.375, p3 = (T)0.75, p1 = (T)0.25;
    // down-legs
    for (int l = t0; l < L - 1 && !up; ++l) {
        const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, l);
        const TailPtr<T> R = tail_ptr<DIM, T>(lds, tab, l + 1);
        for (int p = tid; p < Q.N; p += nth) {
            int i, j, k;
            tail_ijk(Q, p, i, j, k);
            U[p] = pre ? cmul<T>(jweight<T>(tail_diag<DIM, T>(Q, i, j, k, p), omega), Q.F[p]) : zero;
        }
        __syncthreads();
        for (int p = tid; p < Q.N; p += nth) {
            int i, j, k;
            tail_ijk(Q, p, i, j, k);
            C D = tail_diag<DIM, T>(Q, i, j, k, p);
            Q.E[p] = csub<T>(Q.F[p], tail_Mu<DIM, T>(Q, U, D, i, j, k, p));   // residual kept in E
        }
        __syncthreads();
        for (int p = tid; p < R.N; p += nth) {
            int I, J, K;
            tail_ijk(R, p, I, J, K);
            C acc_z = zero;
            for (int c = 0; c < (DIM == 3 ? 4 : 1); ++c) {
                const T wz = (c == 0 || c == 3) ? w0 : w1;
                const int kk = DIM == 3 ? 2 * K - 1 + c : 0;
                const bool kin = DIM == 2 || (kk >= 0 && kk < Q.nz);
                C acc_y = zero;
                const int kc = kk < 0 ? 0 : (kk >= Q.nz ? Q.nz - 1 : kk);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T wy = (b == 0 || b == 3) ? w0 : w1;
                    const int jj = 2 * J - 1 + b;
                    const bool jin = kin && jj >= 0 && jj < Q.ny;
                    const int jc = jj < 0 ? 0 : (jj >= Q.ny ? Q.ny - 1 : jj);
                    // reads clamped into the level, points outside it masked to zero
                    C v[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int ii = 2 * I - 1 + a;
                        const int ic = ii < 0 ? 0 : (ii >= Q.nx ? Q.nx - 1 : ii);
                        const C e = Q.E[ic + Q.nx * (jc + Q.ny * kc)];
                        v[a] = (jin && ii >= 0 && ii < Q.nx) ? e : zero;
                    }
                    C sx = crs<T>(w0, v[0]);
                    sx = crsadd<T>(sx, w1, v[1]);
                    sx = crsadd<T>(sx, w1, v[2]);
                    sx = crsadd<T>(sx, w0, v[3]);
                    acc_y = b == 0 ? crs<T>(wy, sx) : crsadd<T>(acc_y, wy, sx);
                }
                if (DIM == 3) acc_z = c == 0 ? crs<T>(wz, acc_y) : crsadd<T>(acc_z, wz, acc_y);
                else acc_z = acc_y;
            }
            R.F[p] = acc_z;
        }
        __syncthreads();
    }
    if (!up && split) {
        // hand the restricted right-hand sides to k_coarse and the up-legs
        for (int l = t0 + 1; l < L; ++l) {
            const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, l);
            C *fg = Lv[l].f;
            for (int p = tid; p < Q.N; p += nth) stg(fg, p, Q.F[p]);
        }
        return;
    }
    // coarsest solve
    if (!up) {
        const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, L - 1);
        if constexpr (sizeof(T) == 4) {
            // at most 64 unknowns (one segment) from registers, else 65..128
            // (two segments) from memory
            if (mreg) coarse_rows_reg<T, MR>(mt, Q.F, Q.E, Q.N, tid >> 6, nth >> 6);
            else coarse_rows_seg<T, 2>(Minv, Q.F, Q.E, Q.N, tid >> 6, nth >> 6);
        } else {
            coarse_rows_tail<T>(Minv, Q.F, Q.E, Q.N, tid >> 6, nth >> 6);
        }
        __syncthreads();
    }
    // up-legs
    for (int l = L - 2; l >= t0; --l) {
        const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, l);
        const TailPtr<T> R = tail_ptr<DIM, T>(lds, tab, l + 1);
        for (int p = tid; p < Q.N; p += nth) {
            int i, j, k;
            tail_ijk(Q, p, i, j, k);
            C u1 = pre ? cmul<T>(jweight<T>(tail_diag<DIM, T>(Q, i, j, k, p), omega), Q.F[p]) : zero;
            const int Ix = i >> 1, Iox = (i & 1) ? Ix + 1 : Ix - 1;
            const int Iy = j >> 1, Ioy = (j & 1) ? Iy + 1 : Iy - 1;
            // coarse values outside the level are zero (read clamped, then masked)
            auto ev = [R](int a, int b, int c) -> C {
                const int ac = a < 0 ? 0 : (a >= R.nx ? R.nx - 1 : a);
                const int bc = b < 0 ? 0 : (b >= R.ny ? R.ny - 1 : b);
                const int cc = c < 0 ? 0 : (c >= R.nz ? R.nz - 1 : c);
                const C e = R.E[ac + R.nx * (bc + R.ny * cc)];
                return (a >= 0 && a < R.nx && b >= 0 && b < R.ny && c >= 0 && c < R.nz) ? e : cmk<T>(0, 0);
            };
            C pe;
            if (DIM == 2) {
                C a0 = crs2<T>(p3, ev(Ix, Iy, 0), p1, ev(Iox, Iy, 0));
                C a1 = crs2<T>(p3, ev(Ix, Ioy, 0), p1, ev(Iox, Ioy, 0));
                pe = crs2<T>(p3, a0, p1, a1);
            } else {
                const int Iz = k >> 1, Ioz = (k & 1) ? Iz + 1 : Iz - 1;
                C pz[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int zz = c == 0 ? Iz : Ioz;
                    C a0 = crs2<T>(p3, ev(Ix, Iy, zz), p1, ev(Iox, Iy, zz));
                    C a1 = crs2<T>(p3, ev(Ix, Ioy, zz), p1, ev(Iox, Ioy, zz));
                    pz[c] = crs2<T>(p3, a0, p1, a1);
                }
                pe = crs2<T>(p3, pz[0], p1, pz[1]);
            }
            U[p] = cadd<T>(u1, pe);
        }
        __syncthreads();
        for (int p = tid; p < Q.N; p += nth) {
            int i, j, k;
            tail_ijk(Q, p, i, j, k);
            C D = tail_diag<DIM, T>(Q, i, j, k, p);
            C mu = tail_Mu<DIM, T>(Q, U, D, i, j, k, p);
            Q.E[p] = cmadd<T>(U[p], jweight<T>(D, omega), csub<T>(Q.F[p], mu));
        }
        __syncthreads();
    }
    // write e at the top tail level
    {
        const TailPtr<T> Q = tail_ptr<DIM, T>(lds, tab, t0);
        for (int p = tid; p < Q.N; p += nth) stg(eg_top, p, Q.E[p]);
    }
}

// Waves k_coarse gives one coarsest solve of n unknowns (rows per wave as in
// coarse_rows_seg).
template <typename T> __host__ __device__ inline int coarse_waves(int n)
{
    const int seg = coarse_seg(n);
    const int rpb = coarse_slots<T>(seg) / seg;
    return (n + rpb - 1) / rpb;
}

// Coarsest solve e = Minv f with the rows spread over workgroups: wave w of
// the problem takes rows w, w + W, ... (W waves in all), each row summed
// exactly as in the tail kernel.  f is staged in LDS.  SEG = coarse_seg(Nc)
// of every problem in the launch.
template <typename T, int SEG>
__global__ __launch_bounds__(HH_WG) void k_coarse(Ctx cx)
{
    using C = V2<T>;
    const Tile tl = tile_of(cx);
    if (phase_of(cx, tl.prob) != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const LevelDev<T> *Lv = levels_of<T>(cx, pd);
    const int L = pd->nlev, n = pd->Nc;
    __shared__ C fs[HH_MAX_COARSE];
    const C *__restrict__ fg = Lv[L - 1].f;
    for (int i = threadIdx.x; i < n; i += HH_WG) fs[i] = ldg(fg, i);
    __syncthreads();
    const C *__restrict__ Minv = (const C *)(sizeof(T) == 8 ? (const void *)pd->Minv64 : (const void *)pd->Minv32);
    const int w = tl.idx * (HH_WG / 64) + (int)(threadIdx.x >> 6), W = coarse_waves<T>(n);
    if (w >= W) return;
    coarse_rows_seg<T, SEG>(Minv, fs, Lv[L - 1].e, n, w, W);
}

// ---------------------------------------------------------------------------
// Bi-CGSTAB passes (right preconditioned; s is kept in r).  Each pass
// reduces its dot products per chunk and finalises in its last workgroup.
// ---------------------------------------------------------------------------
#define CHUNK_P(s_) (base + threadIdx.x + (int64_t)HH_VWG * (s_))

// p = r + beta (p - omega v)
__global__ __launch_bounds__(HH_VWG) void k_bicg_p(Ctx cx)
{
    const Tile tl = tile_of(cx);
    const Ctrl ct = ctrl_of(cx, tl.prob);
    if (ct.phase != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const double2 beta = ct.beta, omega = ct.omega;
    double2 *__restrict__ pv = (double2 *)pd->vec[VS_P];
    const double2 *__restrict__ r = (const double2 *)pd->vec[VS_R];
    const double2 *__restrict__ v = (const double2 *)pd->vec[VS_V];
    const int64_t N = pd->N, base = (int64_t)tl.idx * HH_SPAN;
    double2 pr[HH_PER_SLOT], rr[HH_PER_SLOT], vr[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N) {
            pr[s] = ldg(pv, CHUNK_P(s));
            rr[s] = ldg(r, CHUNK_P(s));
            vr[s] = ldg(v, CHUNK_P(s));
        }
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N)
            stg(pv, CHUNK_P(s), cadd<double>(rr[s], cmul<double>(beta, csub<double>(pr[s], cmul<double>(omega, vr[s])))));
}

// v = H phat ; partial (rhat, v) ; finalise alpha
template <int DIM, typename SP>
__global__ __launch_bounds__(HH_VWG) void k_bicg_v(Ctx cx)
{
    const Tile tl = tile_of(cx);
    if (phase_of(cx, tl.prob) != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const HView h = hview(pd);
    const SP *__restrict__ ph = (const SP *)pd->vec[VS_PH];
    double2 *__restrict__ v = (double2 *)pd->vec[VS_V];
    const double2 *__restrict__ rh = (const double2 *)pd->vec[VS_RH];
    const int64_t base = (int64_t)tl.idx * HH_SPAN;
    double2 y[HH_PER_SLOT], a[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = CHUNK_P(s);
        if (p < h.N) {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            y[s] = stencil<DIM, double>(h, ph, i, j, k, p);
            a[s] = ldg(rh, p);
        }
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = CHUNK_P(s);
        if (p < h.N) {
            stg(v, p, y[s]);
            acc[0] = acc[0] + (a[s].x * y[s].x + a[s].y * y[s].y);
            acc[1] = acc[1] + (a[s].x * y[s].y - a[s].y * y[s].x);
        }
    }
    group_finish<2>(pd, tl.idx, acc);
}

// s = r - alpha v (in r) ; partial ||s||^2 (value 3, checked by the omega
// finaliser before it uses t)
__global__ __launch_bounds__(HH_VWG) void k_bicg_s(Ctx cx)
{
    const Tile tl = tile_of(cx);
    const Ctrl ct = ctrl_of(cx, tl.prob);
    if (ct.phase != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const double2 alpha = ct.alpha;
    double2 *__restrict__ r = (double2 *)pd->vec[VS_R];
    const double2 *__restrict__ v = (const double2 *)pd->vec[VS_V];
    const int64_t N = pd->N, base = (int64_t)tl.idx * HH_SPAN;
    double2 rr[HH_PER_SLOT], vr[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N) {
            rr[s] = ldg(r, CHUNK_P(s));
            vr[s] = ldg(v, CHUNK_P(s));
        }
    double acc[1] = {0.0};
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N) {
            double2 sv = csub<double>(rr[s], cmul<double>(alpha, vr[s]));
            stg(r, CHUNK_P(s), sv);
            acc[0] = acc[0] + (sv.x * sv.x + sv.y * sv.y);
        }
    group_finish<1>(pd, tl.idx, acc, 3);   // ||s||^2, finalised with omega
}

// t = H shat ; partials (t, s), (t, t) ; finalise omega
template <int DIM, typename SP>
__global__ __launch_bounds__(HH_VWG) void k_bicg_t(Ctx cx)
{
    const Tile tl = tile_of(cx);
    if (phase_of(cx, tl.prob) != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const HView h = hview(pd);
    const SP *__restrict__ sh = (const SP *)pd->vec[VS_SH];
    double2 *__restrict__ t = (double2 *)pd->vec[VS_T];
    const double2 *__restrict__ sv = (const double2 *)pd->vec[VS_R];
    const int64_t base = (int64_t)tl.idx * HH_SPAN;
    double2 y[HH_PER_SLOT], b[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = CHUNK_P(s);
        if (p < h.N) {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            y[s] = stencil<DIM, double>(h, sh, i, j, k, p);
            b[s] = ldg(sv, p);
        }
    }
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = CHUNK_P(s);
        if (p < h.N) {
            stg(t, p, y[s]);
            acc[0] = acc[0] + (y[s].x * b[s].x + y[s].y * b[s].y);
            acc[1] = acc[1] + (y[s].x * b[s].y - y[s].y * b[s].x);
            acc[2] = acc[2] + (y[s].x * y[s].x + y[s].y * y[s].y);
        }
    }
    group_finish<3>(pd, tl.idx, acc);
}

// x = x + alpha phat + omega shat ; r = s - omega t ; partials (rhat, r),
// ||r||^2 ; finalise rho/beta (half-step exit: x = x + alpha phat only)
template <typename SP>
__global__ __launch_bounds__(HH_VWG) void k_bicg_xr(Ctx cx)
{
    const Tile tl = tile_of(cx);
    const Ctrl ct = ctrl_of(cx, tl.prob);
    const int phase = ct.phase;
    if (phase != PH_RUN && phase != PH_HALF) return;
    const ProbDev *pd = cx.P + tl.prob;
    const double2 alpha = ct.alpha, omega = ct.omega;
    double2 *__restrict__ x = (double2 *)pd->vec[VS_X];
    const SP *__restrict__ ph = (const SP *)pd->vec[VS_PH];
    const SP *__restrict__ sh = (const SP *)pd->vec[VS_SH];
    double2 *__restrict__ r = (double2 *)pd->vec[VS_R];
    const double2 *__restrict__ t = (const double2 *)pd->vec[VS_T];
    const double2 *__restrict__ rh = (const double2 *)pd->vec[VS_RH];
    const int64_t N = pd->N, base = (int64_t)tl.idx * HH_SPAN;
    double acc[3] = {0.0, 0.0, 0.0};
    if (phase == PH_HALF) {
        double2 xr[HH_PER_SLOT], pr[HH_PER_SLOT];
#pragma unroll
        for (int s = 0; s < HH_PER_SLOT; ++s)
            if (CHUNK_P(s) < N) {
                xr[s] = ldg(x, CHUNK_P(s));
                pr[s] = ccvt<double>(ldg(ph, CHUNK_P(s)));
            }
#pragma unroll
        for (int s = 0; s < HH_PER_SLOT; ++s)
            if (CHUNK_P(s) < N) stg(x, CHUNK_P(s), cadd<double>(xr[s], cmul<double>(alpha, pr[s])));
    } else {
        double2 xr[HH_PER_SLOT], pr[HH_PER_SLOT], sr[HH_PER_SLOT], rr[HH_PER_SLOT], tr[HH_PER_SLOT], hr[HH_PER_SLOT];
#pragma unroll
        for (int s = 0; s < HH_PER_SLOT; ++s)
            if (CHUNK_P(s) < N) {
                const int64_t p = CHUNK_P(s);
                xr[s] = ldg(x, p);
                pr[s] = ccvt<double>(ldg(ph, p));
                sr[s] = ccvt<double>(ldg(sh, p));
                rr[s] = ldg(r, p);
                tr[s] = ldg(t, p);
                hr[s] = ldg(rh, p);
            }
#pragma unroll
        for (int s = 0; s < HH_PER_SLOT; ++s)
            if (CHUNK_P(s) < N) {
                const int64_t p = CHUNK_P(s);
                stg(x, p, cadd<double>(cadd<double>(xr[s], cmul<double>(alpha, pr[s])), cmul<double>(omega, sr[s])));
                double2 rn = csub<double>(rr[s], cmul<double>(omega, tr[s]));
                stg(r, p, rn);
                acc[0] = acc[0] + (hr[s].x * rn.x + hr[s].y * rn.y);
                acc[1] = acc[1] + (hr[s].x * rn.y - hr[s].y * rn.x);
                acc[2] = acc[2] + (rn.x * rn.x + rn.y * rn.y);
            }
    }
    group_finish<3>(pd, tl.idx, acc);
}

// out = b - H x.  mode 0 (Bi-CGSTAB start): out = r, also rhat = r, p = v = 0,
// partials (rhat, r) and ||r||^2, finalise INIT.  mode 1 (true residual):
// out = tmp, partial ||.||^2 in slot 2, finalise TRUE.  mode 2 (IDR start):
// out = r, partial ||r||^2, finalise IDR_INIT.
template <int DIM>
__global__ __launch_bounds__(HH_VWG) void k_resid(Ctx cx, int mode)
{
    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    const HView h = hview(pd);
    const double2 *__restrict__ x = (const double2 *)pd->vec[VS_X];
    const double2 *__restrict__ b = (const double2 *)pd->vec[VS_B];
    double2 *__restrict__ out = (double2 *)pd->vec[mode == 1 ? VS_TMP : VS_R];
    double2 *__restrict__ rh = (double2 *)pd->vec[VS_RH];
    double2 *__restrict__ pv = (double2 *)pd->vec[VS_P];
    double2 *__restrict__ v = (double2 *)pd->vec[VS_V];
    const int64_t base = (int64_t)tl.idx * HH_SPAN;
    double2 rr[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = CHUNK_P(s);
        if (p < h.N) {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            double2 hx = stencil<DIM, double>(h, x, i, j, k, p);
            rr[s] = csub<double>(ldg(b, p), hx);
        }
    }
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        const int64_t p = CHUNK_P(s);
        if (p < h.N) {
            const double2 rv = rr[s];
            stg(out, p, rv);
            if (mode == 0) {
                stg(rh, p, rv);
                stg(pv, p, cmk<double>(0.0, 0.0));
                stg(v, p, cmk<double>(0.0, 0.0));
                acc[0] = acc[0] + (rv.x * rv.x + rv.y * rv.y);
                acc[1] = acc[1] + (rv.x * rv.y - rv.y * rv.x);
            }
            acc[2] = acc[2] + (rv.x * rv.x + rv.y * rv.y);
        }
    }
    group_finish<3>(pd, tl.idx, acc);
}

// partial ||vec||^2 (slot 2) ; finalise ||b||
__global__ __launch_bounds__(HH_VWG) void k_norm(Ctx cx, int sel)
{
    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    const double2 *__restrict__ x = (const double2 *)pd->vec[sel];
    const int64_t N = pd->N, base = (int64_t)tl.idx * HH_SPAN;
    double2 xr[HH_PER_SLOT];
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N) xr[s] = ldg(x, CHUNK_P(s));
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N) acc[2] = acc[2] + (xr[s].x * xr[s].x + xr[s].y * xr[s].y);
    group_finish<3>(pd, tl.idx, acc);
}

// set a complex double vector to zero
__global__ __launch_bounds__(HH_VWG) void k_zero(Ctx cx, int sel)
{
    const Tile tl = tile_of(cx);
    const ProbDev *pd = cx.P + tl.prob;
    double2 *__restrict__ x = (double2 *)pd->vec[sel];
    const int64_t N = pd->N, base = (int64_t)tl.idx * HH_SPAN;
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s)
        if (CHUNK_P(s) < N) stg(x, CHUNK_P(s), cmk<double>(0.0, 0.0));
}

} // namespace hh
