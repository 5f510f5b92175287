// hh_kernels.hpp -- gfx950 kernels of the CSG-preconditioned Helmholtz solver.
//
// Every kernel takes the device array of problem descriptors and a tile list
// (problem id, tile index); one workgroup of 256 threads (4 x wave64) handles
// one tile, so a single launch covers any number of independent problems.
// Kernels whose problem is not in the running phase return at once.
//
// Arithmetic follows a fixed operation order (no FMA contraction; the build
// passes -ffp-contract=off), so FP64 results are reproducible run to run and
// independent of how problems are batched:
//   complex multiply (ar*br - ai*bi, ar*bi + ai*br); Jacobi weight
//   g = omega conj(D)/|D|^2 with D = (d_x + d_y + d_z) - phi; stencil
//   y = D u - a_x u_w - c_x u_e - a_y u_s - c_y u_n - a_z u_d - c_z u_u;
//   full weighting (1,3,3,1)/8 applied x, then y, then z; prolongation
//   3/4 near + 1/4 far applied x, then y, then z; reductions over chunks of
//   2048 elements, thread slot t summing elements t + 256 j (j = 0..7) in
//   order, slots combined by a pairwise tree (wave butterfly, then
//   (w0 + w1) + (w2 + w3)), chunk partials by a pairwise tree.
#include "hh_common.h"

namespace hh {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Pairwise tree over the 256 thread slots of the workgroup; thread 0 writes
// the NV sums to out[0..NV).
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], double *out)
{
    __shared__ double red[4 * NV];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = v[q] + __shfl_xor(v[q], off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[w * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] = (red[q] + red[NV + q]) + (red[2 * NV + q] + red[3 * NV + q]);
}

// Pairwise sum of v[0..n) with zero padding to a power of two >= 256, by one
// workgroup; returns the sum in thread 0.  Each thread sums its contiguous
// segment with the iterative (binary counter) form of the pairwise tree.
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
        double x = e < n ? v[(int64_t)e * stride] : 0.0;
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
// helpers
// ---------------------------------------------------------------------------
template <typename T> __device__ inline const LevelDev<T> *levels(const ProbDev &pd);
template <> __device__ inline const LevelDev<double> *levels<double>(const ProbDev &pd) { return pd.L64; }
template <> __device__ inline const LevelDev<float> *levels<float>(const ProbDev &pd) { return pd.L32; }

__device__ inline bool running(const ProbDev &pd) { return pd.st == nullptr || pd.st->phase == PH_RUN; }

template <typename S> __device__ inline double2 ld64(const S *p, int64_t i) { return ccvt<double>(p[i]); }

// y = H x at fine point (i, j, k), FP64 ECS coefficients; x of storage type S.
template <int DIM, typename S>
__device__ inline double2 applyH_at(const ProbDev &pd, const S *x, int i, int j, int k, int64_t p)
{
    const int nx = pd.n[0], ny = pd.n[1], nz = pd.n[2];
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const double2 zero = cmk<double>(0.0, 0.0);
    double2 d = pd.dH[0][i];
    d = cadd<double>(d, pd.dH[1][j]);
    if (DIM == 3) d = cadd<double>(d, pd.dH[2][k]);
    double2 D = cmk<double>(d.x - pd.phi[p], d.y);
    double2 t = cmul<double>(D, ld64(x, p));
    double2 uw = i > 0 ? ld64(x, p - 1) : zero, ue = i < nx - 1 ? ld64(x, p + 1) : zero;
    t = csub<double>(t, cmul<double>(pd.aH[0][i], uw));
    t = csub<double>(t, cmul<double>(pd.cH[0][i], ue));
    double2 us = j > 0 ? ld64(x, p - sy) : zero, un = j < ny - 1 ? ld64(x, p + sy) : zero;
    t = csub<double>(t, cmul<double>(pd.aH[1][j], us));
    t = csub<double>(t, cmul<double>(pd.cH[1][j], un));
    if (DIM == 3) {
        double2 ud = k > 0 ? ld64(x, p - sz) : zero, uu = k < nz - 1 ? ld64(x, p + sz) : zero;
        t = csub<double>(t, cmul<double>(pd.aH[2][k], ud));
        t = csub<double>(t, cmul<double>(pd.cH[2][k], uu));
    }
    return t;
}

// y = M x on level `lev` in precision T at point (i,j,k); x of type V2<T>.
template <int DIM, typename T>
__device__ inline V2<T> applyM_at(const LevelDev<T> &L, const V2<T> *x, int i, int j, int k, int64_t p)
{
    using C = V2<T>;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const C zero = cmk<T>(0, 0);
    C d = L.d[0][i];
    d = cadd<T>(d, L.d[1][j]);
    if (DIM == 3) d = cadd<T>(d, L.d[2][k]);
    C D = cmk<T>(d.x - L.phi[p], d.y);
    C t = cmul<T>(D, x[p]);
    t = csub<T>(t, cmul<T>(L.a[0][i], i > 0 ? x[p - 1] : zero));
    t = csub<T>(t, cmul<T>(L.c[0][i], i < nx - 1 ? x[p + 1] : zero));
    t = csub<T>(t, cmul<T>(L.a[1][j], j > 0 ? x[p - sy] : zero));
    t = csub<T>(t, cmul<T>(L.c[1][j], j < ny - 1 ? x[p + sy] : zero));
    if (DIM == 3) {
        t = csub<T>(t, cmul<T>(L.a[2][k], k > 0 ? x[p - sz] : zero));
        t = csub<T>(t, cmul<T>(L.c[2][k], k < nz - 1 ? x[p + sz] : zero));
    }
    return t;
}

__device__ inline void coords(const ProbDev &pd, int64_t p, int &i, int &j, int &k)
{
    uint32_t q = fdiv((uint32_t)p, pd.fx);
    i = (int)((uint32_t)p - q * (uint32_t)pd.n[0]);
    k = (int)fdiv((uint32_t)p, pd.fxy);
    j = (int)(q - (uint32_t)k * (uint32_t)pd.n[1]);
}

// ---------------------------------------------------------------------------
// operator apply (standalone): y = H x or y = M x on the finest level
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(HH_WG) void k_applyH(const ProbDev *P, const Tile *tiles, const void *xp, void *yp)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    const double2 *x = (const double2 *)xp;
    double2 *y = (double2 *)yp;
    const int64_t base = (int64_t)tl.idx * HH_CHUNK;
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        int64_t p = base + threadIdx.x + (int64_t)HH_WG * s;
        if (p < pd.N) {
            int i, j, k;
            coords(pd, p, i, j, k);
            y[p] = applyH_at<DIM>(pd, x, i, j, k, p);
        }
    }
}

template <int DIM, typename T>
__global__ __launch_bounds__(HH_WG) void k_applyM(const ProbDev *P, const Tile *tiles, const void *xp, void *yp)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    const LevelDev<T> &L = levels<T>(pd)[0];
    const V2<T> *x = (const V2<T> *)xp;
    V2<T> *y = (V2<T> *)yp;
    const int64_t base = (int64_t)tl.idx * HH_CHUNK;
#pragma unroll
    for (int s = 0; s < HH_PER_SLOT; ++s) {
        int64_t p = base + threadIdx.x + (int64_t)HH_WG * s;
        if (p < pd.N) {
            int i, j, k;
            coords(pd, p, i, j, k);
            y[p] = applyM_at<DIM, T>(L, x, i, j, k, p);
        }
    }
}

// ---------------------------------------------------------------------------
// fused V-cycle down-leg on level lev -> lev+1:
//   u1 = g f (one Jacobi sweep from zero), r = f - M u1, f_{lev+1} = R r.
// Only f_{lev+1} is written; u1 is recomputed by the up-leg.
// Tile = a box of coarse points; LDS holds f, phi and u1 on the fine box
// with a halo of 2 (restriction footprint + stencil).
// ---------------------------------------------------------------------------
template <int DIM, typename T, typename TF>
__global__ __launch_bounds__(HH_WG) void k_vdown(const ProbDev *P, const Tile *tiles, int lev, int fsel, const void *fptr)
{
    using C = V2<T>;
    constexpr int CX = VTile<DIM, T>::X, CY = VTile<DIM, T>::Y, CZ = VTile<DIM, T>::Z;
    constexpr int RX = 2 * CX + 4, RY = 2 * CY + 4, RZ = DIM == 3 ? 2 * CZ + 4 : 1;
    constexpr int RN = RX * RY * RZ;
    __shared__ C U[RN];
    __shared__ C F[RN];
    __shared__ T PH[RN];
    __shared__ C A[3][RX > RY ? (RX > RZ ? RX : RZ) : (RY > RZ ? RY : RZ)];
    __shared__ C Cc[3][RX > RY ? (RX > RZ ? RX : RZ) : (RY > RZ ? RY : RZ)];
    __shared__ C Dd[3][RX > RY ? (RX > RZ ? RX : RZ) : (RY > RZ ? RY : RZ)];

    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const LevelDev<T> &Lf = levels<T>(pd)[lev];
    const LevelDev<T> &Lc = levels<T>(pd)[lev + 1];
    const int nfx = Lf.n[0], nfy = Lf.n[1], nfz = Lf.n[2];
    const int ncx = Lc.n[0], ncy = Lc.n[1], ncz = Lc.n[2];
    const int tx = (ncx + CX - 1) / CX, ty = (ncy + CY - 1) / CY;
    int t = tl.idx;
    const int bx = t % tx;
    t /= tx;
    const int by = t % ty, bz = t / ty;
    const int c0x = bx * CX, c0y = by * CY, c0z = DIM == 3 ? bz * CZ : 0;
    const int ox = 2 * c0x - 2, oy = 2 * c0y - 2, oz = DIM == 3 ? 2 * c0z - 2 : 0;
    const TF *f = lev == 0 ? (const TF *)(fptr ? fptr : pd.vec[fsel]) : (const TF *)Lf.f;
    const T omega = (T)pd.omega;
    const C zero = cmk<T>(0, 0);
    const int64_t sy = nfx, sz = (int64_t)nfx * nfy;

    // per-axis coefficients of the box
    for (int l = threadIdx.x; l < RX + RY + RZ; l += HH_WG) {
        int ax = l < RX ? 0 : (l < RX + RY ? 1 : 2);
        int q = ax == 0 ? l : (ax == 1 ? l - RX : l - RX - RY);
        int g = (ax == 0 ? ox : (ax == 1 ? oy : oz)) + q;
        int nn = ax == 0 ? nfx : (ax == 1 ? nfy : nfz);
        bool in = (ax < DIM) && g >= 0 && g < nn;
        A[ax][q] = in ? Lf.a[ax][g] : zero;
        Cc[ax][q] = in ? Lf.c[ax][g] : zero;
        Dd[ax][q] = in ? Lf.d[ax][g] : zero;
    }
    __syncthreads();
    // step 1: f, phi and u1 = g f on the whole box
    for (int l = threadIdx.x; l < RN; l += HH_WG) {
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        C fv = zero, u1 = zero;
        T ph = 0;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz))) {
            const int64_t p = gx + sy * gy + sz * gz;
            fv = ccvt<T>(f[p]);
            ph = Lf.phi[p];
            C d = cadd<T>(Dd[0][lx], Dd[1][ly]);
            if (DIM == 3) d = cadd<T>(d, Dd[2][lz]);
            C D = cmk<T>(d.x - ph, d.y);
            T q = omega / (D.x * D.x + D.y * D.y);
            C gw = cmk<T>(D.x * q, -(D.y * q));
            u1 = cmul<T>(gw, fv);
        }
        U[l] = u1;
        F[l] = fv;
        PH[l] = ph;
    }
    __syncthreads();
    // step 2: r = f - M u1 on the box minus its outer ring, in place in F
    {
        constexpr int QX = RX - 2, QY = RY - 2, QZ = DIM == 3 ? RZ - 2 : 1;
        for (int r = threadIdx.x; r < QX * QY * QZ; r += HH_WG) {
            const int lx = 1 + r % QX, ly = 1 + (r / QX) % QY, lz = (DIM == 3 ? 1 : 0) + r / (QX * QY);
            const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
            const int l = lx + RX * (ly + RY * lz);
            C res = zero;
            if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz))) {
                C d = cadd<T>(Dd[0][lx], Dd[1][ly]);
                if (DIM == 3) d = cadd<T>(d, Dd[2][lz]);
                C D = cmk<T>(d.x - PH[l], d.y);
                C mu = cmul<T>(D, U[l]);
                mu = csub<T>(mu, cmul<T>(A[0][lx], U[l - 1]));
                mu = csub<T>(mu, cmul<T>(Cc[0][lx], U[l + 1]));
                mu = csub<T>(mu, cmul<T>(A[1][ly], U[l - RX]));
                mu = csub<T>(mu, cmul<T>(Cc[1][ly], U[l + RX]));
                if (DIM == 3) {
                    mu = csub<T>(mu, cmul<T>(A[2][lz], U[l - RX * RY]));
                    mu = csub<T>(mu, cmul<T>(Cc[2][lz], U[l + RX * RY]));
                }
                res = csub<T>(F[l], mu);
            }
            F[l] = res;
        }
    }
    __syncthreads();
    // step 3: full weighting, x then y then z
    const T w0 = (T)0.125, w1 = (T)0.375;
    for (int cl = threadIdx.x; cl < CX * CY * CZ; cl += HH_WG) {
        const int ix = cl % CX, iy = (cl / CX) % CY, iz = cl / (CX * CY);
        const int I = c0x + ix, J = c0y + iy, K = c0z + iz;
        if (I >= ncx || J >= ncy || (DIM == 3 && K >= ncz)) continue;
        const int bxl = 2 * ix + 1, byl = 2 * iy + 1, bzl = DIM == 3 ? 2 * iz + 1 : 0;
        C acc_z = zero;
        for (int c = 0; c < (DIM == 3 ? 4 : 1); ++c) {
            const T wz = (c == 0 || c == 3) ? w0 : w1;
            C acc_y = zero;
            for (int b = 0; b < 4; ++b) {
                const T wy = (b == 0 || b == 3) ? w0 : w1;
                const C *row = &F[bxl + RX * ((byl + b) + RY * (bzl + c))];
                C sx = crs<T>(w0, row[0]);
                sx = cadd<T>(sx, crs<T>(w1, row[1]));
                sx = cadd<T>(sx, crs<T>(w1, row[2]));
                sx = cadd<T>(sx, crs<T>(w0, row[3]));
                acc_y = b == 0 ? crs<T>(wy, sx) : cadd<T>(acc_y, crs<T>(wy, sx));
            }
            if (DIM == 3) acc_z = c == 0 ? crs<T>(wz, acc_y) : cadd<T>(acc_z, crs<T>(wz, acc_y));
            else acc_z = acc_y;
        }
        Lc.f[I + (int64_t)ncx * (J + (int64_t)ncy * K)] = acc_z;
    }
}

// ---------------------------------------------------------------------------
// fused V-cycle up-leg on level lev (coarse correction from lev+1):
//   u2 = g f + P e_{lev+1},  u = u2 + g (f - M u2).
// Output: e_lev (lev >= 1) or the output vector (lev == 0, storage TO).
// ---------------------------------------------------------------------------
template <int DIM, typename T, typename TF, typename TO>
__global__ __launch_bounds__(HH_WG) void k_vup(const ProbDev *P, const Tile *tiles, int lev, int fsel, int osel, const void *fptr, void *optr)
{
    using C = V2<T>;
    constexpr int CX = VTile<DIM, T>::X, CY = VTile<DIM, T>::Y, CZ = VTile<DIM, T>::Z;
    constexpr int FX = 2 * CX, FY = 2 * CY, FZ = DIM == 3 ? 2 * CZ : 1;
    constexpr int RX = FX + 2, RY = FY + 2, RZ = DIM == 3 ? FZ + 2 : 1;
    constexpr int RN = RX * RY * RZ;
    constexpr int EX = CX + 4, EY = CY + 4, EZ = DIM == 3 ? CZ + 4 : 1;
    constexpr int EN = EX * EY * EZ;
    constexpr int RM = RX > RY ? (RX > RZ ? RX : RZ) : (RY > RZ ? RY : RZ);
    __shared__ C U[RN];
    __shared__ C F[RN];
    __shared__ T PH[RN];
    __shared__ C E[EN];
    __shared__ C A[3][RM];
    __shared__ C Cc[3][RM];
    __shared__ C Dd[3][RM];

    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const LevelDev<T> &Lf = levels<T>(pd)[lev];
    const LevelDev<T> &Lc = levels<T>(pd)[lev + 1];
    const int nfx = Lf.n[0], nfy = Lf.n[1], nfz = Lf.n[2];
    const int ncx = Lc.n[0], ncy = Lc.n[1], ncz = Lc.n[2];
    const int tx = (nfx + FX - 1) / FX, ty = (nfy + FY - 1) / FY;
    int t = tl.idx;
    const int bx = t % tx;
    t /= tx;
    const int by = t % ty, bz = t / ty;
    const int f0x = bx * FX, f0y = by * FY, f0z = DIM == 3 ? bz * FZ : 0;
    const int ox = f0x - 1, oy = f0y - 1, oz = DIM == 3 ? f0z - 1 : 0;
    const int ex0 = (f0x >> 1) - 2, ey0 = (f0y >> 1) - 2, ez0 = DIM == 3 ? (f0z >> 1) - 2 : 0;
    const TF *f = lev == 0 ? (const TF *)(fptr ? fptr : pd.vec[fsel]) : (const TF *)Lf.f;
    const T omega = (T)pd.omega;
    const C zero = cmk<T>(0, 0);
    const int64_t sy = nfx, sz = (int64_t)nfx * nfy;

    for (int l = threadIdx.x; l < EN; l += HH_WG) {
        const int lx = l % EX, ly = (l / EX) % EY, lz = l / (EX * EY);
        const int gx = ex0 + lx, gy = ey0 + ly, gz = ez0 + lz;
        C v = zero;
        if (gx >= 0 && gx < ncx && gy >= 0 && gy < ncy && (DIM == 2 || (gz >= 0 && gz < ncz)))
            v = Lc.e[gx + (int64_t)ncx * (gy + (int64_t)ncy * gz)];
        E[l] = v;
    }
    for (int l = threadIdx.x; l < RX + RY + RZ; l += HH_WG) {
        int ax = l < RX ? 0 : (l < RX + RY ? 1 : 2);
        int q = ax == 0 ? l : (ax == 1 ? l - RX : l - RX - RY);
        int g = (ax == 0 ? ox : (ax == 1 ? oy : oz)) + q;
        int nn = ax == 0 ? nfx : (ax == 1 ? nfy : nfz);
        bool in = (ax < DIM) && g >= 0 && g < nn;
        A[ax][q] = in ? Lf.a[ax][g] : zero;
        Cc[ax][q] = in ? Lf.c[ax][g] : zero;
        Dd[ax][q] = in ? Lf.d[ax][g] : zero;
    }
    __syncthreads();
    const T p3 = (T)0.75, p1 = (T)0.25;
    // step 1: u2 = g f + P e on the tile plus a halo of one
    for (int l = threadIdx.x; l < RN; l += HH_WG) {
        const int lx = l % RX, ly = (l / RX) % RY, lz = l / (RX * RY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        C fv = zero, u2 = zero;
        T ph = 0;
        if (gx >= 0 && gx < nfx && gy >= 0 && gy < nfy && (DIM == 2 || (gz >= 0 && gz < nfz))) {
            const int64_t p = gx + sy * gy + sz * gz;
            fv = ccvt<T>(f[p]);
            ph = Lf.phi[p];
            C d = cadd<T>(Dd[0][lx], Dd[1][ly]);
            if (DIM == 3) d = cadd<T>(d, Dd[2][lz]);
            C D = cmk<T>(d.x - ph, d.y);
            T q = omega / (D.x * D.x + D.y * D.y);
            C gw = cmk<T>(D.x * q, -(D.y * q));
            C u1 = cmul<T>(gw, fv);
            // prolongation: per axis near = g>>1, far = near -/+ 1
            const int Ix = (gx >> 1) - ex0, Iox = ((gx & 1) ? (gx >> 1) + 1 : (gx >> 1) - 1) - ex0;
            const int Iy = (gy >> 1) - ey0, Ioy = ((gy & 1) ? (gy >> 1) + 1 : (gy >> 1) - 1) - ey0;
            C pe;
            if (DIM == 2) {
                C a0 = cadd<T>(crs<T>(p3, E[Ix + EX * Iy]), crs<T>(p1, E[Iox + EX * Iy]));
                C a1 = cadd<T>(crs<T>(p3, E[Ix + EX * Ioy]), crs<T>(p1, E[Iox + EX * Ioy]));
                pe = cadd<T>(crs<T>(p3, a0), crs<T>(p1, a1));
            } else {
                const int Iz = (gz >> 1) - ez0, Ioz = ((gz & 1) ? (gz >> 1) + 1 : (gz >> 1) - 1) - ez0;
                C pz[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int zz = c == 0 ? Iz : Ioz;
                    C a0 = cadd<T>(crs<T>(p3, E[Ix + EX * (Iy + EY * zz)]), crs<T>(p1, E[Iox + EX * (Iy + EY * zz)]));
                    C a1 = cadd<T>(crs<T>(p3, E[Ix + EX * (Ioy + EY * zz)]), crs<T>(p1, E[Iox + EX * (Ioy + EY * zz)]));
                    pz[c] = cadd<T>(crs<T>(p3, a0), crs<T>(p1, a1));
                }
                pe = cadd<T>(crs<T>(p3, pz[0]), crs<T>(p1, pz[1]));
            }
            u2 = cadd<T>(u1, pe);
        }
        U[l] = u2;
        F[l] = fv;
        PH[l] = ph;
    }
    __syncthreads();
    // step 2: post-smoothing on the tile
    TO *outv = lev == 0 ? (TO *)(optr ? optr : pd.vec[osel]) : nullptr;
    for (int r = threadIdx.x; r < FX * FY * FZ; r += HH_WG) {
        const int lx = 1 + r % FX, ly = 1 + (r / FX) % FY, lz = (DIM == 3 ? 1 : 0) + r / (FX * FY);
        const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
        if (gx >= nfx || gy >= nfy || (DIM == 3 && gz >= nfz)) continue;
        const int l = lx + RX * (ly + RY * lz);
        C d = cadd<T>(Dd[0][lx], Dd[1][ly]);
        if (DIM == 3) d = cadd<T>(d, Dd[2][lz]);
        C D = cmk<T>(d.x - PH[l], d.y);
        T q = omega / (D.x * D.x + D.y * D.y);
        C gw = cmk<T>(D.x * q, -(D.y * q));
        C mu = cmul<T>(D, U[l]);
        mu = csub<T>(mu, cmul<T>(A[0][lx], U[l - 1]));
        mu = csub<T>(mu, cmul<T>(Cc[0][lx], U[l + 1]));
        mu = csub<T>(mu, cmul<T>(A[1][ly], U[l - RX]));
        mu = csub<T>(mu, cmul<T>(Cc[1][ly], U[l + RX]));
        if (DIM == 3) {
            mu = csub<T>(mu, cmul<T>(A[2][lz], U[l - RX * RY]));
            mu = csub<T>(mu, cmul<T>(Cc[2][lz], U[l + RX * RY]));
        }
        C u = cadd<T>(U[l], cmul<T>(gw, csub<T>(F[l], mu)));
        const int64_t p = gx + sy * gy + sz * gz;
        if (lev == 0) {
            TO o;
            o.x = u.x;
            o.y = u.y;
            outv[p] = o;
        } else {
            Lf.e[p] = u;
        }
    }
}

// ---------------------------------------------------------------------------
// coarsest solve e = Minv f: one wave per row, pairwise over the row
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(HH_WG) void k_coarse(const ProbDev *P, const Tile *tiles)
{
    using C = V2<T>;
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const LevelDev<T> &L = levels<T>(pd)[pd.nlev - 1];
    const C *Minv = (const C *)(sizeof(T) == 8 ? (const void *)pd.Minv64 : (const void *)pd.Minv32);
    const int n = pd.Nc;
    const int row = tl.idx * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    int np = 64;
    while (np < n) np <<= 1;
    const int seg = np >> 6;   // 1..16
    T re[16], im[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        re[i] = 0;
        im[i] = 0;
        const int col = lane * seg + i;
        if (i < seg && col < n) {
            C pr = cmul<T>(Minv[(int64_t)row * n + col], L.f[col]);
            re[i] = pr.x;
            im[i] = pr.y;
        }
    }
#pragma unroll
    for (int w = 1; w < 16; w <<= 1) {
        if (w < seg) {
#pragma unroll
            for (int i = 0; i + w < 16; i += 2 * w) {
                re[i] = re[i] + re[i + w];
                im[i] = im[i] + im[i + w];
            }
        }
    }
    T sr = re[0], si = im[0];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        sr = sr + __shfl_xor(sr, off, 64);
        si = si + __shfl_xor(si, off, 64);
    }
    if (lane == 0) L.e[row] = cmk<T>(sr, si);
}

// ---------------------------------------------------------------------------
// Bi-CGSTAB passes (right preconditioned; s is kept in r)
// ---------------------------------------------------------------------------
#define CHUNK_LOOP(...)                                                               \
    const int64_t base = (int64_t)tl.idx * HH_CHUNK;                                  \
    _Pragma("unroll") for (int s_ = 0; s_ < HH_PER_SLOT; ++s_)                        \
    {                                                                                 \
        const int64_t p = base + threadIdx.x + (int64_t)HH_WG * s_;                   \
        if (p < pd.N) { __VA_ARGS__ }                                                 \
    }

// p = r + beta (p - omega v)
__global__ __launch_bounds__(HH_WG) void k_bicg_p(const ProbDev *P, const Tile *tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const double2 beta = pd.st->beta, omega = pd.st->omega;
    double2 *pv = (double2 *)pd.vec[VS_P];
    const double2 *r = (const double2 *)pd.vec[VS_R], *v = (const double2 *)pd.vec[VS_V];
    CHUNK_LOOP(pv[p] = cadd<double>(r[p], cmul<double>(beta, csub<double>(pv[p], cmul<double>(omega, v[p]))));)
}

// v = H phat ; partial (rhat, v)
template <int DIM, typename SP>
__global__ __launch_bounds__(HH_WG) void k_bicg_v(const ProbDev *P, const Tile *tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const SP *ph = (const SP *)pd.vec[VS_PH];
    double2 *v = (double2 *)pd.vec[VS_V];
    const double2 *rh = (const double2 *)pd.vec[VS_RH];
    double acc[2] = {0.0, 0.0};
    CHUNK_LOOP({
        int i, j, k;
        coords(pd, p, i, j, k);
        double2 y = applyH_at<DIM>(pd, ph, i, j, k, p);
        v[p] = y;
        double2 a = rh[p];
        acc[0] = acc[0] + (a.x * y.x + a.y * y.y);
        acc[1] = acc[1] + (a.x * y.y - a.y * y.x);
    })
    block_reduce<2>(acc, pd.part + (int64_t)tl.idx * HH_NPART);
}

// s = r - alpha v (in r) ; partial ||s||^2
__global__ __launch_bounds__(HH_WG) void k_bicg_s(const ProbDev *P, const Tile *tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const double2 alpha = pd.st->alpha;
    double2 *r = (double2 *)pd.vec[VS_R];
    const double2 *v = (const double2 *)pd.vec[VS_V];
    double acc[1] = {0.0};
    CHUNK_LOOP({
        double2 s = csub<double>(r[p], cmul<double>(alpha, v[p]));
        r[p] = s;
        acc[0] = acc[0] + (s.x * s.x + s.y * s.y);
    })
    block_reduce<1>(acc, pd.part + (int64_t)tl.idx * HH_NPART);
}

// t = H shat ; partials (t, s), (t, t)
template <int DIM, typename SP>
__global__ __launch_bounds__(HH_WG) void k_bicg_t(const ProbDev *P, const Tile *tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    if (!running(pd)) return;
    const SP *sh = (const SP *)pd.vec[VS_SH];
    double2 *t = (double2 *)pd.vec[VS_T];
    const double2 *s = (const double2 *)pd.vec[VS_R];
    double acc[3] = {0.0, 0.0, 0.0};
    CHUNK_LOOP({
        int i, j, k;
        coords(pd, p, i, j, k);
        double2 y = applyH_at<DIM>(pd, sh, i, j, k, p);
        t[p] = y;
        double2 b = s[p];
        acc[0] = acc[0] + (y.x * b.x + y.y * b.y);
        acc[1] = acc[1] + (y.x * b.y - y.y * b.x);
        acc[2] = acc[2] + (y.x * y.x + y.y * y.y);
    })
    block_reduce<3>(acc, pd.part + (int64_t)tl.idx * HH_NPART);
}

// x = x + alpha phat + omega shat ; r = s - omega t ; partials (rhat, r), ||r||^2
// (half-step exit: x = x + alpha phat only)
template <typename SP>
__global__ __launch_bounds__(HH_WG) void k_bicg_xr(const ProbDev *P, const Tile *tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    const int phase = pd.st->phase;
    if (phase != PH_RUN && phase != PH_HALF) return;
    const double2 alpha = pd.st->alpha, omega = pd.st->omega;
    double2 *x = (double2 *)pd.vec[VS_X];
    const SP *ph = (const SP *)pd.vec[VS_PH];
    if (phase == PH_HALF) {
        CHUNK_LOOP(x[p] = cadd<double>(x[p], cmul<double>(alpha, ld64(ph, p)));)
        return;
    }
    const SP *sh = (const SP *)pd.vec[VS_SH];
    double2 *r = (double2 *)pd.vec[VS_R];
    const double2 *t = (const double2 *)pd.vec[VS_T], *rh = (const double2 *)pd.vec[VS_RH];
    double acc[3] = {0.0, 0.0, 0.0};
    CHUNK_LOOP({
        x[p] = cadd<double>(cadd<double>(x[p], cmul<double>(alpha, ld64(ph, p))), cmul<double>(omega, ld64(sh, p)));
        double2 rn = csub<double>(r[p], cmul<double>(omega, t[p]));
        r[p] = rn;
        double2 a = rh[p];
        acc[0] = acc[0] + (a.x * rn.x + a.y * rn.y);
        acc[1] = acc[1] + (a.x * rn.y - a.y * rn.x);
        acc[2] = acc[2] + (rn.x * rn.x + rn.y * rn.y);
    })
    block_reduce<3>(acc, pd.part + (int64_t)tl.idx * HH_NPART);
}

// out = b - H x.  mode 0 (Bi-CGSTAB start): out = r, also rhat = r, p = v = 0,
// partials (rhat, r) and ||r||^2.  mode 1 (true residual): out = tmp,
// partial ||.||^2 in slot 2.  mode 2 (IDR start): out = r, partial ||r||^2.
template <int DIM>
__global__ __launch_bounds__(HH_WG) void k_resid(const ProbDev *P, const Tile *tiles, int mode)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    const double2 *x = (const double2 *)pd.vec[VS_X], *b = (const double2 *)pd.vec[VS_B];
    double2 *out = (double2 *)pd.vec[mode == 1 ? VS_TMP : VS_R];
    double2 *rh = (double2 *)pd.vec[VS_RH], *pv = (double2 *)pd.vec[VS_P], *v = (double2 *)pd.vec[VS_V];
    double acc[3] = {0.0, 0.0, 0.0};
    CHUNK_LOOP({
        int i, j, k;
        coords(pd, p, i, j, k);
        double2 hx = applyH_at<DIM>(pd, x, i, j, k, p);
        double2 r = csub<double>(b[p], hx);
        out[p] = r;
        if (mode == 0) {
            rh[p] = r;
            pv[p] = cmk<double>(0.0, 0.0);
            v[p] = cmk<double>(0.0, 0.0);
            acc[0] = acc[0] + (r.x * r.x + r.y * r.y);
            acc[1] = acc[1] + (r.x * r.y - r.y * r.x);
        }
        acc[2] = acc[2] + (r.x * r.x + r.y * r.y);
    })
    block_reduce<3>(acc, pd.part + (int64_t)tl.idx * HH_NPART);
}

// partial ||vec||^2 (slot 2) ; used for ||b||
__global__ __launch_bounds__(HH_WG) void k_norm(const ProbDev *P, const Tile *tiles, int sel)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    const double2 *x = (const double2 *)pd.vec[sel];
    double acc[3] = {0.0, 0.0, 0.0};
    CHUNK_LOOP({
        double2 a = x[p];
        acc[2] = acc[2] + (a.x * a.x + a.y * a.y);
    })
    block_reduce<3>(acc, pd.part + (int64_t)tl.idx * HH_NPART);
}

// set a complex double vector to zero
__global__ __launch_bounds__(HH_WG) void k_zero(const ProbDev *P, const Tile *tiles, int sel)
{
    const Tile tl = tiles[blockIdx.x];
    const ProbDev &pd = P[tl.prob];
    double2 *x = (double2 *)pd.vec[sel];
    CHUNK_LOOP(x[p] = cmk<double>(0.0, 0.0);)
}

// ---------------------------------------------------------------------------
// finalisation: one workgroup per problem reduces the chunk partials and
// advances the scalar state.
// ---------------------------------------------------------------------------
enum FinKind { FIN_BNORM = 0, FIN_INIT, FIN_ALPHA, FIN_S, FIN_OMEGA, FIN_RHO, FIN_TRUE };

__device__ inline bool fin_ok(double v) { return isfinite(v); }
__device__ inline bool cfin(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__device__ inline void stop(SolveState *st, int reason)
{
    st->phase = PH_STOP;
    st->reason = reason;
}

__device__ inline void record(const ProbDev &pd, SolveState *st, double rel)
{
    st->rel = rel;
    if (pd.hist && st->mv - 1 < st->hist_len && st->mv >= 1) pd.hist[st->mv - 1] = rel;
}

__global__ __launch_bounds__(HH_WG) void k_fin(const ProbDev *P, const int *probs, int kind)
{
    const ProbDev &pd = P[probs[blockIdx.x]];
    SolveState *st = pd.st;
    const int phase = st->phase;
    if (kind == FIN_RHO) {
        if (phase != PH_RUN && phase != PH_HALF) return;
    } else if (kind != FIN_BNORM && kind != FIN_INIT && kind != FIN_TRUE) {
        if (phase != PH_RUN) return;
    }
    __syncthreads();
    double s[3] = {0.0, 0.0, 0.0};
    const int nv = (kind == FIN_S || kind == FIN_BNORM || kind == FIN_TRUE) ? 1 : (kind == FIN_ALPHA ? 2 : 3);
    const int first = (kind == FIN_S) ? 0 : ((kind == FIN_BNORM || kind == FIN_TRUE) ? 2 : 0);
    for (int q = 0; q < nv; ++q) s[q] = pairwise_wg(pd.part + first + q, HH_NPART, pd.nchunk);
    if (threadIdx.x != 0) return;
    switch (kind) {
    case FIN_BNORM:
        st->bnorm = sqrt(s[0]);
        break;
    case FIN_TRUE:
        st->true_rel = sqrt(s[0]) / st->bnorm;
        break;
    case FIN_INIT: {
        // start (or restart) of Bi-CGSTAB: rho = alpha = omega = 1, then the
        // first beta from rho1 = (rhat, r)
        const double2 one = cmk<double>(1.0, 0.0);
        st->rho = one;
        st->alpha = one;
        st->omega = one;
        st->phase = PH_RUN;
        st->reason = RS_NONE;
        double2 rho1 = cmk<double>(s[0], s[1]);
        if (!cfin(rho1)) { stop(st, RS_NONFIN); break; }
        if (rho1.x == 0.0 && rho1.y == 0.0) { stop(st, RS_BREAK); break; }
        st->beta = cmul<double>(cdiv<double>(rho1, st->rho), cdiv<double>(st->alpha, st->omega));
        st->rho = rho1;
        break;
    }
    case FIN_ALPHA: {
        st->mv += 1;
        double2 rv = cmk<double>(s[0], s[1]);
        if (!cfin(rv)) { stop(st, RS_NONFIN); break; }
        if (rv.x == 0.0 && rv.y == 0.0) { stop(st, RS_BREAK); break; }
        st->alpha = cdiv<double>(st->rho, rv);
        break;
    }
    case FIN_S: {
        double rel = sqrt(s[0]) / st->bnorm;
        record(pd, st, rel);
        if (!fin_ok(rel)) { stop(st, RS_NONFIN); break; }
        if (rel < st->tol) { st->phase = PH_HALF; st->reason = RS_CONV; break; }
        if (st->mv >= st->max_mv) { st->phase = PH_HALF; st->reason = RS_MAXMV; break; }
        break;
    }
    case FIN_OMEGA: {
        st->mv += 1;
        double2 ts = cmk<double>(s[0], s[1]);
        double tt = s[2];
        if (!cfin(ts) || !fin_ok(tt)) { stop(st, RS_NONFIN); break; }
        if (tt == 0.0) { stop(st, RS_BREAK); break; }
        st->omega = cmk<double>(ts.x / tt, ts.y / tt);
        break;
    }
    case FIN_RHO: {
        st->it += 1;
        if (phase == PH_HALF) { st->phase = PH_STOP; break; }
        double rel = sqrt(s[2]) / st->bnorm;
        record(pd, st, rel);
        if (!fin_ok(rel)) { stop(st, RS_NONFIN); break; }
        if (rel < st->tol) { stop(st, RS_CONV); break; }
        if (st->omega.x == 0.0 && st->omega.y == 0.0) { stop(st, RS_BREAK); break; }
        if (st->mv >= st->max_mv) { stop(st, RS_MAXMV); break; }
        double2 rho1 = cmk<double>(s[0], s[1]);
        if (!cfin(rho1)) { stop(st, RS_NONFIN); break; }
        if (rho1.x == 0.0 && rho1.y == 0.0) { stop(st, RS_BREAK); break; }
        st->beta = cmul<double>(cdiv<double>(rho1, st->rho), cdiv<double>(st->alpha, st->omega));
        st->rho = rho1;
        break;
    }
    }
}

} // namespace hh
