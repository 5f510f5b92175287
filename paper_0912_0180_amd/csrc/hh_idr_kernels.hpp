// hh_idr_kernels.hpp -- IDR(s) passes (right preconditioned, x-space form of
// the prototype algorithm of Sonneveld & van Gijzen, with the
// minimal-residual omega), one step = one matvec (V-cycle + H apply):
//
//   P1  k_idr_v   start-up: v = r;  cycle step: q = -sum_j dR_j c_j, v = r + q
//   --  V-cycle   w = V(v)
//   P3  k_idr_t   start-up / k = 0: t = H w, partials (t, v), (t, t)
//                 k >= 1: dX_old = om w - sum_j dX_j c_j
//   fin           omega = (t, v) / (t, t)   (start-up and k = 0)
//   P4  k_idr_up  start-up: dX_k = om w, dR_k = -om t
//                 k = 0:    dR_old = q - om t, dX_old = om w - sum_j dX_j c_j
//                 k >= 1:   dR_old = -H dX_old
//                 then r += dR, x += dX; partials ||r||^2, P^H dR (and P^H r
//                 at start-up)
//   fin           residual check, G(:, old) = P^H dR, m += P^H dR, next c
//                 from the s x s LU solve G c = m
//
// Sums over columns run j = 0..s-1 left to right; the small solve uses LU
// with partial pivoting (first maximum of |re| + |im|) -- the same order as
// the CPU oracle, so FP64 iterates agree value for value.
#pragma once
#include "hh_kernels.hpp"

namespace hh {

__device__ int idr_nvals(const ProbDev *pd, int kind)
{
    const SolveState *st = pd->st;
    if (kind == FIN_IDR_OMEGA) return 3;
    if (kind == FIN_IDR_STEP) return st->startup >= 0 ? 1 + 4 * HH_MAX_S : 1 + 2 * st->s;
    return 1;
}

// s x s complex LU solve G c = m (G row major), same algorithm as the host
// setup's dense LU.  Returns false for an exactly singular pivot.
__device__ bool small_solve(const double2 *Gin, int s, const double2 *m, double2 *c)
{
    __shared__ double2 A[HH_MAX_S * HH_MAX_S];   // thread 0 only (keeps the solve out of scratch memory)
    __shared__ int perm[HH_MAX_S];
    for (int i = 0; i < s * s; ++i) A[i] = Gin[i];
    for (int i = 0; i < s; ++i) perm[i] = i;
    for (int k = 0; k < s; ++k) {
        int p = k;
        double best = fabs(A[k * s + k].x) + fabs(A[k * s + k].y);
        for (int i = k + 1; i < s; ++i) {
            double v = fabs(A[i * s + k].x) + fabs(A[i * s + k].y);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        if (best == 0.0) return false;
        if (p != k) {
            for (int j = 0; j < s; ++j) {
                double2 t = A[k * s + j];
                A[k * s + j] = A[p * s + j];
                A[p * s + j] = t;
            }
            int t = perm[k];
            perm[k] = perm[p];
            perm[p] = t;
        }
        const double2 piv = A[k * s + k];
        for (int i = k + 1; i < s; ++i) {
            double2 l = cdiv<double>(A[i * s + k], piv);
            A[i * s + k] = l;
            for (int j = k + 1; j < s; ++j) A[i * s + j] = csub<double>(A[i * s + j], cmul<double>(l, A[k * s + j]));
        }
    }
    for (int i = 0; i < s; ++i) {
        double2 v = m[perm[i]];
        for (int j = 0; j < i; ++j) v = csub<double>(v, cmul<double>(A[i * s + j], c[j]));
        c[i] = v;
    }
    for (int i = s - 1; i >= 0; --i) {
        double2 v = c[i];
        for (int j = i + 1; j < s; ++j) v = csub<double>(v, cmul<double>(A[i * s + j], c[j]));
        c[i] = cdiv<double>(v, A[i * s + i]);
    }
    return true;
}

__device__ void idr_finalize(const ProbDev *pd, SolveState *st, int kind, const double *v, int phase)
{
    const int s = st->s;
    if (kind == FIN_IDR_INIT) {
        st->phase = PH_RUN;
        st->reason = RS_NONE;
        st->startup = 0;
        st->kstep = 0;
        st->oldest = 0;
        st->om_idr = cmk<double>(1.0, 0.0);
        st->best_rel = INFINITY;
        st->best_mv = st->mv;
        return;
    }
    if (phase != PH_RUN) return;
    const int mode = st->startup >= 0 ? 0 : (st->kstep == 0 ? 1 : 2);
    if (kind == FIN_IDR_OMEGA) {
        if (mode == 2) return;
        st->mv += 1;
        double2 tv = cmk<double>(v[0], v[1]);
        double tt = v[2];
        if (!cfin(tv) || !isfinite(tt)) { stop(st, RS_NONFIN); return; }
        if (tt == 0.0) { stop(st, RS_BREAK); return; }
        st->om_idr = cmk<double>(tv.x / tt, tv.y / tt);
        return;
    }
    // FIN_IDR_STEP
    if (mode == 2) st->mv += 1;
    if (mode != 0) st->it += 1;
    const double rel = sqrt(v[0]) / st->bnorm;
    record(pd, st, rel);
    if (!isfinite(rel)) { stop(st, RS_NONFIN); return; }
    if (rel < st->tol) { stop(st, RS_CONV); return; }
    if (st->mv >= st->max_mv) { stop(st, RS_MAXMV); return; }
    if (st->guard && drift(rel, st->mv, st->best_rel, st->best_mv, st->drift_grow, st->drift_stall)) { stop(st, RS_DRIFT); return; }
    const int col = mode == 0 ? st->startup : st->oldest;
    for (int i = 0; i < s; ++i) {
        double2 dm = cmk<double>(v[1 + 2 * i], v[2 + 2 * i]);
        st->G[i * s + col] = dm;
        if (mode != 0) st->m[i] = cadd<double>(st->m[i], dm);
    }
    if (mode == 0) {
        st->startup += 1;
        if (st->startup < s) return;
        st->startup = -1;
        st->oldest = 0;
        st->kstep = 0;
        for (int i = 0; i < s; ++i) st->m[i] = cmk<double>(v[1 + 2 * HH_MAX_S + 2 * i], v[2 + 2 * HH_MAX_S + 2 * i]);
    } else {
        st->oldest = st->oldest + 1 == s ? 0 : st->oldest + 1;
        st->kstep = st->kstep + 1 == s + 1 ? 0 : st->kstep + 1;
    }
    if (!small_solve(st->G, s, st->m, st->c)) stop(st, RS_BREAK);
}

// P1: v = r (start-up) or q = -sum_j dR_j c_j, v = r + q
__global__ __launch_bounds__(HH_VWG) void k_idr_v(Ctx cx)
{
    const Tile tl = tile_of(cx);
    const Ctrl ct = ctrl_of(cx, tl.prob);
    if (ct.phase != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const int64_t N = pd->N, base = (int64_t)tl.idx * HH_SPAN;
    const double2 *__restrict__ r = (const double2 *)pd->vec[VS_R];
    double2 *__restrict__ v = (double2 *)pd->vec[VS_V];
    double2 *__restrict__ q = (double2 *)pd->vec[VS_Q];
    if (ct.mode == 0) {
        double2 rr[HH_PER_SLOT];
#pragma unroll
        for (int e = 0; e < HH_PER_SLOT; ++e)
            if (CHUNK_P(e) < N) rr[e] = ldg(r, CHUNK_P(e));
#pragma unroll
        for (int e = 0; e < HH_PER_SLOT; ++e)
            if (CHUNK_P(e) < N) stg(v, CHUNK_P(e), rr[e]);
        return;
    }
    const int ns = pd->nidr;
    const double2 *__restrict__ dR = pd->dR;
#pragma unroll
    for (int e = 0; e < HH_PER_SLOT; ++e) {
        const int64_t p = CHUNK_P(e);
        if (p < N) {
            double2 col[HH_MAX_S];
#pragma unroll
            for (int j = 0; j < HH_MAX_S; ++j)
                if (j < ns) col[j] = ldg(dR, (int64_t)j * N + p);
            const double2 rv = ldg(r, p);
            double2 acc = cmul<double>(col[0], ct.c[0]);
#pragma unroll
            for (int j = 1; j < HH_MAX_S; ++j)
                if (j < ns) acc = cadd<double>(acc, cmul<double>(col[j], ct.c[j]));
            const double2 qv = cmk<double>(-acc.x, -acc.y);
            stg(v, p, cadd<double>(rv, qv));
            if (ct.mode == 1) stg(q, p, qv);
        }
    }
}

// P3: t = H w with partials (t, v), (t, t)   (start-up, k = 0)
//     dX_old = om w - sum_j dX_j c_j          (k >= 1)
template <int DIM, typename SW>
__global__ __launch_bounds__(HH_VWG) void k_idr_t(Ctx cx)
{
    const Tile tl = tile_of(cx);
    const Ctrl ct = ctrl_of(cx, tl.prob);
    if (ct.phase != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const SW *__restrict__ w = (const SW *)pd->vec[VS_W];
    const int64_t base = (int64_t)tl.idx * HH_SPAN;
    if (ct.mode == 2) {
        const int64_t N = pd->N;
        const int ns = pd->nidr;
        double2 *__restrict__ dX = pd->dX;
#pragma unroll
        for (int e = 0; e < HH_PER_SLOT; ++e) {
            const int64_t p = CHUNK_P(e);
            if (p < N) {
                double2 col[HH_MAX_S];
#pragma unroll
                for (int j = 0; j < HH_MAX_S; ++j)
                    if (j < ns) col[j] = ldg(dX, (int64_t)j * N + p);
                const double2 wv = ld64(w, p);
                double2 acc = cmul<double>(col[0], ct.c[0]);
#pragma unroll
                for (int j = 1; j < HH_MAX_S; ++j)
                    if (j < ns) acc = cadd<double>(acc, cmul<double>(col[j], ct.c[j]));
                stg(dX, (int64_t)ct.old * N + p, csub<double>(cmul<double>(ct.om_idr, wv), acc));
            }
        }
        return;
    }
    const HView h = hview(pd);
    double2 *__restrict__ t = (double2 *)pd->vec[VS_T];
    const double2 *__restrict__ vv = (const double2 *)pd->vec[VS_V];
    double2 y[HH_PER_SLOT], b[HH_PER_SLOT];
#pragma unroll
    for (int e = 0; e < HH_PER_SLOT; ++e) {
        const int64_t p = CHUNK_P(e);
        if (p < h.N) {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            y[e] = stencil<DIM, double>(h, w, i, j, k, p);
            b[e] = ldg(vv, p);
        }
    }
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < HH_PER_SLOT; ++e) {
        const int64_t p = CHUNK_P(e);
        if (p < h.N) {
            stg(t, p, y[e]);
            acc[0] = acc[0] + (y[e].x * b[e].x + y[e].y * b[e].y);
            acc[1] = acc[1] + (y[e].x * b[e].y - y[e].y * b[e].x);
            acc[2] = acc[2] + (y[e].x * y[e].x + y[e].y * y[e].y);
        }
    }
    group_finish<3>(pd, tl.idx, acc);
}

// P4: the dR/dX column of this step, r += dR, x += dX; partials ||r||^2,
// P^H dR (and P^H r during start-up)
template <int DIM, typename SW>
__global__ __launch_bounds__(HH_VWG) void k_idr_up(Ctx cx)
{
    constexpr int NV = 1 + 4 * HH_MAX_S;
    const Tile tl = tile_of(cx);
    const Ctrl ct = ctrl_of(cx, tl.prob);
    if (ct.phase != PH_RUN) return;
    const ProbDev *pd = cx.P + tl.prob;
    const HView h = hview(pd);
    const int64_t N = h.N, base = (int64_t)tl.idx * HH_SPAN;
    const int ns = pd->nidr, mode = ct.mode;
    const double2 om = ct.om_idr;
    const SW *__restrict__ w = (const SW *)pd->vec[VS_W];
    double2 *__restrict__ x = (double2 *)pd->vec[VS_X];
    double2 *__restrict__ r = (double2 *)pd->vec[VS_R];
    const double2 *__restrict__ t = (const double2 *)pd->vec[VS_T];
    const double2 *__restrict__ q = (const double2 *)pd->vec[VS_Q];
    double2 *__restrict__ dR = pd->dR;
    double2 *__restrict__ dX = pd->dX;
    const double2 *__restrict__ Pm = pd->P;
    double2 *__restrict__ dRo = dR + (int64_t)ct.old * N;
    double2 *__restrict__ dXo = dX + (int64_t)ct.old * N;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int e = 0; e < HH_PER_SLOT; ++e) {
        const int64_t p = CHUNK_P(e);
        if (p >= N) continue;
        double2 dr, dx;
        if (mode == 0) {
            const double2 ot = cmul<double>(om, ldg(t, p));
            dx = cmul<double>(om, ld64(w, p));
            dr = cmk<double>(-ot.x, -ot.y);
        } else if (mode == 1) {
            double2 col[HH_MAX_S];
#pragma unroll
            for (int j = 0; j < HH_MAX_S; ++j)
                if (j < ns) col[j] = ldg(dX, (int64_t)j * N + p);
            const double2 tv = ldg(t, p), qv = ldg(q, p), wv = ld64(w, p);
            double2 ax = cmul<double>(col[0], ct.c[0]);
#pragma unroll
            for (int j = 1; j < HH_MAX_S; ++j)
                if (j < ns) ax = cadd<double>(ax, cmul<double>(col[j], ct.c[j]));
            dr = csub<double>(qv, cmul<double>(om, tv));
            dx = csub<double>(cmul<double>(om, wv), ax);
        } else {
            int i, j, k;
            split(p, h.nx, h.ny, h.fx, h.fxy, i, j, k);
            const double2 hv = stencil<DIM, double>(h, dXo, i, j, k, p);
            dr = cmk<double>(-hv.x, -hv.y);
            dx = ldg(dXo, p);
        }
        if (mode != 2) stg(dXo, p, dx);
        stg(dRo, p, dr);
        const double2 rn = cadd<double>(ldg(r, p), dr);
        stg(r, p, rn);
        stg(x, p, cadd<double>(ldg(x, p), dx));
        acc[0] = acc[0] + (rn.x * rn.x + rn.y * rn.y);
#pragma unroll
        for (int i = 0; i < HH_MAX_S; ++i) {
            if (i < ns) {
                const double2 pv = ldg(Pm, (int64_t)i * N + p);
                acc[1 + 2 * i] = acc[1 + 2 * i] + (pv.x * dr.x + pv.y * dr.y);
                acc[2 + 2 * i] = acc[2 + 2 * i] + (pv.x * dr.y - pv.y * dr.x);
                if (mode == 0) {
                    acc[1 + 2 * HH_MAX_S + 2 * i] = acc[1 + 2 * HH_MAX_S + 2 * i] + (pv.x * rn.x + pv.y * rn.y);
                    acc[2 + 2 * HH_MAX_S + 2 * i] = acc[2 + 2 * HH_MAX_S + 2 * i] + (pv.x * rn.y - pv.y * rn.x);
                }
            }
        }
    }
    if (mode == 0) {
        group_finish<NV>(pd, tl.idx, acc);
    } else {
        double a2[1 + 2 * HH_MAX_S];
#pragma unroll
        for (int k = 0; k < 1 + 2 * HH_MAX_S; ++k) a2[k] = acc[k];
        group_finish<1 + 2 * HH_MAX_S>(pd, tl.idx, a2);
    }
}

} // namespace hh
