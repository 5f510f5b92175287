// hh_select.hip -- automatic choice of the preconditioner's stretch or shift.
//
// Sec. 6.2 (remark on choosing the CSL and CSG parameters): start from a
// given CSG angle (or CSL imaginary shift), run multigrid alone on the
// preconditioner problem M u = f while watching the residual after each
// cycle, and reduce the angle (shift) towards the value at which the
// multigrid method just converges; that value then serves every later Krylov
// solve.  Here the candidates are start, start*factor, start*factor^2, ...;
// a candidate converges when ||f - M u_k|| / ||f|| drops below `reduction`
// within `max_cycles` cycles of u_k = u_{k-1} + V(f - M u_{k-1}), u_0 = 0
// (the tables' "cycles to reduce the residual by 7 orders"), and the search
// stops at the first candidate that does not.  The answer is the last one that
// did.
//
// Every cycle is hh_vcycle in complex double and every residual
// hh_apply_operator(M); the vector updates are exact elementwise adds and
// subtractions, and the norms use the fixed reduction order of the arithmetic
// contract (pairwise trees over 256-element chunks, then over the chunk sums
// zero-padded to a power of two), so the choice is reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "hh_common.h"
#include "hh_lib.h"
#include "hh_setup.h"

namespace {

#define SELCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return hh_fail(HH_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int SEL_WG = 256;      // one reduction chunk per workgroup
constexpr int SEL_TREE = 1024;   // block of the final tree

// u <- u + v
__global__ __launch_bounds__(SEL_WG) void k_sel_add(double2 *__restrict__ u, const double2 *__restrict__ v, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * SEL_WG + threadIdx.x;
    if (e < n) {
        const double2 a = u[e], b = v[e];
        u[e] = cmk<double>(a.x + b.x, a.y + b.y);
    }
}

// r <- f - y (y null: r <- f - 0) and the chunk's pairwise sum of |r|^2:
// slot t holds 0 + |r_e|^2 (0 past the end), summed by recursive halving.
__global__ __launch_bounds__(SEL_WG) void k_sel_resid(const double2 *__restrict__ f, const double2 *__restrict__ y,
                                                     double2 *__restrict__ r, int64_t n, double *__restrict__ part)
{
    __shared__ double s[SEL_WG];
    const int t = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x * SEL_WG + t;
    double acc = 0.0;
    if (e < n) {
        const double2 a = f[e], b = y ? y[e] : cmk<double>(0.0, 0.0);
        const double2 d = cmk<double>(a.x - b.x, a.y - b.y);
        if (r) r[e] = d;
        acc = acc + (d.x * d.x + d.y * d.y);
    }
    s[t] = acc;
    __syncthreads();
    for (int w = 1; w < SEL_WG; w *= 2) {
        if ((t & (2 * w - 1)) == 0) s[t] = s[t] + s[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = s[0];
}

// Pairwise sum of nch chunk sums zero-padded to np (a power of two): aligned
// blocks of SEL_TREE are subtrees of that tree, so their sums, then the tree
// over the block sums, give the same result.  One workgroup.
__global__ __launch_bounds__(SEL_TREE) void k_sel_tree(const double *__restrict__ part, int64_t nch, int64_t np,
                                                      double *__restrict__ out)
{
    __shared__ double s[SEL_TREE];
    __shared__ double blk[SEL_TREE];
    const int t = threadIdx.x;
    const int64_t bw = np < SEL_TREE ? np : SEL_TREE;   // block width
    const int64_t nb = np / bw;                        // blocks (<= SEL_TREE)
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t i = b * bw + t;
        s[t] = (t < bw && i < nch) ? part[i] : 0.0;
        __syncthreads();
        for (int w = 1; w < bw; w *= 2) {
            if (t < bw && (t & (2 * w - 1)) == 0) s[t] = s[t] + s[t + w];
            __syncthreads();
        }
        if (t == 0) blk[b] = s[0];
        __syncthreads();
    }
    for (int w = 1; w < nb; w *= 2) {
        if (t < nb && (t & (2 * w - 1)) == 0) blk[t] = blk[t] + blk[t + w];
        __syncthreads();
    }
    if (t == 0) out[0] = blk[0];
}

struct SelBuffers {
    double2 *f = nullptr, *u = nullptr, *r = nullptr, *v = nullptr;
    double *part = nullptr, *sum = nullptr;
    int64_t n = 0, nch = 0, np = 1;
};

// ||f - y|| (and r = f - y when r is given) in the contract's order.
hh_status sel_norm(const SelBuffers &B, const double2 *y, double2 *r, hipStream_t s, double &out)
{
    hipLaunchKernelGGL(k_sel_resid, dim3((unsigned)B.nch), dim3(SEL_WG), 0, s, B.f, y, r, B.n, B.part);
    hipLaunchKernelGGL(k_sel_tree, dim3(1), dim3(SEL_TREE), 0, s, B.part, B.nch, B.np, B.sum);
    SELCHK(hipGetLastError());
    double h = 0.0;
    SELCHK(hipMemcpyAsync(&h, B.sum, sizeof(double), hipMemcpyDeviceToHost, s));
    SELCHK(hipStreamSynchronize(s));
    out = std::sqrt(h);
    return HH_OK;
}

// Multigrid alone on M u = f with the grid's FP64 V-cycle; returns the cycles
// it took to reach `reduction` (0 if it did not within max_cycles) and the
// last relative residual.
hh_status sel_run(hh_grid *g, const SelBuffers &B, double fnorm, int max_cycles, double reduction, hipStream_t s,
                  int &cycles, double &rel)
{
    cycles = 0;
    rel = 1.0;
    SELCHK(hipMemsetAsync(B.u, 0, sizeof(double2) * B.n, s));
    SELCHK(hipMemcpyAsync(B.r, B.f, sizeof(double2) * B.n, hipMemcpyDeviceToDevice, s));
    const unsigned nb = (unsigned)((B.n + SEL_WG - 1) / SEL_WG);
    for (int k = 1; k <= max_cycles; ++k) {
        hh_status st = hh_vcycle(g, HH_C128, B.r, B.v, s);
        if (st != HH_OK) return st;
        hipLaunchKernelGGL(k_sel_add, dim3(nb), dim3(SEL_WG), 0, s, B.u, B.v, B.n);
        st = hh_apply_operator(g, HH_OP_M, HH_C128, B.u, B.v, s);
        if (st != HH_OK) return st;
        double nr = 0.0;
        st = sel_norm(B, B.v, B.r, s, nr);
        if (st != HH_OK) return st;
        rel = nr / fnorm;
        if (rel < reduction) {
            cycles = k;
            return HH_OK;
        }
        if (!std::isfinite(rel) || rel > 1e3) return HH_OK;   // diverging: no point in going on
    }
    return HH_OK;
}

void sel_free(SelBuffers &B)
{
    if (B.u) (void)hipFree(B.u);
    B = SelBuffers();
}

} // namespace

extern "C" hh_status hh_select_preconditioner(const hh_grid_desc *d, const hh_select_opts *o, const void *f,
                                              hh_select_result *res, double *trace, void *stream)
{
    if (!d || !o || !f || !res) return hh_fail(HH_ERR_ARG, "null argument");
    if (o->which != HH_SELECT_CSG_ANGLE && o->which != HH_SELECT_CSL_SHIFT)
        return hh_fail(HH_ERR_ARG, "which must be HH_SELECT_CSG_ANGLE or HH_SELECT_CSL_SHIFT");
    if (!(o->factor > 0.0 && o->factor < 1.0) || !(std::fabs(o->start) > 0.0) || !std::isfinite(o->start) ||
        o->max_cycles < 1 || !(o->reduction > 0.0 && o->reduction < 1.0) || o->max_steps < 1 || !(o->min_value >= 0.0))
        return hh_fail(HH_ERR_ARG, "need start != 0, 0 < factor < 1, min_value >= 0, max_cycles >= 1, "
                                   "0 < reduction < 1, max_steps >= 1");
    if (o->which == HH_SELECT_CSG_ANGLE && !(std::fabs(o->start) < 1.5707963267948966))
        return hh_fail(HH_ERR_ARG, "a CSG angle must lie in (-pi/2, pi/2)");
    memset(res, 0, sizeof *res);
    hipStream_t s = (hipStream_t)stream;
    hh_grid_desc cd = *d;
    cd.host_only = 0;
    if (o->which == HH_SELECT_CSG_ANGLE) {
        cd.csg_mode = cd.csg_mode == HH_CSL ? HH_CSG_UNIFORM : cd.csg_mode;
        cd.theta_csg = o->start;
    } else {
        cd.csg_mode = HH_CSL;
        cd.csl_shift[0] = 1.0;
        cd.csl_shift[1] = o->start;
    }
    int nl = 0, nc = 0;
    std::string err;
    hh_status st = desc_check(&cd, nl, nc, err);
    if (st != HH_OK) return hh_fail(st, "%s", err.c_str());
    if (cd.centering != HH_CELL) return hh_fail(HH_ERR_ARG, "a vertex-centred grid has no multigrid hierarchy");
    SelBuffers B;
    B.n = 1;
    for (int a = 0; a < cd.dim; ++a) B.n *= cd.n[a];
    B.nch = (B.n + SEL_WG - 1) / SEL_WG;
    while (B.np < B.nch) B.np *= 2;
    {
        const size_t vb = ((sizeof(double2) * B.n + 255) / 256) * 256;
        char *mem = nullptr;
        hipError_t e = hipMalloc((void **)&mem, 3 * vb + sizeof(double) * (B.nch + 64));
        if (e != hipSuccess) return hh_fail(HH_ERR_OOM, "hipMalloc for the selection vectors: %s", hipGetErrorString(e));
        B.u = (double2 *)mem;
        B.r = (double2 *)(mem + vb);
        B.v = (double2 *)(mem + 2 * vb);
        B.part = (double *)(mem + 3 * vb);
        B.sum = B.part + B.nch + 32;
    }
    B.f = (double2 *)f;
    double fnorm = 0.0;
    st = sel_norm(B, nullptr, nullptr, s, fnorm);
    if (st != HH_OK || !(fnorm > 0.0) || !std::isfinite(fnorm)) {
        sel_free(B);
        return st != HH_OK ? st : hh_fail(HH_ERR_ARG, "f must be finite and nonzero");
    }
    double value = o->start;
    bool found = false;
    for (int step = 0; step < o->max_steps && std::fabs(value) >= o->min_value; ++step) {
        if (o->which == HH_SELECT_CSG_ANGLE) {
            cd.theta_csg = value;
        } else {
            cd.csl_shift[0] = 1.0;
            cd.csl_shift[1] = value;
        }
        hh_grid *g = nullptr;
        st = hh_setup_grid(&cd, &g);
        if (st != HH_OK) break;
        int cycles = 0;
        double rel = 0.0;
        st = sel_run(g, B, fnorm, o->max_cycles, o->reduction, s, cycles, rel);
        hh_free_grid(g);
        if (st != HH_OK) break;
        if (trace) {
            trace[3 * step] = value;
            trace[3 * step + 1] = cycles;
            trace[3 * step + 2] = rel;
        }
        res->tried = step + 1;
        if (cycles == 0) break;
        found = true;
        res->value = value;
        res->cycles = cycles;
        res->factor = std::pow(rel, 1.0 / cycles);
        value = value * o->factor;
    }
    sel_free(B);
    if (st != HH_OK) return st;
    res->status = found ? HH_OK : HH_ERR_NOCONV;
    if (!found) return hh_fail(HH_ERR_NOCONV, "multigrid does not converge within %d cycles at the start value",
                               o->max_cycles);
    return HH_OK;
}
