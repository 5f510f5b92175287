// hh_solve.hip -- host drivers of the right-preconditioned Krylov solves.
//
// The device runs every pass for all problems of a batch at once; the host
// only watches the per-problem state blocks between iterations and decides
// restarts from the true residual (paper Sec. 6.2: the solve stops on the
// relative residual; here the final ||b - H x|| / ||b|| is checked in FP64
// and a false stop or a breakdown restarts from the true residual).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hh_lib.h"

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return hh_fail(HH_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

void workspace_release(Workspace &w)
{
    if (w.mem) (void)hipFree(w.mem);
    w = Workspace();
}

static hh_status workspace_ensure(hh_grid *g, int method, bool fp32, int s, int hist_len)
{
    Workspace &w = g->ws;
    if (w.mem && w.method == method && w.fp32 == (int)fp32 && w.s >= s && w.hist_cap >= hist_len) return HH_OK;
    workspace_release(w);
    const int64_t N = g->hs.lev[0].N;
    const size_t c16 = al256(sizeof(double2) * N), clow = al256((fp32 ? sizeof(float2) : sizeof(double2)) * N);
    const int nch = ceil_div(N, HH_CHUNK);
    size_t bytes = al256(sizeof(double) * HH_NPART * nch) + al256(sizeof(SolveState)) + al256(sizeof(double) * std::max(hist_len, 1));
    if (method == HH_METHOD_BICGSTAB) bytes += 5 * c16 + 2 * clow;
    else bytes += 4 * c16 + clow + 2 * (size_t)s * c16;
    hipError_t e = hipMalloc(&w.mem, bytes);
    if (e != hipSuccess) {
        w.mem = nullptr;
        return hh_fail(HH_ERR_OOM, "hipMalloc(%zu) for the solve work space: %s", bytes, hipGetErrorString(e));
    }
    w.bytes = bytes;
    w.method = method;
    w.fp32 = fp32;
    w.s = s;
    w.hist_cap = hist_len;
    char *c = (char *)w.mem;
    auto take = [&](size_t b) { void *p = c; c += b; return p; };
    w.part = (double *)take(al256(sizeof(double) * HH_NPART * nch));
    w.st = (SolveState *)take(al256(sizeof(SolveState)));
    w.hist = (double *)take(al256(sizeof(double) * std::max(hist_len, 1)));
    if (method == HH_METHOD_BICGSTAB) {
        w.r = (double2 *)take(c16);
        w.rh = (double2 *)take(c16);
        w.p = (double2 *)take(c16);
        w.v = (double2 *)take(c16);
        w.t = (double2 *)take(c16);
        w.ph = take(clow);
        w.sh = take(clow);
    } else {
        w.r = (double2 *)take(c16);
        w.v = (double2 *)take(c16);
        w.t = (double2 *)take(c16);
        w.q = (double2 *)take(c16);
        w.wlow = take(clow);
        w.dR = (double2 *)take((size_t)s * c16);
        w.dX = (double2 *)take((size_t)s * c16);
    }
    return HH_OK;
}

static void fill_solve_prob(hh_grid *g, const hh_solve_opts *o, const void *b, void *x, ProbDev &pd)
{
    grid_fill_prob(g, pd);
    Workspace &w = g->ws;
    pd.vec[VS_X] = x;
    pd.vec[VS_B] = (void *)b;
    pd.vec[VS_R] = w.r;
    pd.vec[VS_RH] = w.rh;
    pd.vec[VS_P] = w.p;
    pd.vec[VS_V] = w.v;
    pd.vec[VS_T] = w.t;
    pd.vec[VS_TMP] = w.t;
    pd.vec[VS_PH] = w.ph;
    pd.vec[VS_SH] = w.sh;
    pd.vec[VS_W] = w.wlow;
    pd.vec[VS_Q] = w.q;
    pd.dR = w.dR;
    pd.dX = w.dX;
    pd.P = (const double2 *)o->idr_P;
    pd.part = w.part;
    pd.st = w.st;
    pd.hist = o->history && o->history_len > 0 ? w.hist : nullptr;
    pd.nidr = o->method == HH_METHOD_IDR ? o->s : 0;
}

namespace {

struct Ctl {
    hh_grid *g;
    const hh_solve_opts *o;
    hh_solve_info *info;
    int status = HH_OK;
    bool done = false;
    int restarts = 0;
    int chunk0 = 0, nchunk = 0;   // range of the problem in the plan's chunk list
};

// device scratch for tile lists of subsets of the batch
struct Subset {
    Tile *t = nullptr;
    int *p = nullptr;
    void *mem = nullptr;
    std::vector<Tile> ht;
    std::vector<int> hp;
    ~Subset() { if (mem) (void)hipFree(mem); }
    hh_status alloc(int nchunks, int nprob)
    {
        size_t b = al256(sizeof(Tile) * nchunks) + al256(sizeof(int) * nprob);
        if (hipMalloc(&mem, b) != hipSuccess) return hh_fail(HH_ERR_OOM, "hipMalloc for subset lists");
        t = (Tile *)mem;
        p = (int *)((char *)mem + al256(sizeof(Tile) * nchunks));
        return HH_OK;
    }
    hh_status set(const std::vector<Ctl> &C, const std::vector<int> &which, hipStream_t s)
    {
        ht.clear();
        hp.clear();
        for (int q : which) {
            for (int i = 0; i < C[q].nchunk; ++i) ht.push_back(Tile{q, i});
            hp.push_back(q);
        }
        if (!ht.empty()) HIPCHK(hipMemcpyAsync(t, ht.data(), sizeof(Tile) * ht.size(), hipMemcpyHostToDevice, s));
        if (!hp.empty()) HIPCHK(hipMemcpyAsync(p, hp.data(), sizeof(int) * hp.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        return HH_OK;
    }
    DevList list() const { DevList d; d.t = t; d.n = (int)ht.size(); return d; }
};

hh_status read_states(const std::vector<Ctl> &C, std::vector<SolveState> &S, hipStream_t s)
{
    for (size_t q = 0; q < C.size(); ++q)
        HIPCHK(hipMemcpyAsync(&S[q], C[q].g->ws.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

} // namespace

// Bi-CGSTAB and IDR(s) share the driver: start (r = b - H x and the method's
// initial scalars), iterations of the method's passes, true-residual checks
// and restarts.
static hh_status solve_krylov(std::vector<Ctl> &C, Plan &pl, const void *const *b, void *const *x, hipStream_t s,
                              int method)
{
    const int init_mode = method == HH_METHOD_BICGSTAB ? 0 : 2;
    const int init_fin = method == HH_METHOD_BICGSTAB ? 1 /*FIN_INIT*/ : 10 /*FIN_IDR_INIT*/;
    auto iterate1 = [&]() {
        if (method == HH_METHOD_BICGSTAB) launch_bicg_iteration(pl, s);
        else launch_idr_step(pl, s);
    };
    // K iterations per check of the control blocks, replayed from a graph
    const char *ek = getenv("HH_ITERS_PER_CHECK");
    const int K = ek ? std::max(1, atoi(ek)) : 4;
    const bool use_graph = !getenv("HH_NO_GRAPH");
    const void *key = C[0].g->ws.mem;
    auto iterate = [&]() -> hh_status {
        if (!use_graph) {
            for (int k = 0; k < K; ++k) iterate1();
            return HH_OK;
        }
        if (!pl.gexec || pl.gmethod != method || pl.gK != K || pl.gkey != key) {
            if (pl.gexec) {
                HIPCHK(hipGraphExecDestroy(pl.gexec));
                pl.gexec = nullptr;
            }
            hipGraph_t graph;
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < K; ++k) iterate1();
            HIPCHK(hipStreamEndCapture(s, &graph));
            hipError_t e = hipGraphInstantiate(&pl.gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hh_fail(HH_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
            pl.gmethod = method;
            pl.gK = K;
            pl.gkey = key;
        }
        HIPCHK(hipGraphLaunch(pl.gexec, s));
        return HH_OK;
    };
    auto read_ctrl = [&]() -> hh_status {
        HIPCHK(hipMemcpyAsync(pl.hctrl, pl.ctrl, sizeof(Ctrl) * C.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return HH_OK;
    };
    const int nb = (int)C.size();
    std::vector<ProbDev> hp(nb);
    std::vector<Ctrl> hc(nb);
    for (int q = 0; q < nb; ++q) {
        fill_solve_prob(C[q].g, C[q].o, b[q], x[q], hp[q]);
        hp[q].ctrl = pl.ctrl + q;
        memset(&hc[q], 0, sizeof(Ctrl));
        hc[q].phase = PH_IDLE;
    }
    pl.host = hp;
    HIPCHK(hipMemcpyAsync(pl.probs, hp.data(), sizeof(ProbDev) * nb, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(pl.ctrl, hc.data(), sizeof(Ctrl) * nb, hipMemcpyHostToDevice, s));
    int total_chunks = 0;
    for (int q = 0; q < nb; ++q) {
        C[q].chunk0 = total_chunks;
        C[q].nchunk = ceil_div(C[q].g->hs.lev[0].N, HH_CHUNK);
        total_chunks += C[q].nchunk;
        SolveState st;
        memset(&st, 0, sizeof st);
        st.phase = PH_IDLE;
        st.tol = C[q].o->tol;
        st.max_mv = C[q].o->max_matvec;
        st.hist_len = C[q].o->history ? C[q].o->history_len : 0;
        st.s = method == HH_METHOD_IDR ? C[q].o->s : 0;
        st.startup = -1;
        HIPCHK(hipMemcpyAsync(C[q].g->ws.st, &st, sizeof st, hipMemcpyHostToDevice, s));
    }
    Subset sub;
    hh_status rc = sub.alloc(total_chunks, nb);
    if (rc != HH_OK) return rc;
    std::vector<SolveState> S(nb);
    // ||b||
    launch_norm(pl, pl.chunks, VS_B, s);
    launch_fin(pl, pl.fin, pl.nfin, 0 /*FIN_BNORM*/, s);
    HIPCHK(hipGetLastError());
    rc = read_states(C, S, s);
    if (rc != HH_OK) return rc;
    std::vector<int> zero_x, start;
    for (int q = 0; q < nb; ++q) {
        if (!C[q].o->x0_given) zero_x.push_back(q);
        if (!std::isfinite(S[q].bnorm)) {
            C[q].done = true;
            C[q].status = HH_ERR_NONFINITE;
        } else if (S[q].bnorm == 0.0) {
            C[q].done = true;
            C[q].status = HH_OK;
            if (C[q].o->x0_given) zero_x.push_back(q);
        } else {
            start.push_back(q);
        }
    }
    if (!zero_x.empty()) {
        rc = sub.set(C, zero_x, s);
        if (rc != HH_OK) return rc;
        launch_zero(pl, sub.list(), VS_X, s);
    }
    if (!start.empty()) {
        rc = sub.set(C, start, s);
        if (rc != HH_OK) return rc;
        launch_resid(pl, sub.list(), init_mode, s);
        launch_fin(pl, sub.p, (int)start.size(), init_fin, s);
    }
    HIPCHK(hipGetLastError());
    int active = (int)start.size();
    while (active > 0) {
        rc = iterate();
        if (rc != HH_OK) return rc;
        HIPCHK(hipGetLastError());
        rc = read_ctrl();
        if (rc != HH_OK) return rc;
        std::vector<int> verify;
        for (int q = 0; q < nb; ++q) {
            if (C[q].done || pl.hctrl[q].phase != PH_STOP) continue;
            S[q].reason = pl.hctrl[q].reason;
            if (S[q].reason == RS_NONFIN) {
                C[q].done = true;
                C[q].status = HH_ERR_NONFINITE;
                --active;
            } else if (S[q].reason == RS_MAXMV) {
                C[q].done = true;
                C[q].status = HH_ERR_NOCONV;
                --active;
            } else {
                verify.push_back(q);
            }
        }
        if (verify.empty()) continue;
        rc = sub.set(C, verify, s);
        if (rc != HH_OK) return rc;
        launch_resid(pl, sub.list(), 1, s);
        launch_fin(pl, sub.p, (int)verify.size(), 6 /*FIN_TRUE*/, s);
        HIPCHK(hipGetLastError());
        rc = read_states(C, S, s);
        if (rc != HH_OK) return rc;
        std::vector<int> restart;
        for (int q : verify) {
            if (S[q].reason == RS_CONV && S[q].true_rel < C[q].o->tol) {
                C[q].done = true;
                C[q].status = HH_OK;
                --active;
            } else if (C[q].restarts >= C[q].o->max_restarts) {
                C[q].done = true;
                C[q].status = S[q].reason == RS_BREAK ? HH_ERR_BREAKDOWN : HH_ERR_NOCONV;
                --active;
            } else {
                C[q].restarts++;
                restart.push_back(q);
            }
        }
        if (!restart.empty()) {
            rc = sub.set(C, restart, s);
            if (rc != HH_OK) return rc;
            launch_resid(pl, sub.list(), init_mode, s);
            launch_fin(pl, sub.p, (int)restart.size(), init_fin, s);
            HIPCHK(hipGetLastError());
        }
    }
    // final true residual of every finished problem with finite data
    std::vector<int> fin;
    for (int q = 0; q < nb; ++q)
        if (C[q].status != HH_ERR_NONFINITE && S[q].bnorm > 0.0) fin.push_back(q);
    if (!fin.empty()) {
        rc = sub.set(C, fin, s);
        if (rc != HH_OK) return rc;
        launch_resid(pl, sub.list(), 1, s);
        launch_fin(pl, sub.p, (int)fin.size(), 6 /*FIN_TRUE*/, s);
        HIPCHK(hipGetLastError());
    }
    rc = read_states(C, S, s);
    if (rc != HH_OK) return rc;
    for (int q = 0; q < nb; ++q) {
        hh_solve_info &in = *C[q].info;
        in.status = C[q].status;
        in.matvecs = S[q].mv;
        in.iterations = S[q].it;
        in.restarts = C[q].restarts;
        in.rel_res_recurrence = S[q].bnorm > 0.0 ? S[q].rel : 0.0;
        in.rel_res_true = S[q].bnorm > 0.0 ? S[q].true_rel : 0.0;
        if (C[q].status == HH_ERR_NONFINITE) in.rel_res_true = NAN;
        const hh_solve_opts *o = C[q].o;
        if (o->history && o->history_len > 0) {
            int n = std::min(S[q].mv, o->history_len);
            if (n > 0) HIPCHK(hipMemcpy(o->history, C[q].g->ws.hist, sizeof(double) * n, hipMemcpyDeviceToHost));
        }
    }
    return HH_OK;
}

static hh_status check_opts(const hh_grid *g, const hh_solve_opts *o)
{
    if (!o) return hh_fail(HH_ERR_ARG, "null options");
    if (o->method != HH_METHOD_BICGSTAB && o->method != HH_METHOD_IDR) return hh_fail(HH_ERR_ARG, "unknown method %d", o->method);
    if (o->method == HH_METHOD_IDR && (o->s < 1 || o->s > HH_MAX_S || !o->idr_P))
        return hh_fail(HH_ERR_ARG, "IDR(s) needs 1 <= s <= %d and a shadow space", HH_MAX_S);
    if (!(o->tol > 0.0) || o->max_matvec < 1 || o->max_restarts < 0) return hh_fail(HH_ERR_ARG, "need tol > 0, max_matvec >= 1, max_restarts >= 0");
    if (o->vcycle_prec != HH_C128 && o->vcycle_prec != HH_C64) return hh_fail(HH_ERR_ARG, "unknown vcycle precision");
    if (g->host_only) return hh_fail(HH_ERR_ARG, "grid was built host-only");
    return HH_OK;
}


extern "C" hh_status hh_solve_batch(hh_grid *const *g, int32_t count, const hh_solve_opts *o, const void *const *b,
                                    void *const *x, hh_solve_info *info, void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!g || !o || !b || !x || !info || count < 1) return hh_fail(HH_ERR_ARG, "null argument or empty batch");
    hipStream_t s = (hipStream_t)stream;
    std::vector<Ctl> C(count);
    for (int q = 0; q < count; ++q) {
        if (!g[q] || !b[q] || !x[q]) return hh_fail(HH_ERR_ARG, "problem %d: null grid or vector", q);
        hh_status rc = check_opts(g[q], &o[q]);
        if (rc != HH_OK) return rc;
        if (o[q].method != o[0].method || o[q].vcycle_prec != o[0].vcycle_prec)
            return hh_fail(HH_ERR_ARG, "all problems of a batch need the same method and V-cycle precision");
        if (g[q]->hs.dim != g[0]->hs.dim) return hh_fail(HH_ERR_ARG, "all problems of a batch need the same dimension");
        for (int r = 0; r < q; ++r)
            if (g[r] == g[q]) return hh_fail(HH_ERR_ARG, "grid used twice in one batch");
        C[q].g = g[q];
        C[q].o = &o[q];
        C[q].info = &info[q];
        memset(&info[q], 0, sizeof(hh_solve_info));
    }
    const bool fp32 = o[0].vcycle_prec == HH_C64;
    for (int q = 0; q < count; ++q) {
        hh_status rc = workspace_ensure(g[q], o[q].method, fp32, o[q].method == HH_METHOD_IDR ? o[q].s : 0,
                                        o[q].history ? o[q].history_len : 0);
        if (rc != HH_OK) return rc;
    }
    Plan local;
    Plan *pl = &local;
    if (count == 1) {
        if (g[0]->plan_fp32 != (int)fp32 || !g[0]->plan.mem) {
            std::vector<const hh_grid *> G{g[0]};
            hh_status rc = plan_build(g[0]->plan, G, fp32);
            if (rc != HH_OK) return rc;
            g[0]->plan_fp32 = fp32;
        }
        pl = &g[0]->plan;
    } else {
        std::vector<const hh_grid *> G(g, g + count);
        hh_status rc = plan_build(local, G, fp32);
        if (rc != HH_OK) return rc;
    }
    // the solve runs on the plan's own stream (graphs cannot be captured on
    // the null stream), ordered after the caller's stream by an event
    if (!pl->stream) HIPCHK(hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking));
    if (!pl->hctrl) HIPCHK(hipHostMalloc((void **)&pl->hctrl, sizeof(Ctrl) * pl->count, 0));
    {
        hipEvent_t ev;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, s));
        HIPCHK(hipStreamWaitEvent(pl->stream, ev, 0));
        HIPCHK(hipEventDestroy(ev));
    }
    hh_status rc = solve_krylov(C, *pl, b, x, pl->stream, o[0].method);
    HIPCHK(hipStreamSynchronize(pl->stream));
    if (pl == &local) plan_release(local);
    if (rc != HH_OK) return rc;
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    hh_status first = HH_OK;
    for (int q = 0; q < count; ++q) {
        info[q].seconds = secs;
        if (first == HH_OK && info[q].status != HH_OK) first = (hh_status)info[q].status;
    }
    if (first != HH_OK) hh_fail(first, "problem did not converge (status %d)", (int)first);
    return first;
}

extern "C" hh_status hh_solve(hh_grid *g, const hh_solve_opts *o, const void *b, void *x, hh_solve_info *info, void *stream)
{
    hh_grid *gg[1] = {g};
    const void *bb[1] = {b};
    void *xx[1] = {x};
    return hh_solve_batch(gg, 1, o, bb, xx, info, stream);
}

