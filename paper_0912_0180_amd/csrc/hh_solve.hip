// hh_solve.hip -- host drivers of the right-preconditioned Krylov solves.
//
// The device runs every pass for all problems of a batch at once; the host
// only watches the per-problem state blocks between iterations and decides
// restarts from the true residual (paper Sec. 6.2: the solve stops on the
// relative residual; here the final ||b - H x|| / ||b|| is checked in FP64
// and a false stop or a breakdown restarts from the true residual).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hh_batch.h"

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return hh_fail(HH_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t solve_vectors_bytes(int64_t N, int method, bool fp32, int s)
{
    const size_t c16 = al256(sizeof(double2) * N), clow = al256((fp32 ? sizeof(float2) : sizeof(double2)) * N);
    if (method == HH_METHOD_BICGSTAB) return 5 * c16 + 2 * clow;
    return 4 * c16 + clow + 2 * (size_t)s * c16;
}

size_t solve_workspace_bytes(int64_t N, int method, bool fp32, int s, int hist_len)
{
    const int ngr = ceil_div(N, HH_SPAN);
    return al256(sizeof(double) * HH_NPART * ngr) + al256(sizeof(SolveState)) +
           al256(sizeof(double) * std::max(hist_len, 1)) + solve_vectors_bytes(N, method, fp32, s);
}

void workspace_release(Workspace &w)
{
    if (w.mem) (void)hipFree(w.mem);
    w = Workspace();
}

hh_status workspace_ensure(hh_grid *g, int method, bool fp32, int s, int hist_len)
{
    Workspace &w = g->ws;
    if (w.mem && w.method == method && w.fp32 == (int)fp32 && w.s >= s && w.hist_cap >= hist_len) return HH_OK;
    workspace_release(w);
    const int64_t N = g->hs.lev[0].N;
    const size_t c16 = al256(sizeof(double2) * N), clow = al256((fp32 ? sizeof(float2) : sizeof(double2)) * N);
    const int ngr = ceil_div(N, HH_SPAN);
    const size_t bytes = solve_workspace_bytes(N, method, fp32, s, hist_len);
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
    w.part = (double *)take(al256(sizeof(double) * HH_NPART * ngr));
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

// ---------------------------------------------------------------------------
// KBatch
// ---------------------------------------------------------------------------
KBatch::KBatch(int method, bool fp32, Plan *external) : method_(method), fp32_(fp32), pl_(external ? external : &own_)
{
    // iterations per graph replay between host checks: each check idles the
    // GPU for a copy and a synchronisation, while iterations after a stop are
    // early-returning no-ops (1024^2: 16 takes 175 ms against 179 ms for 4;
    // 32 gains little more and costs the short 3D solves)
    const char *ek = getenv("HH_ITERS_PER_CHECK");
    K_ = ek ? std::max(1, atoi(ek)) : 16;
    graph_ = !getenv("HH_NO_GRAPH");
    const char *eg = getenv("HH_DRIFT_GROW"), *es = getenv("HH_DRIFT_STALL");
    drift_grow_ = eg ? atof(eg) : HH_DRIFT_GROW;
    drift_stall_ = es ? atoi(es) : HH_DRIFT_STALL;
    // Mixed precision runs in stages: each stops once the recurrence residual
    // has dropped by a fixed factor from the stage's starting true residual,
    // and the next restarts from the FP64 true residual with a fresh shadow
    // vector.  An FP32 V-cycle differs by rounding from one application to
    // the next; the short recurrences of Bi-CGSTAB and IDR(s) assume one fixed
    // preconditioner, and on indefinite problems that mismatch accumulates
    // (relative perturbations of 1e-7 double the matvecs of a 5.4-points-per-
    // wavelength problem, and the FP32 cycle stalls it).  A restart discards
    // the accumulated mismatch.  Bi-CGSTAB restarts cheaply and gains from
    // frequent stages; an IDR(s) restart repeats s start-up steps and rebuilds
    // its shadow-space matrix, so it takes rare ones.  HH_MIXED_STAGE sets the
    // factor for both, 0 turns stages off.
    const char *st = getenv("HH_MIXED_STAGE");
    const double def = method == HH_METHOD_BICGSTAB ? HH_MIXED_STAGE_BICG : HH_MIXED_STAGE_IDR;
    stage_ = fp32_ ? (st ? atof(st) : def) : 0.0;
    if (!(stage_ > 0.0 && stage_ < 1.0)) stage_ = 0.0;
}

KBatch::~KBatch()
{
    if (sub_mem_) (void)hipFree(sub_mem_);
    plan_release(own_);
}

int KBatch::running() const
{
    int n = 0;
    for (const KProb *p : P_) n += !p->done;
    return n;
}

hh_status KBatch::set(const std::vector<KProb *> &probs)
{
    // current control blocks of problems carried over
    std::vector<Ctrl> old(P_.size());
    if (!P_.empty() && pl_->ctrl && pl_->stream) {
        HIPCHK(hipMemcpyAsync(old.data(), pl_->ctrl, sizeof(Ctrl) * P_.size(), hipMemcpyDeviceToHost, pl_->stream));
        HIPCHK(hipStreamSynchronize(pl_->stream));
    }
    // carried-over problems are recognised by serial (a freed problem's
    // address may have been reused by a new one)
    std::vector<Ctrl> hc(probs.size());
    for (size_t q = 0; q < probs.size(); ++q) {
        memset(&hc[q], 0, sizeof(Ctrl));
        hc[q].phase = PH_IDLE;
        if (probs[q]->serial == 0) continue;
        for (size_t r = 0; r < ids_.size(); ++r)
            if (ids_[r] == probs[q]->serial) hc[q] = old[r];
    }
    if (pl_ == &own_) {
        std::vector<const hh_grid *> G;
        for (KProb *p : probs) G.push_back(p->g);
        hh_status rc = plan_build(own_, G, fp32_);
        if (rc != HH_OK) return rc;
    } else if (pl_->count != (int)probs.size()) {
        return hh_fail(HH_ERR_ARG, "external plan does not match the problem set");
    }
    P_ = probs;
    ids_.resize(P_.size());
    for (size_t q = 0; q < P_.size(); ++q) {
        if (P_[q]->serial == 0) P_[q]->serial = next_serial_++;
        ids_[q] = P_[q]->serial;
    }
    if (!pl_->stream) HIPCHK(hipStreamCreateWithFlags(&pl_->stream, hipStreamNonBlocking));
    if (!pl_->hctrl || pl_->hcap < (int)probs.size()) {
        if (pl_->hctrl) (void)hipHostFree(pl_->hctrl);
        pl_->hctrl = nullptr;
        pl_->hcap = 0;
        HIPCHK(hipHostMalloc((void **)&pl_->hctrl, sizeof(Ctrl) * std::max<size_t>(probs.size(), 1), 0));
        pl_->hcap = (int)std::max<size_t>(probs.size(), 1);
    }
    const int nb = (int)P_.size();
    std::vector<ProbDev> hp(nb);
    int total_groups = 0;
    for (int q = 0; q < nb; ++q) {
        fill_solve_prob(P_[q]->g, &P_[q]->o, P_[q]->b, P_[q]->x, hp[q]);
        hp[q].ctrl = pl_->ctrl + q;
        total_groups += hp[q].ngroup;
    }
    pl_->host = hp;
    hipStream_t s = pl_->stream;
    if (nb > 0) {
        HIPCHK(hipMemcpyAsync(pl_->probs, hp.data(), sizeof(ProbDev) * nb, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(pl_->ctrl, hc.data(), sizeof(Ctrl) * nb, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const size_t need = al256(sizeof(Tile) * std::max(total_groups, 1)) + al256(sizeof(int) * std::max(nb, 1));
    if (need > sub_bytes_) {
        if (sub_mem_) (void)hipFree(sub_mem_);
        sub_mem_ = nullptr;
        sub_bytes_ = 0;
        hipError_t e = hipMalloc(&sub_mem_, need);
        if (e != hipSuccess) {
            sub_mem_ = nullptr;
            return hh_fail(HH_ERR_OOM, "hipMalloc(%zu) for subset lists: %s", need, hipGetErrorString(e));
        }
        sub_bytes_ = need;
    }
    sub_t_ = (Tile *)sub_mem_;
    sub_p_ = (int *)((char *)sub_mem_ + al256(sizeof(Tile) * std::max(total_groups, 1)));
    return HH_OK;
}

hh_status KBatch::sub_set(const std::vector<int> &which)
{
    ht_.clear();
    hp_.clear();
    for (int q : which) {
        const int ngr = pl_->host[q].ngroup;
        for (int i = 0; i < ngr; ++i) ht_.push_back(Tile{q, i});
        hp_.push_back(q);
    }
    hipStream_t s = pl_->stream;
    if (!ht_.empty()) HIPCHK(hipMemcpyAsync(sub_t_, ht_.data(), sizeof(Tile) * ht_.size(), hipMemcpyHostToDevice, s));
    if (!hp_.empty()) HIPCHK(hipMemcpyAsync(sub_p_, hp_.data(), sizeof(int) * hp_.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

hh_status KBatch::read_states(const std::vector<int> &which)
{
    hipStream_t s = pl_->stream;
    for (int q : which)
        HIPCHK(hipMemcpyAsync(&P_[q]->S, P_[q]->g->ws.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HH_OK;
}

hh_status KBatch::start(const std::vector<KProb *> &probs)
{
    const int init_mode = method_ == HH_METHOD_BICGSTAB ? 0 : 2;
    const int init_fin = method_ == HH_METHOD_BICGSTAB ? FIN_INIT : FIN_IDR_INIT;
    hipStream_t s = pl_->stream;
    std::vector<int> idx;
    for (KProb *p : probs) {
        int q = -1;
        for (size_t r = 0; r < P_.size(); ++r)
            if (P_[r] == p) q = (int)r;
        if (q < 0) return hh_fail(HH_ERR_ARG, "start: problem not in the set");
        idx.push_back(q);
        SolveState st;
        memset(&st, 0, sizeof st);
        st.phase = PH_IDLE;
        p->stage_rel = 1.0;
        p->stages = stage_ > 0.0 ? 1 : 0;
        p->stage_tol = stage_ > 0.0 ? std::max(p->o.tol, stage_) : p->o.tol;
        st.tol = p->stage_tol;
        st.max_mv = p->o.max_matvec;
        st.hist_len = p->o.history ? p->o.history_len : 0;
        st.s = method_ == HH_METHOD_IDR ? p->o.s : 0;
        st.startup = -1;
        st.guard = fp32_ ? 1 : 0;
        st.drift_grow = drift_grow_;
        st.drift_stall = drift_stall_;
        st.mv = p->mv0;
        st.it = p->it0;
        p->S = st;
        p->done = p->closed = p->drift = false;
        p->status = HH_OK;
        HIPCHK(hipMemcpyAsync(p->g->ws.st, &p->S, sizeof st, hipMemcpyHostToDevice, s));
    }
    if (idx.empty()) return HH_OK;
    hh_status rc = sub_set(idx);
    if (rc != HH_OK) return rc;
    DevList dl{sub_t_, (int)ht_.size()};
    launch_norm(*pl_, dl, VS_B, s);
    launch_fin(*pl_, sub_p_, (int)idx.size(), FIN_BNORM, s);
    HIPCHK(hipGetLastError());
    rc = read_states(idx);
    if (rc != HH_OK) return rc;
    std::vector<int> zero_x, go;
    for (int q : idx) {
        KProb *p = P_[q];
        if (!p->o.x0_given) zero_x.push_back(q);
        if (!std::isfinite(p->S.bnorm)) {
            p->done = true;
            p->status = HH_ERR_NONFINITE;
        } else if (p->S.bnorm == 0.0) {
            p->done = true;
            p->status = HH_OK;
            if (p->o.x0_given) zero_x.push_back(q);
        } else {
            go.push_back(q);
        }
    }
    if (!zero_x.empty()) {
        rc = sub_set(zero_x);
        if (rc != HH_OK) return rc;
        launch_zero(*pl_, DevList{sub_t_, (int)ht_.size()}, VS_X, s);
    }
    if (!go.empty()) {
        rc = sub_set(go);
        if (rc != HH_OK) return rc;
        launch_resid(*pl_, DevList{sub_t_, (int)ht_.size()}, init_mode, s);
        launch_fin(*pl_, sub_p_, (int)go.size(), init_fin, s);
    }
    HIPCHK(hipGetLastError());
    return HH_OK;
}

hh_status KBatch::launch()
{
    if (running() == 0) return HH_OK;
    hipStream_t s = pl_->stream;
    auto iterate1 = [&]() {
        if (method_ == HH_METHOD_BICGSTAB) launch_bicg_iteration(*pl_, s);
        else launch_idr_step(*pl_, s);
    };
    if (!graph_) {
        for (int k = 0; k < K_; ++k) iterate1();
        HIPCHK(hipGetLastError());
        return HH_OK;
    }
    // the graph bakes in the plan's lists and, for one-problem plans, the
    // problem descriptor the finalisation takes by value, with the work-space
    // vectors the V-cycle reads and writes (a work space reallocated at the
    // same address may be carved differently)
    ProbDev key;
    memset(&key, 0, sizeof key);
    if (pl_->count == 1) memcpy(&key, &pl_->host[0], sizeof key);   // padding zero (grid_fill_prob)
    if (!pl_->gexec || pl_->gmethod != method_ || pl_->gK != K_ || memcmp(&key, &pl_->gpd, sizeof key) != 0) {
        if (pl_->gexec) {
            HIPCHK(hipGraphExecDestroy(pl_->gexec));
            pl_->gexec = nullptr;
        }
        hipGraph_t graph;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K_; ++k) iterate1();
        HIPCHK(hipStreamEndCapture(s, &graph));
        hipError_t e = hipGraphInstantiate(&pl_->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            pl_->gexec = nullptr;
            return hh_fail(HH_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        pl_->gmethod = method_;
        pl_->gK = K_;
        memcpy(&pl_->gpd, &key, sizeof key);
    }
    HIPCHK(hipGraphLaunch(pl_->gexec, s));
    return HH_OK;
}

hh_status KBatch::close(const std::vector<int> &which, std::vector<KProb *> &closed)
{
    if (which.empty()) return HH_OK;
    hipStream_t s = pl_->stream;
    std::vector<int> fin;
    for (int q : which)
        if (P_[q]->status != HH_ERR_NONFINITE && P_[q]->S.bnorm > 0.0) fin.push_back(q);
    if (!fin.empty()) {
        hh_status rc = sub_set(fin);
        if (rc != HH_OK) return rc;
        launch_resid(*pl_, DevList{sub_t_, (int)ht_.size()}, 1, s);
        launch_fin(*pl_, sub_p_, (int)fin.size(), FIN_TRUE, s);
        HIPCHK(hipGetLastError());
    }
    hh_status rc = read_states(which);
    if (rc != HH_OK) return rc;
    for (int q : which) {
        KProb *p = P_[q];
        const SolveState &S = p->S;
        hh_solve_info &in = p->info;
        memset(&in, 0, sizeof in);
        in.status = p->status;
        in.matvecs = S.mv;
        in.iterations = S.it;
        in.restarts = p->restarts;
        in.stages = p->stages;
        in.rel_res_recurrence = S.bnorm > 0.0 ? S.rel : 0.0;
        in.rel_res_true = S.bnorm > 0.0 ? S.true_rel : 0.0;
        if (p->status == HH_ERR_NONFINITE) in.rel_res_true = NAN;
        if (p->o.history && p->o.history_len > 0) {
            // entries of this phase only: [mv0, mv)
            const int lo = p->mv0, hi = std::min(S.mv, p->o.history_len);
            if (hi > lo) {
                HIPCHK(hipMemcpyAsync(p->o.history + lo, p->g->ws.hist + lo, sizeof(double) * (hi - lo),
                                      hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            }
        }
        p->closed = true;
        closed.push_back(p);
    }
    return HH_OK;
}

hh_status KBatch::collect(std::vector<KProb *> &closed)
{
    const int init_mode = method_ == HH_METHOD_BICGSTAB ? 0 : 2;
    const int init_fin = method_ == HH_METHOD_BICGSTAB ? FIN_INIT : FIN_IDR_INIT;
    hipStream_t s = pl_->stream;
    const int nb = (int)P_.size();
    if (running() > 0) {
        HIPCHK(hipMemcpyAsync(pl_->hctrl, pl_->ctrl, sizeof(Ctrl) * nb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int> verify;
        for (int q = 0; q < nb; ++q) {
            KProb *p = P_[q];
            if (p->done || pl_->hctrl[q].phase != PH_STOP) continue;
            const int reason = pl_->hctrl[q].reason;
            if (reason == RS_NONFIN) {
                p->done = true;
                p->status = HH_ERR_NONFINITE;
            } else if (reason == RS_MAXMV) {
                p->done = true;
                p->status = HH_ERR_NOCONV;
            } else if (reason == RS_DRIFT) {
                p->done = true;
                p->drift = true;
                p->status = HH_ERR_NOCONV;
            } else {
                verify.push_back(q);
            }
        }
        if (!verify.empty()) {
            hh_status rc = sub_set(verify);
            if (rc != HH_OK) return rc;
            launch_resid(*pl_, DevList{sub_t_, (int)ht_.size()}, 1, s);
            launch_fin(*pl_, sub_p_, (int)verify.size(), FIN_TRUE, s);
            HIPCHK(hipGetLastError());
            rc = read_states(verify);
            if (rc != HH_OK) return rc;
            std::vector<int> restart;
            for (int q : verify) {
                KProb *p = P_[q];
                if (p->S.reason == RS_CONV && p->S.true_rel < p->o.tol) {
                    p->done = true;
                    p->status = HH_OK;
                } else if (stage_ > 0.0 && p->S.reason == RS_CONV && p->S.true_rel < p->stage_rel) {
                    // a stage ended with progress: the next one starts from
                    // the true residual and aims `stage_` lower
                    p->stage_rel = p->S.true_rel;
                    p->stages++;
                    p->stage_tol = std::max(p->o.tol, stage_ * p->S.true_rel);
                    HIPCHK(hipMemcpyAsync((char *)p->g->ws.st + offsetof(SolveState, tol), &p->stage_tol,
                                          sizeof(double), hipMemcpyHostToDevice, s));
                    restart.push_back(q);
                } else if (p->restarts >= p->o.max_restarts) {
                    p->done = true;
                    p->status = p->S.reason == RS_BREAK ? HH_ERR_BREAKDOWN : HH_ERR_NOCONV;
                } else {
                    p->restarts++;
                    restart.push_back(q);
                }
            }
            if (!restart.empty()) {
                rc = sub_set(restart);
                if (rc != HH_OK) return rc;
                launch_resid(*pl_, DevList{sub_t_, (int)ht_.size()}, init_mode, s);
                launch_fin(*pl_, sub_p_, (int)restart.size(), init_fin, s);
                HIPCHK(hipGetLastError());
            }
        }
    }
    std::vector<int> to_close;
    for (int q = 0; q < nb; ++q)
        if (P_[q]->done && !P_[q]->closed) to_close.push_back(q);
    return close(to_close, closed);
}

hh_status check_solve_opts(const hh_grid *g, const hh_solve_opts *o)
{
    if (!o) return hh_fail(HH_ERR_ARG, "null options");
    if (o->method != HH_METHOD_BICGSTAB && o->method != HH_METHOD_IDR) return hh_fail(HH_ERR_ARG, "unknown method %d", o->method);
    if (o->method == HH_METHOD_IDR && (o->s < 1 || o->s > HH_MAX_S || !o->idr_P))
        return hh_fail(HH_ERR_ARG, "IDR(s) needs 1 <= s <= %d and a shadow space", HH_MAX_S);
    if (!(o->tol > 0.0) || o->max_matvec < 1 || o->max_restarts < 0) return hh_fail(HH_ERR_ARG, "need tol > 0, max_matvec >= 1, max_restarts >= 0");
    if (o->vcycle_prec != HH_C128 && o->vcycle_prec != HH_C64) return hh_fail(HH_ERR_ARG, "unknown vcycle precision");
    if (g->host_only) return hh_fail(HH_ERR_ARG, "grid was built host-only");
    if (g->hs.centering != HH_CELL) return hh_fail(HH_ERR_ARG, "a vertex-centred grid cannot be solved (operator apply only)");
    if (g->hs.smoother == HH_SMOOTH_ILU0 && o->vcycle_prec != HH_C128)
        return hh_fail(HH_ERR_ARG, "ILU(0) smoothing runs in the FP64 V-cycle only (vcycle_prec HH_C128)");
    return HH_OK;
}


// One phase of a batch solve: every problem from start to stop in one
// KBatch.  A single problem uses (and keeps) the plan cached in its grid.
static hh_status run_phase(hh_grid *const *g, const std::vector<KProb *> &ptrs, int method, bool fp32, hipStream_t s)
{
    const int count = (int)ptrs.size();
    Plan *ext = nullptr;
    if (count == 1) {
        if (g[0]->plan_fp32 != (int)fp32 || !g[0]->plan.mem) {
            std::vector<const hh_grid *> G{g[0]};
            hh_status rc = plan_build(g[0]->plan, G, fp32);
            if (rc != HH_OK) return rc;
            g[0]->plan_fp32 = fp32;
        }
        ext = &g[0]->plan;
    }
    KBatch kb(method, fp32, ext);
    hh_status rc = kb.set(ptrs);
    if (rc != HH_OK) return rc;
    // the solve runs on the plan's own stream (graphs cannot be captured on
    // the null stream), ordered after the caller's stream by an event
    {
        hipEvent_t ev;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, s));
        HIPCHK(hipStreamWaitEvent(kb.stream(), ev, 0));
        HIPCHK(hipEventDestroy(ev));
    }
    rc = kb.start(ptrs);
    std::vector<KProb *> closed;
    while (rc == HH_OK && (int)closed.size() < count) {
        rc = kb.launch();
        if (rc == HH_OK) rc = kb.collect(closed);
    }
    HIPCHK(hipStreamSynchronize(kb.stream()));
    return rc;
}

extern "C" hh_status hh_solve_batch(hh_grid *const *g, int32_t count, const hh_solve_opts *o, const void *const *b,
                                    void *const *x, hh_solve_info *info, void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!g || !o || !b || !x || !info || count < 1) return hh_fail(HH_ERR_ARG, "null argument or empty batch");
    hipStream_t s = (hipStream_t)stream;
    std::vector<KProb> K(count);
    std::vector<KProb *> ptrs(count);
    for (int q = 0; q < count; ++q) {
        if (!g[q] || !b[q] || !x[q]) return hh_fail(HH_ERR_ARG, "problem %d: null grid or vector", q);
        hh_status rc = check_solve_opts(g[q], &o[q]);
        if (rc != HH_OK) return rc;
        if (o[q].method != o[0].method || o[q].vcycle_prec != o[0].vcycle_prec)
            return hh_fail(HH_ERR_ARG, "all problems of a batch need the same method and V-cycle precision");
        if (g[q]->hs.dim != g[0]->hs.dim) return hh_fail(HH_ERR_ARG, "all problems of a batch need the same dimension");
        for (int r = 0; r < q; ++r)
            if (g[r] == g[q]) return hh_fail(HH_ERR_ARG, "grid used twice in one batch");
        K[q].g = g[q];
        K[q].o = o[q];
        K[q].b = b[q];
        K[q].x = x[q];
        ptrs[q] = &K[q];
        memset(&info[q], 0, sizeof(hh_solve_info));
    }
    const bool fp32 = o[0].vcycle_prec == HH_C64;
    for (int q = 0; q < count; ++q) {
        hh_status rc = workspace_ensure(g[q], o[q].method, fp32, o[q].method == HH_METHOD_IDR ? o[q].s : 0,
                                        o[q].history ? o[q].history_len : 0);
        if (rc != HH_OK) return rc;
    }
    hh_status rc = run_phase(g, ptrs, o[0].method, fp32, s);
    if (rc != HH_OK) return rc;
    // mixed-precision solves stopped by the drift guard continue from their
    // current iterate with the FP64 V-cycle
    std::vector<KProb> E;
    std::vector<int> eq;
    for (int q = 0; q < count; ++q)
        if (K[q].drift && fp32) eq.push_back(q);
    if (!eq.empty()) {
        std::vector<hh_grid *> eg;
        for (int q : eq) {
            rc = workspace_ensure(g[q], o[q].method, false, o[q].method == HH_METHOD_IDR ? o[q].s : 0,
                                  o[q].history ? o[q].history_len : 0);
            if (rc != HH_OK) return rc;
            KProb e = K[q];
            e.o.vcycle_prec = HH_C128;
            e.o.x0_given = 1;
            e.mv0 = K[q].info.matvecs;
            e.it0 = K[q].info.iterations;
            e.serial = 0;
            e.done = e.closed = e.drift = false;
            E.push_back(e);
            eg.push_back(g[q]);
        }
        std::vector<KProb *> ep;
        for (KProb &e : E) ep.push_back(&e);
        rc = run_phase(eg.data(), ep, o[0].method, false, s);
        if (rc != HH_OK) return rc;
        for (size_t i = 0; i < eq.size(); ++i) {
            const int st0 = K[eq[i]].info.stages;
            K[eq[i]].info = E[i].info;
            K[eq[i]].info.fp64_fallback = 1;
            K[eq[i]].info.stages = st0;
        }
    }
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    hh_status first = HH_OK;
    for (int q = 0; q < count; ++q) {
        info[q] = K[q].info;
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

