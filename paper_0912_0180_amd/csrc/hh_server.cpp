// hh_server.cpp -- request server: continuous batching of Helmholtz solves.
//
// Requests are admitted in arrival order while their device footprint fits
// the byte budget and a slot is free.  Admitted problems of the same
// dimension, method and V-cycle precision form one batch whose passes run as
// single launches over all their tiles; a finished problem leaves and a new
// one joins at the next check of the control blocks, while the Krylov state of
// every other problem stays on the device.  Host setup (node maps, coarse
// inverse) runs on preparation threads ahead of admission.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hh_batch.h"

namespace {

constexpr int kPrepThreads = 2;

struct Req {
    uint64_t ticket = 0;
    hh_grid_desc desc{};
    std::vector<double> phi;
    hh_solve_opts opts{};
    std::vector<double2> b, P;
    void *x_host = nullptr;
    uint64_t foot = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    // preparation
    bool preparing = false, prepared = false;
    hh_status prep_status = HH_OK;
    std::string prep_err;
    std::unique_ptr<HostSetup> hs;
    // device
    hh_grid *g = nullptr;
    void *io = nullptr;          // b, x, P
    size_t io_bytes = 0;
    KProb kp;
    int group = -1;
    bool escalated = false;      // continued with the FP64 V-cycle after a drift stop
    hh_result result{};
    // guarded by the server mutex
    bool finished = false;       // result valid (x_host written)
    bool polled = false;         // result handed to the caller
    bool worker_done = false;    // the worker holds no reference any more
};

struct Group {
    int dim, method;
    bool fp32;
    std::unique_ptr<KBatch> kb;
    std::vector<Req *> members;  // admitted, not finished
    std::vector<Req *> joining;  // admitted since the last set()
    bool dirty = false;
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

} // namespace

struct hh_server {
    hh_server_opts opts{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_prep;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Req *> queue;                 // submitted, not admitted (arrival order)
    std::map<uint64_t, Req *> live;          // every ticket not yet polled
    hh_server_stats st{};
    std::thread worker;
    std::vector<std::thread> preps;
    // worker-only state
    std::vector<Group> groups;
};

static hh_status req_check_opts(const hh_request *r)
{
    const hh_solve_opts *o = &r->opts;
    if (o->method != HH_METHOD_BICGSTAB && o->method != HH_METHOD_IDR) return hh_fail(HH_ERR_ARG, "unknown method %d", o->method);
    if (o->method == HH_METHOD_IDR && (o->s < 1 || o->s > HH_MAX_S || !r->idr_P_host))
        return hh_fail(HH_ERR_ARG, "IDR(s) needs 1 <= s <= %d and idr_P_host", HH_MAX_S);
    if (!(o->tol > 0.0) || o->max_matvec < 1 || o->max_restarts < 0)
        return hh_fail(HH_ERR_ARG, "need tol > 0, max_matvec >= 1, max_restarts >= 0");
    if (o->vcycle_prec != HH_C128 && o->vcycle_prec != HH_C64) return hh_fail(HH_ERR_ARG, "unknown vcycle precision");
    if (!r->b_host || !r->x_host) return hh_fail(HH_ERR_ARG, "b_host and x_host are required");
    return HH_OK;
}

// --------------------------------------------------------------------------
// preparation threads: host setup of queued requests, in arrival order, at
// most max_slots requests ahead of admission
// --------------------------------------------------------------------------
static void prep_loop(hh_server *sv)
{
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        Req *r = nullptr;
        sv->cv_prep.wait(lk, [&] {
            if (sv->stop) return true;
            int ahead = 0;
            for (Req *q : sv->queue) {
                if (q->prepared || q->preparing) {
                    ++ahead;
                    continue;
                }
                if (ahead < std::max(2, sv->opts.max_slots)) return true;
                break;
            }
            return false;
        });
        if (sv->stop) return;
        int ahead = 0;
        for (Req *q : sv->queue) {
            if (q->prepared || q->preparing) {
                ++ahead;
                continue;
            }
            if (ahead < std::max(2, sv->opts.max_slots)) r = q;
            break;
        }
        if (!r) continue;
        r->preparing = true;
        lk.unlock();
        std::unique_ptr<HostSetup> hs(new HostSetup());
        std::string err;
        hh_grid_desc d = r->desc;
        d.phi = r->phi.empty() ? nullptr : r->phi.data();
        hh_status st = host_setup(&d, *hs, err);
        lk.lock();
        r->preparing = false;
        r->prepared = true;
        r->prep_status = st;
        r->prep_err = err;
        if (st == HH_OK) r->hs = std::move(hs);
        sv->cv_work.notify_all();
    }
}

// --------------------------------------------------------------------------
// worker
// --------------------------------------------------------------------------
static void finish_req(hh_server *sv, Req *r, int status)
{
    // caller holds no lock; result fields are published under the lock below
    r->result.info = r->kp.info;
    if (status != HH_OK) r->result.info.status = status;
    r->t_done = now_s(sv->t0);
    r->result.t_submit = r->t_submit;
    r->result.t_admit = r->t_admit;
    r->result.t_done = r->t_done;
    r->result.info.seconds = r->t_done - r->t_admit;
    r->result.info.fp64_fallback = r->escalated ? 1 : 0;
}

static void release_req_device(Req *r)
{
    if (r->g) (void)hh_free_grid(r->g);
    r->g = nullptr;
    if (r->io) (void)hipFree(r->io);
    r->io = nullptr;
    r->hs.reset();
}

// Builds the device side of an admitted request: grid, work space, b, x, P.
static hh_status admit_device(Req *r)
{
    hh_grid_desc d = r->desc;
    d.phi = nullptr;
    d.host_only = 0;
    hh_status st = grid_create(std::move(*r->hs), &d, &r->g);
    r->hs.reset();
    if (st != HH_OK) return st;
    const bool fp32 = r->opts.vcycle_prec == HH_C64;
    const int s = r->opts.method == HH_METHOD_IDR ? r->opts.s : 0;
    st = workspace_ensure(r->g, r->opts.method, fp32, s, 0);
    if (st != HH_OK) return st;
    const size_t N = (size_t)r->g->hs.lev[0].N;
    const size_t vb = (sizeof(double2) * N + 255) & ~(size_t)255;
    r->io_bytes = 2 * vb + (s > 0 ? ((sizeof(double2) * N * s + 255) & ~(size_t)255) : 0);
    if (hipMalloc(&r->io, r->io_bytes) != hipSuccess) {
        r->io = nullptr;
        return hh_fail(HH_ERR_OOM, "hipMalloc(%zu) for request vectors", r->io_bytes);
    }
    char *base = (char *)r->io;
    void *b = base, *x = base + vb, *P = s > 0 ? base + 2 * vb : nullptr;
    if (hipMemcpy(b, r->b.data(), sizeof(double2) * N, hipMemcpyHostToDevice) != hipSuccess ||
        (P && hipMemcpy(P, r->P.data(), sizeof(double2) * N * s, hipMemcpyHostToDevice) != hipSuccess))
        return hh_fail(HH_ERR_HIP, "copy of request inputs failed");
    // host copies are no longer needed
    std::vector<double2>().swap(r->b);
    std::vector<double2>().swap(r->P);
    std::vector<double>().swap(r->phi);
    r->kp = KProb();
    r->kp.g = r->g;
    r->kp.o = r->opts;
    r->kp.o.history = nullptr;
    r->kp.o.history_len = 0;
    r->kp.o.x0_given = 0;
    r->kp.o.idr_P = P;
    r->kp.b = b;
    r->kp.x = x;
    r->kp.tag = r;
    return HH_OK;
}

static int group_of(hh_server *sv, int dim, int method, bool fp32)
{
    for (size_t i = 0; i < sv->groups.size(); ++i)
        if (sv->groups[i].dim == dim && sv->groups[i].method == method && sv->groups[i].fp32 == fp32) return (int)i;
    Group gr;
    gr.dim = dim;
    gr.method = method;
    gr.fp32 = fp32;
    gr.kb.reset(new KBatch(method, fp32));
    sv->groups.push_back(std::move(gr));
    return (int)sv->groups.size() - 1;
}

// A drift-stopped mixed-precision problem continues from its iterate with
// the FP64 V-cycle in the FP64 group (its footprint reserved the FP64 work
// space at admission).
static hh_status escalate(hh_server *sv, Req *r)
{
    const int s = r->opts.method == HH_METHOD_IDR ? r->opts.s : 0;
    hh_status st = workspace_ensure(r->g, r->opts.method, false, s, 0);
    if (st != HH_OK) return st;
    KProb e = r->kp;
    e.o.vcycle_prec = HH_C128;
    e.o.x0_given = 1;
    e.mv0 = r->kp.info.matvecs;
    e.it0 = r->kp.info.iterations;
    e.serial = 0;
    e.done = e.closed = e.drift = false;
    r->kp = e;
    r->escalated = true;
    const int gi = group_of(sv, r->desc.dim, r->opts.method, false);
    r->group = gi;
    sv->groups[gi].members.push_back(r);
    sv->groups[gi].joining.push_back(r);
    sv->groups[gi].dirty = true;
    return HH_OK;
}

static uint64_t req_actual_bytes(const Req *r)
{
    if (!r->g) return 0;
    return r->g->dbytes + r->g->ws.bytes + r->io_bytes;
}

// Marks a request finished (result, counters); `device_held`: its footprint
// was counted in the budget.
static void publish(hh_server *sv, Req *r, bool device_held, bool worker_done)
{
    std::lock_guard<std::mutex> lk(sv->mu);
    r->finished = true;
    sv->st.completed++;
    if (device_held) {
        sv->st.active_slots--;
        sv->st.bytes_in_use -= r->foot;
    }
    if (worker_done) {
        r->worker_done = true;
        if (r->polled) delete r;
    }
    sv->cv_work.notify_all();
}

static void drop_worker_ref(hh_server *sv, Req *r)
{
    std::lock_guard<std::mutex> lk(sv->mu);
    r->worker_done = true;
    if (r->polled) delete r;
}

static void worker_loop(hh_server *sv)
{
    (void)hipSetDevice(sv->opts.device);
    // finished requests still named by a batch until its next re-plan
    std::vector<Req *> graveyard;
    for (;;) {
        // ---- admission (arrival order; the head blocks the queue) ----------
        std::vector<Req *> admitted, failed;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            bool any_active = false;
            for (Group &gr : sv->groups) any_active |= !gr.members.empty();
            if (!any_active)
                sv->cv_work.wait(lk, [&] { return sv->stop || (!sv->queue.empty() && sv->queue.front()->prepared); });
            if (sv->stop) break;
            while (!sv->queue.empty()) {
                Req *r = sv->queue.front();
                if (!r->prepared) break;
                if (r->prep_status != HH_OK) {
                    sv->queue.pop_front();
                    failed.push_back(r);
                    continue;
                }
                if (sv->st.active_slots >= sv->opts.max_slots) break;
                if (sv->st.bytes_in_use + r->foot > sv->st.bytes_budget) break;
                sv->queue.pop_front();
                sv->st.active_slots++;
                sv->st.bytes_in_use += r->foot;
                sv->st.peak_bytes = std::max(sv->st.peak_bytes, sv->st.bytes_in_use);
                sv->st.admitted++;
                r->t_admit = now_s(sv->t0);
                admitted.push_back(r);
            }
            sv->st.queued = (int32_t)sv->queue.size();
            sv->cv_prep.notify_all();
        }
        for (Req *r : failed) {
            r->t_admit = now_s(sv->t0);
            r->kp.info.status = r->prep_status;
            finish_req(sv, r, r->prep_status);
            publish(sv, r, false, true);
        }
        for (Req *r : admitted) {
            hh_status st = admit_device(r);
            if (st != HH_OK) {
                release_req_device(r);
                finish_req(sv, r, st);
                publish(sv, r, true, true);
                continue;
            }
            const int gi = group_of(sv, r->desc.dim, r->opts.method, r->opts.vcycle_prec == HH_C64);
            r->group = gi;
            sv->groups[gi].members.push_back(r);
            sv->groups[gi].joining.push_back(r);
            sv->groups[gi].dirty = true;
        }
        // ---- re-plan groups whose membership changed, start new problems --
        for (Group &gr : sv->groups) {
            if (!gr.dirty) continue;
            gr.dirty = false;
            if (gr.members.empty()) {
                gr.kb.reset(new KBatch(gr.method, gr.fp32));   // give the plan back
                gr.joining.clear();
                continue;
            }
            std::vector<KProb *> ps, fresh;
            for (Req *r : gr.members) ps.push_back(&r->kp);
            for (Req *r : gr.joining) fresh.push_back(&r->kp);
            hh_status st = gr.kb->set(ps);
            if (st == HH_OK) st = gr.kb->start(fresh);
            gr.joining.clear();
            if (st != HH_OK) {
                for (Req *r : gr.members) {
                    r->kp.done = r->kp.closed = true;
                    r->kp.info.status = st;
                }
            }
        }
        for (Req *r : graveyard) drop_worker_ref(sv, r);
        graveyard.clear();
        {
            uint64_t act = 0;
            for (Group &gr : sv->groups) {
                if (gr.members.empty()) continue;
                for (Req *r : gr.members) act += req_actual_bytes(r);
                act += gr.kb->device_bytes();
            }
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->st.actual_in_use = act;
            sv->st.peak_actual = std::max(sv->st.peak_actual, act);
        }
        // ---- K iterations of every group, then one check of each ----------
        std::vector<Req *> drifted;
        for (Group &gr : sv->groups)
            if (!gr.members.empty()) {
                hh_status st = gr.kb->launch();
                if (st != HH_OK)
                    for (Req *r : gr.members) {
                        r->kp.done = r->kp.closed = true;
                        r->kp.info.status = st;
                    }
            }
        for (Group &gr : sv->groups) {
            if (gr.members.empty()) continue;
            std::vector<KProb *> closed;
            hh_status st = gr.kb->collect(closed);
            if (st != HH_OK) {
                for (Req *r : gr.members)
                    if (!r->kp.closed) {
                        r->kp.done = r->kp.closed = true;
                        r->kp.info.status = st;
                    }
            }
            std::vector<Req *> out;
            for (Req *r : gr.members)
                if (r->kp.closed) out.push_back(r);
            if (out.empty()) continue;
            (void)hipStreamSynchronize(gr.kb->stream());
            for (Req *r : out) {
                if (r->kp.drift && gr.fp32 && !r->escalated) {
                    gr.members.erase(std::find(gr.members.begin(), gr.members.end(), r));
                    drifted.push_back(r);
                    continue;
                }
                if (r->kp.info.status != HH_ERR_HIP)
                    (void)hipMemcpy(r->x_host, r->kp.x, sizeof(double2) * (size_t)r->g->hs.lev[0].N,
                                    hipMemcpyDeviceToHost);
                release_req_device(r);
                finish_req(sv, r, HH_OK);
                gr.members.erase(std::find(gr.members.begin(), gr.members.end(), r));
                graveyard.push_back(r);
                publish(sv, r, true, false);
            }
            gr.dirty = true;
        }
        for (Req *r : drifted) {
            hh_status st = escalate(sv, r);
            if (st != HH_OK) {
                release_req_device(r);
                finish_req(sv, r, st);
                publish(sv, r, true, true);
            }
        }
    }
    // shutdown: release everything still on the device
    for (Req *r : graveyard) drop_worker_ref(sv, r);
    for (Group &gr : sv->groups) {
        gr.kb.reset();
        for (Req *r : gr.members) release_req_device(r);
    }
    sv->groups.clear();
}

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

hh_status hh_request_footprint(const hh_grid_desc *d, const hh_solve_opts *o, uint64_t *bytes)
{
    if (!d || !o || !bytes) return hh_fail(HH_ERR_ARG, "null argument");
    std::string err;
    uint64_t b = 0;
    hh_status st = footprint_bytes(d, o, b, err);
    if (st != HH_OK) return hh_fail(st, "%s", err.c_str());
    *bytes = b;
    return HH_OK;
}

hh_status hh_server_create(const hh_server_opts *o, hh_server **out)
{
    if (!o || !out) return hh_fail(HH_ERR_ARG, "null argument");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return hh_fail(HH_ERR_HIP, "no HIP device");
    if (o->device < 0 || o->device >= ndev) return hh_fail(HH_ERR_ARG, "device %d out of range", o->device);
    if (hipSetDevice(o->device) != hipSuccess) return hh_fail(HH_ERR_HIP, "hipSetDevice(%d) failed", o->device);
    hh_server *sv = new hh_server();
    sv->opts = *o;
    if (sv->opts.max_slots <= 0) sv->opts.max_slots = 64;
    if (sv->opts.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete sv;
            return hh_fail(HH_ERR_HIP, "hipMemGetInfo failed");
        }
        sv->opts.hbm_budget_bytes = (uint64_t)(0.8 * (double)fr);
    }
    sv->st.bytes_budget = sv->opts.hbm_budget_bytes;
    sv->t0 = std::chrono::steady_clock::now();
    sv->worker = std::thread(worker_loop, sv);
    for (int i = 0; i < kPrepThreads; ++i) sv->preps.emplace_back(prep_loop, sv);
    *out = sv;
    return HH_OK;
}

hh_status hh_submit(hh_server *sv, const hh_request *r, uint64_t *ticket)
{
    if (!sv || !r || !ticket) return hh_fail(HH_ERR_ARG, "null argument");
    if (r->grid.coarse_op == HH_COARSE_GALERKIN)
        return hh_fail(HH_ERR_ARG, "the server batches requests: Galerkin coarse operators are for single solves");
    if (r->grid.smoother == HH_SMOOTH_ILU0)
        return hh_fail(HH_ERR_ARG, "the server batches requests: ILU(0) smoothing is for single solves");
    uint64_t foot = 0;
    std::string err;
    hh_status st = footprint_bytes(&r->grid, &r->opts, foot, err);
    if (st == HH_OK) st = req_check_opts(r);
    else hh_fail(st, "%s", err.c_str());
    if (st == HH_OK && foot > sv->st.bytes_budget) {
        st = hh_fail(HH_ERR_OOM, "request needs %llu device bytes, budget is %llu", (unsigned long long)foot,
                     (unsigned long long)sv->st.bytes_budget);
    }
    if (st != HH_OK) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->st.rejected++;
        return st;
    }
    Req *q = new Req();
    q->desc = r->grid;
    int64_t N = 1;
    for (int a = 0; a < r->grid.dim; ++a) N *= r->grid.n[a];
    if (r->grid.phi) q->phi.assign(r->grid.phi, r->grid.phi + N);
    q->desc.phi = nullptr;
    q->opts = r->opts;
    q->b.assign((const double2 *)r->b_host, (const double2 *)r->b_host + N);
    if (r->opts.method == HH_METHOD_IDR)
        q->P.assign((const double2 *)r->idr_P_host, (const double2 *)r->idr_P_host + N * r->opts.s);
    q->x_host = r->x_host;
    q->foot = foot;
    std::lock_guard<std::mutex> lk(sv->mu);
    q->ticket = sv->next_ticket++;
    q->t_submit = now_s(sv->t0);
    sv->queue.push_back(q);
    sv->live[q->ticket] = q;
    sv->st.submitted++;
    sv->st.queued = (int32_t)sv->queue.size();
    *ticket = q->ticket;
    sv->cv_prep.notify_all();
    sv->cv_work.notify_all();
    return HH_OK;
}

hh_status hh_poll(hh_server *sv, uint64_t ticket, hh_result *out)
{
    if (!sv || !out) return hh_fail(HH_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return hh_fail(HH_ERR_TICKET, "unknown or already collected ticket %llu", (unsigned long long)ticket);
    Req *r = it->second;
    if (!r->finished) return HH_PENDING;
    *out = r->result;
    sv->live.erase(it);
    r->polled = true;
    if (r->worker_done) delete r;
    return HH_OK;
}

hh_status hh_server_query(hh_server *sv, hh_server_stats *st)
{
    if (!sv || !st) return hh_fail(HH_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *st = sv->st;
    return HH_OK;
}

hh_status hh_server_destroy(hh_server *sv)
{
    if (!sv) return HH_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_prep.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (std::thread &t : sv->preps)
        if (t.joinable()) t.join();
    // requests never collected by hh_poll (queued, running or finished)
    for (auto &kv : sv->live) delete kv.second;
    delete sv;
    return HH_OK;
}

} // extern "C"
