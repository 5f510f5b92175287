// hh_batch.h -- a resumable set of Krylov solves sharing one launch plan.
//
// Problems join and leave only between checks of the control blocks; the
// Krylov state of every problem (vectors, scalars, control block contents)
// stays on the device while the plan around it is rebuilt.
#pragma once
#include <vector>

#include "hh_lib.h"

struct KProb {
    hh_grid *g = nullptr;
    hh_solve_opts o{};
    const void *b = nullptr;
    void *x = nullptr;
    hh_solve_info info{};
    int status = HH_OK;
    int restarts = 0;
    bool done = false;      // iteration over (status final); info valid once `closed`
    bool closed = false;
    bool drift = false;     // stopped by the mixed-precision guard
    int mv0 = 0, it0 = 0;   // counts carried over from an earlier phase of the solve
    // staged mixed-precision solve: the true residual at the start of the
    // current stage, the stages begun so far, the current stage tolerance
    double stage_rel = 1.0;
    int stages = 0;
    double stage_tol = 0.0;
    SolveState S{};         // last state read back
    void *tag = nullptr;    // owner's handle
    uint64_t serial = 0;    // set when the problem first joins a batch
};

class KBatch {
  public:
    // `external`: a plan the caller keeps (a grid's cached one-problem plan);
    // otherwise the batch owns its plan.
    KBatch(int method, bool fp32, Plan *external = nullptr);
    ~KBatch();
    KBatch(const KBatch &) = delete;
    KBatch &operator=(const KBatch &) = delete;

    // Replaces the problem set (plan order).  Problems already started keep
    // their device state; their control blocks move to their new slots.
    hh_status set(const std::vector<KProb *> &probs);
    // ||b||, x = 0 unless given, r = b - H x and the method's first scalars,
    // for the listed problems of the current set.
    hh_status start(const std::vector<KProb *> &probs);
    // Enqueues K iterations of every running problem (one graph replay).
    hh_status launch();
    // Waits for them, handles stops (true-residual checks, restarts), and
    // closes finished problems: final FP64 true residual and info.  Appends
    // the problems closed by this call to `closed`.
    hh_status collect(std::vector<KProb *> &closed);
    int running() const;
    const std::vector<KProb *> &problems() const { return P_; }
    hipStream_t stream() const { return pl_->stream; }
    size_t device_bytes() const { return pl_->bytes + sub_bytes_; }

  private:
    hh_status sub_set(const std::vector<int> &which);
    hh_status read_states(const std::vector<int> &which);
    hh_status close(const std::vector<int> &which, std::vector<KProb *> &closed);
    int method_;
    bool fp32_;
    Plan own_;
    Plan *pl_;
    std::vector<KProb *> P_;
    std::vector<uint64_t> ids_;     // serials of P_ (P_ may hold problems freed since)
    uint64_t next_serial_ = 1;
    std::vector<Tile> ht_;
    std::vector<int> hp_;
    void *sub_mem_ = nullptr;
    size_t sub_bytes_ = 0;
    Tile *sub_t_ = nullptr;
    int *sub_p_ = nullptr;
    int K_;
    bool graph_;
    double stage_;          // mixed precision: each stage reduces the true residual by this factor
    double drift_grow_;
    int drift_stall_;
};

hh_status workspace_ensure(hh_grid *g, int method, bool fp32, int s, int hist_len);
hh_status check_solve_opts(const hh_grid *g, const hh_solve_opts *o);
