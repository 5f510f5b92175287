// hh_lib.h -- host-side objects of the library: grids, launch plans, solve
// work spaces, and the launchers the drivers use.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hh_common.h"
#include "hh_setup.h"
#include "../../include/hh.h"

struct DevList {
    Tile *t = nullptr;
    int n = 0;
};

// Tile lists of every pass for a fixed set of problems (one dimension, one
// V-cycle precision), plus the device array of their descriptors.
struct Plan {
    int count = 0, dim = 2, Lmax = 0;
    bool fp32 = false;
    DevList chunks, down[HH_MAXLEV], up[HH_MAXLEV];   // down/up: levels above the tail
    DevList coarse[5];               // k_coarse workgroups of problems with a split tail, by log2(seg)
    bool tail_down = false;          // some problem needs the (full or down-only) tail kernel
    bool tail_up = false;            // some problem needs the up-only tail kernel
    int vdv[HH_MAXLEV] = {}, vuv[HH_MAXLEV] = {};   // tile shape of each level's down- and up-leg
    // one 2D problem: the down-legs of levels mlev0 .. mlev0 + mK - 1 (ending at
    // the tail) run as one merged launch of mdn workgroups, the up-legs of
    // levels mlev0u .. mlev0u + mKup - 1 (ending at the tail too) as one of mup
    int mK = 0, mlev0 = 0, mdn = 0, mKup = 0, mlev0u = 0, mup = 0;
    int *fin = nullptr;
    int nfin = 0;
    ProbDev *probs = nullptr;
    Ctrl *ctrl = nullptr;            // per-problem control blocks (device)
    ProbDev pd1{};                   // one-problem plans: copy of the problem's static descriptor
    const void *L1 = nullptr;        // one-problem plans: LevelDev array of the V-cycle precision
    const LevelDev<double> *lv64h = nullptr;   // one-problem plans: host copies of its level descriptors
    const LevelDev<float> *lv32h = nullptr;
    double omega1 = 0.8;
    int nu1_1 = 1;                   // one-problem plans: pre-smoothing steps
    bool galerkin = false;           // one-problem plans: Galerkin coarse operators (levels >= 1)
    bool ilu = false;                // one-problem plans: ILU(0) up-legs (FP64, V(0,1))
    std::vector<ProbDev> host;       // host copies of the descriptors of the current solve
    void *mem = nullptr;
    size_t bytes = 0;
    // solve execution: an internal stream, K iterations captured as one
    // graph, a pinned copy of the control blocks
    hipStream_t stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gmethod = -1, gK = 0;
    ProbDev gpd{};                   // one-problem plans: the descriptor the graph was captured with
    Ctrl *hctrl = nullptr;
    int hcap = 0;                    // capacity of hctrl (problems)
};

// Solve work space of one grid.
struct Workspace {
    int method = -1, fp32 = -1, s = 0, hist_cap = 0;
    void *mem = nullptr;
    size_t bytes = 0;
    double2 *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *t = nullptr;
    void *ph = nullptr, *sh = nullptr;
    double2 *w = nullptr, *q = nullptr, *dR = nullptr, *dX = nullptr;
    void *wlow = nullptr;       // IDR: V-cycle output in the V-cycle precision
    double *part = nullptr;
    SolveState *st = nullptr;
    double *hist = nullptr;
};

struct hh_grid {
    HostSetup hs;
    hh_grid_desc desc{};
    bool host_only = false;
    int device = 0;
    void *dmem = nullptr;
    size_t dbytes = 0;
    const double2 *aH[3] = {}, *cH[3] = {}, *dH[3] = {};
    LevelDev<double> L64h[HH_MAXLEV] = {};
    LevelDev<float> L32h[HH_MAXLEV] = {};
    LevelDev<double> *L64 = nullptr;
    LevelDev<float> *L32 = nullptr;
    double2 *Minv64 = nullptr;
    float2 *Minv32 = nullptr;
    void *timg64 = nullptr, *timg32 = nullptr;
    TailTab *ttab64 = nullptr, *ttab32 = nullptr;   // tail level tables (see tail_table)
    size_t timg_bytes64 = 0, timg_bytes32 = 0;
    std::vector<uint32_t> tseg64, tseg32;   // segments of the tail images (see tail_image)
    ProbDev pd_static{};
    ProbDev *pd_static_dev = nullptr;
    Tile *chunks_dev = nullptr;
    int nchunks = 0;
    Plan vplan64, vplan32;   // single-problem V-cycle plans (static descriptor)
    // allocation-free V-cycle (hh_vcycle_noalloc): level descriptors whose f and
    // e (levels >= 1) point into the library's static scratch array of this
    // grid's device; scratch_need* = bytes of that layout per precision
    LevelDev<double> L64sh[HH_MAXLEV] = {};
    LevelDev<float> L32sh[HH_MAXLEV] = {};
    LevelDev<double> *L64s = nullptr;
    LevelDev<float> *L32s = nullptr;
    size_t scratch_need64 = 0, scratch_need32 = 0;
    bool scratch_ok = false;     // scratch address found and descriptors uploaded
    Plan plan;               // single-problem solve plan
    int plan_fp32 = -1;
    Workspace ws;
    size_t plan_bytes() const { return plan.bytes + vplan64.bytes + vplan32.bytes; }
};

hh_status hh_fail(hh_status st, const char *fmt, ...);
// the coarsest solve runs in k_coarse (many workgroups) rather than in the tail
bool coarse_split(const HostSetup &hs);
hh_status grid_create(HostSetup &&hs, const hh_grid_desc *d, hh_grid **out);
hh_status footprint_bytes(const hh_grid_desc *d, const hh_solve_opts *o, uint64_t &bytes, std::string &err);
size_t solve_workspace_bytes(int64_t N, int method, bool fp32, int s, int hist_len);
void grid_fill_prob(const hh_grid *g, ProbDev &pd);
hh_status grid_vplan(hh_grid *g, bool fp32);
void workspace_release(Workspace &w);
void plan_release(Plan &p);
hh_status plan_build(Plan &pl, const std::vector<const hh_grid *> &G, bool fp32);

void launch_vcycle(const Plan &pl, int fsel, int osel, const void *fptr, void *optr, hipStream_t s);
void launch_bicg_iteration(const Plan &pl, hipStream_t s);
void launch_idr_step(const Plan &pl, hipStream_t s);
void launch_resid(const Plan &pl, const DevList &tiles, int mode, hipStream_t s);
void launch_norm(const Plan &pl, const DevList &tiles, int sel, hipStream_t s);
void launch_zero(const Plan &pl, const DevList &tiles, int sel, hipStream_t s);
int tail_level(const HostSetup &hs, bool fp32);
std::vector<char> tail_image(const HostSetup &hs, bool fp32, std::vector<uint32_t> *seg);
void launch_fin(const Plan &pl, const int *probs, int n, int kind, hipStream_t s);
