// hh_lib.hip -- grids, launch plans, solver drivers and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "hh_common.h"
#include "hh_kernels.hpp"
#include "hh_idr_kernels.hpp"
#include "hh_lib.h"
#include "hh_setup.h"

using namespace hh;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

hh_status hh_fail(hh_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return hh_fail(HH_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// device arena: one hipMalloc carved into aligned pieces
// ---------------------------------------------------------------------------
struct Carver {
    char *base = nullptr;
    size_t used = 0;
    template <typename X> X *take(size_t count)
    {
        X *p = (X *)(base ? base + used : nullptr);
        used += align256(sizeof(X) * count);
        return p;
    }
};

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free V-cycle (hh_vcycle_noalloc): the
// restricted right-hand sides f_l and level solutions e_l of levels >= 1 live
// here instead of in the grid's memory.  Each device holds its own copy for
// the life of the process.  On the host, `scratch` only names the symbol;
// kernels get the device address hipGetSymbolAddress returns, looked up once
// per device while that device is current (at the first grid set up on it).
// ---------------------------------------------------------------------------
#define HH_SCRATCH_BYTES ((size_t)32 << 20)
static __device__ __align__(256) char scratch[HH_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_addr;

static hh_status scratch_address(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return HH_OK;
    }
    char *p = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return hh_fail(HH_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_addr[dev] = p;
    *out = p;
    return HH_OK;
}

// Byte offsets of f_l and e_l (levels >= 1) in the scratch array for one
// precision; returns the bytes the layout needs.
static size_t scratch_layout(const HostSetup &hs, bool fp32, size_t (*off)[2])
{
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
    size_t used = 0;
    for (int l = 1; l < hs.nlev; ++l) {
        off[l][0] = used;
        used += align256(cb * hs.lev[l].N);
        off[l][1] = used;
        used += align256(cb * hs.lev[l].N);
    }
    return used;
}

// ---------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------
template <typename T> static TailTab tail_table(const LevelDev<T> *Lh, const HostSetup &hs, bool fp32);

// a level's ILU(0) factors in the device layout of the up-leg kernels
// (IluLayout: by band, step and entry, lane-contiguous), from the host's 25
// planes of N points; the level's stencil is the Galerkin one (the 25-point
// sets) when it has Galerkin entries
static size_t ilu_device_count(const HostLevel &L)
{
    return L.gal.empty() ? (size_t)IluLayout<false>(L.n[0], L.n[1]).size()
                         : (size_t)IluLayout<true>(L.n[0], L.n[1]).size();
}
template <bool GAL> static void ilu_pack_set(const HostLevel &L, std::vector<double2> &out)
{
    using S = IluSet<GAL>;
    const IluLayout<GAL> lay(L.n[0], L.n[1]);
    const int nx = L.n[0];
    const int64_t N = L.N;
    for (int b = 0; b < lay.nb; ++b) {
        const int j0 = lay.j0(b), R = lay.j0(b + 1) - j0;
        for (int r = 0; r < R; ++r)
            for (int i = 0; i < nx; ++i) {
                const int j = j0 + r, t = lay.lane(r);
                const int64_t p = i + (int64_t)nx * j, dd = lay.d0(b) + i + S::M * r;
                // the entry of a neighbour outside the grid is +0 exactly: the
                // kernels multiply it by a +0 neighbour value
                auto entry = [&](int sk) {
                    const int ii = i + sk % 5 - 2, jj = j + sk / 5 - 2;
                    return ii >= 0 && ii < nx && jj >= 0 && jj < L.n[1] ? L.ilu[sk * N + p] : double2{0.0, 0.0};
                };
                for (int k = 0; k < S::NLO; ++k) out[lay.lo(dd, k, t)] = entry(S::lo(k));
                out[lay.up(dd, 0, t)] = L.ilu[12 * N + p];
                for (int k = 0; k < S::NLO; ++k) out[lay.up(dd, 1 + k, t)] = entry(S::up(k));
            }
    }
}
// the up-leg's work array: by point, or in the row form's step order
static size_t ilu_w_count(const HostLevel &L)
{
    const size_t d = L.gal.empty() ? (size_t)(IluLayout<false>(L.n[0], L.n[1]).DT * IluLayout<false>(L.n[0], L.n[1]).TS)
                                   : (size_t)(IluLayout<true>(L.n[0], L.n[1]).DT * IluLayout<true>(L.n[0], L.n[1]).TS);
    return std::max((size_t)L.N, d);
}
static std::vector<double2> ilu_device_pack(const HostLevel &L)
{
    std::vector<double2> out(ilu_device_count(L), double2{0.0, 0.0});
    if (L.gal.empty()) ilu_pack_set<false>(L, out);
    else ilu_pack_set<true>(L, out);
    return out;
}

hh_status grid_upload(hh_grid *g)
{
    const HostSetup &hs = g->hs;
    HIPCHK(hipGetDevice(&g->device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, g->device));
    // two passes: size, then carve
    for (int pass = 0; pass < 2; ++pass) {
        Carver c;
        if (pass == 1) {
            hipError_t e = hipMalloc((void **)&c.base, g->dbytes);
            if (e != hipSuccess) return hh_fail(HH_ERR_OOM, "hipMalloc(%zu) for the grid: %s", g->dbytes, hipGetErrorString(e));
            g->dmem = c.base;
        }
        for (int a = 0; a < hs.dim; ++a) {
            g->aH[a] = c.take<double2>(hs.aH[a].size());
            g->cH[a] = c.take<double2>(hs.cH[a].size());
            g->dH[a] = c.take<double2>(hs.dH[a].size());
        }
        for (int l = 0; l < hs.nlev; ++l) {
            const HostLevel &L = hs.lev[l];
            LevelDev<double> &D = g->L64h[l];
            LevelDev<float> &F = g->L32h[l];
            for (int a = 0; a < 3; ++a) { D.n[a] = L.n[a]; F.n[a] = L.n[a]; }
            D.N = F.N = L.N;
            D.fx = F.fx = make_fastdiv((uint32_t)L.n[0]);
            D.fxy = F.fxy = make_fastdiv((uint32_t)(L.n[0] * L.n[1]));
            for (int a = 0; a < 3; ++a) {
                if (a < hs.dim) {
                    D.a[a] = c.take<double2>(L.n[a]); D.c[a] = c.take<double2>(L.n[a]); D.d[a] = c.take<double2>(L.n[a]);
                    F.a[a] = c.take<float2>(L.n[a]); F.c[a] = c.take<float2>(L.n[a]); F.d[a] = c.take<float2>(L.n[a]);
                } else {
                    D.a[a] = D.c[a] = D.d[a] = nullptr;
                    F.a[a] = F.c[a] = F.d[a] = nullptr;
                }
            }
            D.phi = c.take<double>(L.N);
            F.phi = c.take<float>(L.N);
            if (l >= 1) {
                D.f = c.take<double2>(L.N); D.e = c.take<double2>(L.N);
                F.f = c.take<float2>(L.N); F.e = c.take<float2>(L.N);
            } else {
                D.f = D.e = nullptr;
                F.f = F.e = nullptr;
            }
            if (!L.gal.empty()) {
                D.g = c.take<double2>(L.gal.size());
                F.g = c.take<float2>(L.gal.size());
            } else {
                D.g = nullptr;
                F.g = nullptr;
            }
            F.ilu = nullptr;
            F.w = nullptr;
            if (!L.ilu.empty()) {
                D.ilu = c.take<double2>(ilu_device_count(L));
                D.w = c.take<double2>(ilu_w_count(L));
            } else {
                D.ilu = nullptr;
                D.w = nullptr;
            }
        }
        g->Minv64 = c.take<double2>((size_t)hs.Nc * hs.Nc);
        g->Minv32 = c.take<float2>((size_t)hs.Nc * hs.Nc);
        if (pass == 0) {
            g->timg_bytes64 = tail_image(hs, false, nullptr).size();
            g->timg_bytes32 = tail_image(hs, true, nullptr).size();
        }
        g->timg64 = c.take<char>(g->timg_bytes64);
        g->timg32 = c.take<char>(g->timg_bytes32);
        g->ttab64 = c.take<TailTab>(1);
        g->ttab32 = c.take<TailTab>(1);
        g->L64 = c.take<LevelDev<double>>(HH_MAXLEV);
        g->L32 = c.take<LevelDev<float>>(HH_MAXLEV);
        g->L64s = c.take<LevelDev<double>>(HH_MAXLEV);
        g->L32s = c.take<LevelDev<float>>(HH_MAXLEV);
        g->pd_static_dev = c.take<ProbDev>(1);
        g->chunks_dev = c.take<Tile>(ceil_div(hs.lev[0].N, HH_CHUNK));
        if (pass == 0) g->dbytes = c.used;
    }
    // host staging of every array, then one copy each
    std::vector<float2> tmp;
    auto put64 = [&](const void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpy((void *)dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    auto put32c = [&](const float2 *dst, const std::vector<double2> &src) {
        tmp.resize(src.size());
        for (size_t i = 0; i < src.size(); ++i) { tmp[i].x = (float)src[i].x; tmp[i].y = (float)src[i].y; }
        return tmp.empty() ? hipSuccess : hipMemcpy((void *)dst, tmp.data(), sizeof(float2) * tmp.size(), hipMemcpyHostToDevice);
    };
    for (int a = 0; a < hs.dim; ++a) {
        HIPCHK(put64(g->aH[a], hs.aH[a].data(), sizeof(double2) * hs.aH[a].size()));
        HIPCHK(put64(g->cH[a], hs.cH[a].data(), sizeof(double2) * hs.cH[a].size()));
        HIPCHK(put64(g->dH[a], hs.dH[a].data(), sizeof(double2) * hs.dH[a].size()));
    }
    for (int l = 0; l < hs.nlev; ++l) {
        const HostLevel &L = hs.lev[l];
        for (int a = 0; a < hs.dim; ++a) {
            HIPCHK(put64(g->L64h[l].a[a], L.aM[a].data(), sizeof(double2) * L.n[a]));
            HIPCHK(put64(g->L64h[l].c[a], L.cM[a].data(), sizeof(double2) * L.n[a]));
            HIPCHK(put64(g->L64h[l].d[a], L.dM[a].data(), sizeof(double2) * L.n[a]));
            HIPCHK(put32c(g->L32h[l].a[a], L.aM[a]));
            HIPCHK(put32c(g->L32h[l].c[a], L.cM[a]));
            HIPCHK(put32c(g->L32h[l].d[a], L.dM[a]));
        }
        HIPCHK(put64(g->L64h[l].phi, L.phi.data(), sizeof(double) * L.N));
        if (!L.gal.empty()) {
            HIPCHK(put64(g->L64h[l].g, L.gal.data(), sizeof(double2) * L.gal.size()));
            HIPCHK(put32c(g->L32h[l].g, L.gal));
        }
        if (!L.ilu.empty()) {
            const std::vector<double2> pk = ilu_device_pack(L);
            HIPCHK(put64(g->L64h[l].ilu, pk.data(), sizeof(double2) * pk.size()));
        }
        std::vector<float> p32(L.N);
        for (int64_t i = 0; i < L.N; ++i) p32[i] = (float)L.phi[i];
        HIPCHK(put64(g->L32h[l].phi, p32.data(), sizeof(float) * L.N));
    }
    HIPCHK(put64(g->Minv64, hs.Minv.data(), sizeof(double2) * hs.Minv.size()));
    {
        std::vector<char> i64 = tail_image(hs, false, &g->tseg64), i32 = tail_image(hs, true, &g->tseg32);
        HIPCHK(put64(g->timg64, i64.data(), i64.size()));
        HIPCHK(put64(g->timg32, i32.data(), i32.size()));
        const TailTab t64 = tail_table(g->L64h, hs, false), t32 = tail_table(g->L32h, hs, true);
        HIPCHK(put64(g->ttab64, &t64, sizeof t64));
        HIPCHK(put64(g->ttab32, &t32, sizeof t32));
    }
    HIPCHK(put32c(g->Minv32, hs.Minv));
    HIPCHK(put64(g->L64, g->L64h, sizeof(LevelDev<double>) * HH_MAXLEV));
    HIPCHK(put64(g->L32, g->L32h, sizeof(LevelDev<float>) * HH_MAXLEV));
    // the allocation-free V-cycle's descriptors: the same levels with f and e
    // of levels >= 1 in the device's scratch array
    {
        char *sp = nullptr;
        g->scratch_ok = false;
        if (scratch_address(g->device, &sp) == HH_OK) {
            size_t o64[HH_MAXLEV][2] = {}, o32[HH_MAXLEV][2] = {};
            g->scratch_need64 = scratch_layout(hs, false, o64);
            g->scratch_need32 = scratch_layout(hs, true, o32);
            for (int l = 0; l < HH_MAXLEV; ++l) {
                g->L64sh[l] = g->L64h[l];
                g->L32sh[l] = g->L32h[l];
                if (l >= 1 && l < hs.nlev) {
                    const bool fit64 = g->scratch_need64 <= HH_SCRATCH_BYTES, fit32 = g->scratch_need32 <= HH_SCRATCH_BYTES;
                    g->L64sh[l].f = fit64 ? (double2 *)(sp + o64[l][0]) : nullptr;
                    g->L64sh[l].e = fit64 ? (double2 *)(sp + o64[l][1]) : nullptr;
                    g->L32sh[l].f = fit32 ? (float2 *)(sp + o32[l][0]) : nullptr;
                    g->L32sh[l].e = fit32 ? (float2 *)(sp + o32[l][1]) : nullptr;
                }
            }
            HIPCHK(put64(g->L64s, g->L64sh, sizeof(LevelDev<double>) * HH_MAXLEV));
            HIPCHK(put64(g->L32s, g->L32sh, sizeof(LevelDev<float>) * HH_MAXLEV));
            g->scratch_ok = true;
        }
    }
    // static descriptor (no solve state) for hh_apply_operator / hh_vcycle
    ProbDev &pd = g->pd_static;
    grid_fill_prob(g, pd);
    HIPCHK(put64(g->pd_static_dev, &pd, sizeof(ProbDev)));
    std::vector<Tile> ch(ceil_div(hs.lev[0].N, HH_CHUNK));
    for (size_t i = 0; i < ch.size(); ++i) ch[i] = Tile{0, (int)i};
    HIPCHK(put64(g->chunks_dev, ch.data(), sizeof(Tile) * ch.size()));
    g->nchunks = (int)ch.size();
    return HH_OK;
}

void grid_fill_prob(const hh_grid *g, ProbDev &pd)
{
    const HostSetup &hs = g->hs;
    memset(&pd, 0, sizeof pd);
    pd.dim = hs.dim;
    pd.nlev = hs.nlev;
    pd.Nc = hs.Nc;
    for (int a = 0; a < 3; ++a) pd.n[a] = hs.lev[0].n[a];
    pd.N = hs.lev[0].N;
    pd.ngroup = ceil_div(pd.N, HH_SPAN);
    pd.fx = make_fastdiv((uint32_t)pd.n[0]);
    pd.fxy = make_fastdiv((uint32_t)(pd.n[0] * pd.n[1]));
    for (int a = 0; a < 3; ++a) {
        pd.aH[a] = a < hs.dim ? g->aH[a] : nullptr;
        pd.cH[a] = a < hs.dim ? g->cH[a] : nullptr;
        pd.dH[a] = a < hs.dim ? g->dH[a] : nullptr;
    }
    pd.phi = g->L64h[0].phi;
    pd.L64 = g->L64;
    pd.L32 = g->L32;
    pd.Minv64 = g->Minv64;
    pd.Minv32 = g->Minv32;
    pd.omega = hs.omega;
    pd.nu1 = hs.nu1;
    pd.tail64 = tail_level(hs, false);
    pd.tail32 = tail_level(hs, true);
    pd.csplit = coarse_split(hs) ? 1 : 0;
    pd.timg64 = g->timg64;
    pd.timg32 = g->timg32;
    pd.ttab64 = g->ttab64;
    pd.ttab32 = g->ttab32;
    pd.timg_bytes64 = (int)g->timg_bytes64;
    pd.timg_bytes32 = (int)g->timg_bytes32;
    pd.tnseg64 = (int)g->tseg64.size();
    pd.tnseg32 = (int)g->tseg32.size();
    for (int i = 0; i < HH_MAXLEV; ++i) {
        pd.tseg64[i] = i < pd.tnseg64 ? g->tseg64[i] : 0u;
        pd.tseg32[i] = i < pd.tnseg32 ? g->tseg32[i] : 0u;
    }
}

static void grid_release(hh_grid *g)
{
    if (!g) return;
    if (g->dmem) (void)hipFree(g->dmem);
    workspace_release(g->ws);
    plan_release(g->plan);
    delete g;
}

// ---------------------------------------------------------------------------
// Merged coarse legs (one 2D problem), each level exactly twice the next: the
// down-legs of the last K = 2 or 3 levels above the tail run as one launch,
// the up-legs of the last 2 to 4 (their regions stay small) as another.
// Down: C x C tiles of the tail's first level.  Up: UT x UT tiles of the
// first merged up level, UT = 16 over up to three levels and 32 over four
// (about 256 workgroups either way: more would not all be resident at once).
// NT threads (four waves per SIMD hide the LDS latency of the per-point
// chains).  At 1024^2 C = 2, UT = 16 is fastest of C in 1..4, UT in 8..32
// over three levels: more workgroups than that cost more in redundant halo
// work than they gain.  HH_MERGE=0 turns it off.
template <typename T> struct MergeTile;
template <> struct MergeTile<float> { static constexpr int C = 2, UT = 16, UT4 = 32, NT = 1024; };
template <> struct MergeTile<double> { static constexpr int C = 2, UT = 16, UT4 = 32, NT = 1024; };

static void plan_merge(Plan &pl, const hh_grid *const *G, int count, bool fp32)
{
    pl.mK = pl.mlev0 = pl.mdn = pl.mKup = pl.mlev0u = pl.mup = 0;
    if (const char *e = getenv("HH_MERGE"))
        if (atoi(e) == 0) return;
    if (count != 1 || G[0]->hs.dim != 2 || G[0]->host_only || G[0]->hs.coarse_op == HH_COARSE_GALERKIN ||
        G[0]->hs.smoother == HH_SMOOTH_ILU0)
        return;
    const HostSetup &hs = G[0]->hs;
    const int t = tail_level(hs, fp32), K = std::min(3, t - 1), Kup = std::min(4, t - 1);
    if (K < 2) return;
    for (int l = t - Kup; l < t; ++l)
        if (hs.lev[l].n[0] != 2 * hs.lev[l + 1].n[0] || hs.lev[l].n[1] != 2 * hs.lev[l + 1].n[1]) return;
    const int C = fp32 ? MergeTile<float>::C : MergeTile<double>::C;
    const int UT = Kup == 4 ? (fp32 ? MergeTile<float>::UT4 : MergeTile<double>::UT4)
                            : (fp32 ? MergeTile<float>::UT : MergeTile<double>::UT);
    pl.mK = K;
    pl.mlev0 = t - K;
    pl.mdn = ceil_div(hs.lev[t].n[0], C) * ceil_div(hs.lev[t].n[1], C);
    pl.mKup = Kup;
    pl.mlev0u = t - Kup;
    pl.mup = ceil_div(hs.lev[t - Kup].n[0], UT) * ceil_div(hs.lev[t - Kup].n[1], UT);
}

// launch plans: tile lists of every pass for a set of problems
// ---------------------------------------------------------------------------
static void tile_shape(int dim, int v, int &x, int &y, int &z)
{
    if (dim == 2) {
        x = TileSet<2>::X[v];
        y = TileSet<2>::Y[v];
        z = 1;
    } else {
        x = TileSet<3>::X[v];
        y = TileSet<3>::Y[v];
        z = TileSet<3>::Z[v];
    }
}

// workgroups of the down-leg (coarse tiles) and the up-leg (fine tiles of
// twice the size) of one level for tile shape v
static void vtile_counts(int dim, int v, const HostLevel &Lf, const HostLevel &Lc, int &ndown, int &nup)
{
    int CX, CY, CZ;
    tile_shape(dim, v, CX, CY, CZ);
    ndown = ceil_div(Lc.n[0], CX) * ceil_div(Lc.n[1], CY) * (dim == 3 ? ceil_div(Lc.n[2], CZ) : 1);
    nup = ceil_div(Lf.n[0], 2 * CX) * ceil_div(Lf.n[1], 2 * CY) * (dim == 3 ? ceil_div(Lf.n[2], 2 * CZ) : 1);
}

static int tune_leg(const hh_grid *g, bool fp32, int leg, int l);

void plan_release(Plan &p)
{
    if (p.gexec) (void)hipGraphExecDestroy(p.gexec);
    if (p.stream) (void)hipStreamDestroy(p.stream);
    if (p.hctrl) (void)hipHostFree(p.hctrl);
    if (p.mem) (void)hipFree(p.mem);
    p = Plan();
}

// LDS bytes the tail kernel carves for levels t..nlev-1 (same order and
// 16-byte rounding as k_vtail).
static size_t tail_bytes(const HostSetup &hs, int t, bool fp32)
{
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2), rb = fp32 ? sizeof(float) : sizeof(double);
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    size_t off = 0;
    int64_t nmax = 0;
    for (int l = t; l < hs.nlev; ++l) {
        const HostLevel &L = hs.lev[l];
        nmax = std::max(nmax, L.N);
        off += r16(cb * L.N) + r16(cb * L.N) + r16(rb * L.N);
        for (int a = 0; a < 3; ++a) {
            const int na = a < hs.dim ? L.n[a] : 1;
            off += 3 * r16(cb * na);
        }
    }
    off += r16(cb * nmax);
    return off;
}

bool coarse_split(const HostSetup &hs)
{
    return hs.Nc > HH_SPLIT_NC || hs.coarse_op == HH_COARSE_GALERKIN || hs.smoother == HH_SMOOTH_ILU0;
}

// First level of the one-workgroup tail: the finest level >= 1 whose level
// and every coarser one fit the tail's LDS budget.  A Galerkin or ILU(0)
// hierarchy has no tail levels (the tail kernel knows only the rediscretised
// stencil and weighted Jacobi): only its coarsest level, which k_coarse
// solves.
int tail_level(const HostSetup &hs, bool fp32)
{
    if (hs.coarse_op == HH_COARSE_GALERKIN || hs.smoother == HH_SMOOTH_ILU0) return hs.nlev - 1;
    const int cap = fp32 ? TailCap<float>::N : TailCap<double>::N;
    const size_t bytes = fp32 ? TailCap<float>::BYTES : TailCap<double>::BYTES;
    for (int t = 1; t < hs.nlev; ++t)
        if (hs.lev[t].N <= cap && tail_bytes(hs, t, fp32) <= bytes) return t;
    return hs.nlev - 1;
}

// Level table of the tail kernel: the layout of tail_bytes, level by level
// from the tail's first level, with each level's sizes and index dividers
// from its uploaded descriptor (Lh: host copies, either precision).
template <typename T> static TailTab tail_table(const LevelDev<T> *Lh, const HostSetup &hs, bool fp32)
{
    TailTab tab;
    memset(&tab, 0, sizeof tab);
    if (hs.nlev < 2) return tab;   // a one-level grid has no V-cycle
    const int t0 = tail_level(hs, fp32);
    const int cb = sizeof(V2<T>), rb = sizeof(T);
    auto r16 = [](int b) { return (b + 15) & ~15; };
    int off = 0;
    for (int l = t0; l < hs.nlev; ++l) {
        TailOff &o = tab.o[l];
        o.N = (int)Lh[l].N;
        for (int a = 0; a < 3; ++a) o.n[a] = Lh[l].n[a];
        o.F = off; off += r16(cb * o.N);
        o.E = off; off += r16(cb * o.N);
        o.PH = off; off += r16(rb * o.N);
        for (int a = 0; a < 3; ++a) {
            const int na = a < hs.dim ? o.n[a] : 1;
            o.A[a] = off; off += r16(cb * na);
            o.Cc[a] = off; off += r16(cb * na);
            o.Dd[a] = off; off += r16(cb * na);
        }
        o.end = off;
        tab.fx[l] = Lh[l].fx;
        tab.fxy[l] = Lh[l].fxy;
    }
    tab.uoff = off;
    return tab;
}

// Compact image of the tail's LDS block (layout of tail_bytes / k_vtail):
// for each tail level the bytes from its phi to the end of its coefficient
// arrays (a, c, d per axis), levels one after another, values in the V-cycle
// precision.  f, e and the scratch U are never read before the kernel writes
// them, so they are not part of the image.  seg[i] = (LDS offset of level
// t + i's phi in 16-byte units) << 16 | (its length in 16-byte units).
std::vector<char> tail_image(const HostSetup &hs, bool fp32, std::vector<uint32_t> *seg)
{
    if (hs.nlev < 2) {   // a one-level (vertex-centred) grid has no V-cycle
        if (seg) seg->clear();
        return std::vector<char>();
    }
    const int t = tail_level(hs, fp32);
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2), rb = fp32 ? sizeof(float) : sizeof(double);
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    std::vector<char> img;
    if (seg) seg->clear();
    size_t lds = 0;   // LDS offset of the next array
    size_t off = 0;   // image offset of the next array
    auto grow = [&](size_t b) { img.resize(off + r16(b), 0); };
    auto put_c = [&](const std::vector<double2> &v, size_t n) {
        grow(cb * n);
        for (size_t i = 0; i < n; ++i) {
            if (fp32) {
                float2 z;
                z.x = (float)v[i].x;
                z.y = (float)v[i].y;
                memcpy(&img[off + i * cb], &z, cb);
            } else {
                memcpy(&img[off + i * cb], &v[i], cb);
            }
        }
        off += r16(cb * n);
        lds += r16(cb * n);
    };
    for (int l = t; l < hs.nlev; ++l) {
        const HostLevel &L = hs.lev[l];
        lds += r16(cb * L.N) + r16(cb * L.N);   // f and e
        const size_t lds0 = lds, off0 = off;
        grow(rb * L.N);
        for (int64_t i = 0; i < L.N; ++i) {
            if (fp32) {
                float v = (float)L.phi[i];
                memcpy(&img[off + i * rb], &v, rb);
            } else {
                memcpy(&img[off + i * rb], &L.phi[i], rb);
            }
        }
        off += r16(rb * L.N);
        lds += r16(rb * L.N);
        for (int a = 0; a < 3; ++a) {
            if (a < hs.dim) {
                put_c(L.aM[a], L.n[a]);
                put_c(L.cM[a], L.n[a]);
                put_c(L.dM[a], L.n[a]);
            } else {
                const std::vector<double2> zero(1, double2{0.0, 0.0});
                put_c(zero, 1);
                put_c(zero, 1);
                put_c(zero, 1);
            }
        }
        if (seg) seg->push_back((uint32_t)(lds0 / 16) << 16 | (uint32_t)((off - off0) / 16));
    }
    return img;
}

hh_status plan_build(Plan &pl, const std::vector<const hh_grid *> &G, bool fp32)
{
    // a rebuilt plan keeps its stream and pinned control copy (grown below)
    hipStream_t keep_stream = pl.stream;
    Ctrl *keep_hctrl = pl.hctrl;
    int keep_hcap = pl.hcap;
    pl.stream = nullptr;
    pl.hctrl = nullptr;
    plan_release(pl);
    pl.stream = keep_stream;
    pl.hctrl = keep_hctrl;
    pl.hcap = keep_hcap;
    if ((int)G.size() > pl.hcap) {
        if (pl.hctrl) (void)hipHostFree(pl.hctrl);
        pl.hctrl = nullptr;
        pl.hcap = 0;
        HIPCHK(hipHostMalloc((void **)&pl.hctrl, sizeof(Ctrl) * G.size(), 0));
        pl.hcap = (int)G.size();
    }
    if (G.size() > 1)
        for (const hh_grid *g : G) {
            if (g->hs.coarse_op == HH_COARSE_GALERKIN)
                return hh_fail(HH_ERR_ARG, "Galerkin coarse operators are supported for single solves, not batches");
            if (g->hs.smoother == HH_SMOOTH_ILU0)
                return hh_fail(HH_ERR_ARG, "ILU(0) smoothing is supported for single solves, not batches");
        }
    if (fp32)
        for (const hh_grid *g : G)
            if (g->hs.smoother == HH_SMOOTH_ILU0)
                return hh_fail(HH_ERR_ARG, "ILU(0) smoothing runs in the FP64 V-cycle only (vcycle_prec HH_C128)");
    pl.count = (int)G.size();
    pl.dim = G.empty() ? 2 : G[0]->hs.dim;
    pl.fp32 = fp32;
    pl.Lmax = 0;
    std::vector<Tile> chunks, down[HH_MAXLEV], up[HH_MAXLEV], coarse[5];
    std::vector<int> fin;
    pl.tail_down = pl.tail_up = false;
    plan_merge(pl, G.data(), (int)G.size(), fp32);
    // tile shape per level and leg, tuned on the largest problem having the level
    for (int l = 0; l < HH_MAXLEV; ++l) {
        pl.vdv[l] = pl.vuv[l] = 0;
        if (pl.mK && l >= pl.mlev0) continue;   // merged levels (mlev0u <= mlev0)
        const hh_grid *rep = nullptr;
        for (const hh_grid *g : G)
            if (l < tail_level(g->hs, fp32) && (!rep || g->hs.lev[l].N > rep->hs.lev[l].N)) rep = g;
        if (!rep || rep->host_only) continue;
        pl.vdv[l] = tune_leg(rep, fp32, 0, l);
        if (!pl.mK || l < pl.mlev0u) pl.vuv[l] = tune_leg(rep, fp32, 1, l);
    }
    for (int q = 0; q < pl.count; ++q) {
        const HostSetup &hs = G[q]->hs;
        const int t = tail_level(hs, fp32);
        pl.Lmax = std::max(pl.Lmax, t);
        const bool split = coarse_split(hs);
        if (split) {
            const int nwg = ceil_div(fp32 ? coarse_waves<float>(hs.Nc) : coarse_waves<double>(hs.Nc), HH_WG / 64);
            int lg = 0;
            while ((1 << lg) < coarse_seg(hs.Nc)) ++lg;
            for (int i = 0; i < nwg; ++i) coarse[lg].push_back(Tile{q, i});
        }
        if (!split || t < hs.nlev - 1) pl.tail_down = true;
        if (split && t < hs.nlev - 1) pl.tail_up = true;
        const int ngr = ceil_div(hs.lev[0].N, HH_SPAN);
        for (int i = 0; i < ngr; ++i) chunks.push_back(Tile{q, i});
        for (int l = 0; l < t; ++l) {
            int nd, nu;
            vtile_counts(hs.dim, pl.vdv[l], hs.lev[l], hs.lev[l + 1], nd, nu);
            for (int i = 0; i < nd; ++i) down[l].push_back(Tile{q, i});
            vtile_counts(hs.dim, pl.vuv[l], hs.lev[l], hs.lev[l + 1], nd, nu);
            for (int i = 0; i < nu; ++i) up[l].push_back(Tile{q, i});
        }
        fin.push_back(q);
    }
    size_t bytes = align256(sizeof(Tile) * chunks.size()) +
                   align256(sizeof(int) * fin.size()) +
                   align256(sizeof(ProbDev) * pl.count) + align256(sizeof(Ctrl) * pl.count);
    for (int l = 0; l < HH_MAXLEV; ++l) bytes += align256(sizeof(Tile) * down[l].size()) + align256(sizeof(Tile) * up[l].size());
    for (int g = 0; g < 5; ++g) bytes += align256(sizeof(Tile) * coarse[g].size());
    hipError_t e = hipMalloc(&pl.mem, bytes);
    if (e != hipSuccess) return hh_fail(HH_ERR_OOM, "hipMalloc(%zu) for a launch plan: %s", bytes, hipGetErrorString(e));
    pl.bytes = bytes;
    Carver c;
    c.base = (char *)pl.mem;
    auto up_list = [&](std::vector<Tile> &v, DevList &d) -> hipError_t {
        d.n = (int)v.size();
        d.t = c.take<Tile>(v.size());
        return v.empty() ? hipSuccess : hipMemcpy(d.t, v.data(), sizeof(Tile) * v.size(), hipMemcpyHostToDevice);
    };
    HIPCHK(up_list(chunks, pl.chunks));
    for (int g = 0; g < 5; ++g) HIPCHK(up_list(coarse[g], pl.coarse[g]));
    for (int l = 0; l < HH_MAXLEV; ++l) {
        HIPCHK(up_list(down[l], pl.down[l]));
        HIPCHK(up_list(up[l], pl.up[l]));
    }
    pl.fin = c.take<int>(fin.size());
    pl.nfin = (int)fin.size();
    HIPCHK(hipMemcpy(pl.fin, fin.data(), sizeof(int) * fin.size(), hipMemcpyHostToDevice));
    pl.probs = c.take<ProbDev>(pl.count);
    pl.ctrl = c.take<Ctrl>(pl.count);
    if (pl.count == 1) {
        pl.galerkin = G[0]->hs.coarse_op == HH_COARSE_GALERKIN;
        pl.ilu = G[0]->hs.smoother == HH_SMOOTH_ILU0;
        pl.pd1 = G[0]->pd_static;
        pl.L1 = fp32 ? (const void *)G[0]->L32 : (const void *)G[0]->L64;
        pl.omega1 = G[0]->hs.omega;
        pl.nu1_1 = G[0]->hs.nu1;
        pl.lv64h = G[0]->L64h;
        pl.lv32h = G[0]->L32h;
    }
    return HH_OK;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define LAUNCH(kernel, n, stream, ...)                                                  \
    do {                                                                                \
        if ((n) > 0) hipLaunchKernelGGL(kernel, dim3(n), dim3(HH_WG), 0, stream, __VA_ARGS__); \
    } while (0)

// Krylov vector passes: workgroups of HH_GROUP chunks
#define LAUNCH_K(kernel, n, stream, ...)                                                 \
    do {                                                                                \
        if ((n) > 0) hipLaunchKernelGGL(kernel, dim3(n), dim3(HH_VWG), 0, stream, __VA_ARGS__); \
    } while (0)

// level kernels: workgroup size of tile shape v
#define LAUNCH_V(kernel, v, n, stream, ...)                                                          \
    do {                                                                                             \
        if ((n) > 0) hipLaunchKernelGGL(kernel, dim3(n), dim3(TileSet<DIM>::T[v]), 0, stream, __VA_ARGS__); \
    } while (0)

// launch context of a pass over `tiles` (a one-problem plan needs no tile
// list: the workgroup index is the tile index)
static Ctx ctx_of(const Plan &pl, const DevList &tiles)
{
    Ctx c;
    c.P = pl.probs;
    c.tiles = pl.count == 1 ? nullptr : tiles.t;
    c.ctrl = pl.ctrl;
    c.L = pl.count == 1 ? pl.L1 : nullptr;
    c.omega = pl.omega1;
    c.nu1 = pl.nu1_1;
    return c;
}

template <int DIM, typename T, typename TF>
static void launch_down_v(int v, int n, hipStream_t s, const Ctx &c, int lev, int fsel, const void *fptr,
                          const LvPair<T> &lp)
{
    switch (v) {
    case 0: LAUNCH_V((k_vdown<DIM, T, TF, 0>), 0, n, s, c, lev, fsel, fptr, lp); break;
    case 1: LAUNCH_V((k_vdown<DIM, T, TF, 1>), 1, n, s, c, lev, fsel, fptr, lp); break;
    case 2: LAUNCH_V((k_vdown<DIM, T, TF, 2>), 2, n, s, c, lev, fsel, fptr, lp); break;
    case 3: LAUNCH_V((k_vdown<DIM, T, TF, 3>), 3, n, s, c, lev, fsel, fptr, lp); break;
    case 4: LAUNCH_V((k_vdown<DIM, T, TF, 4>), 4, n, s, c, lev, fsel, fptr, lp); break;
    case 5: LAUNCH_V((k_vdown<DIM, T, TF, 5>), 5, n, s, c, lev, fsel, fptr, lp); break;
    case 6: LAUNCH_V((k_vdown<DIM, T, TF, 6>), 6, n, s, c, lev, fsel, fptr, lp); break;
    default:
        if constexpr (DIM == 3) {
            if (v == 7) LAUNCH_V((k_vdown_z<T, TF, 7>), 7, n, s, c, lev, fsel, fptr, lp);
            else LAUNCH_V((k_vdown_z<T, TF, 8>), 8, n, s, c, lev, fsel, fptr, lp);
        } else {
            LAUNCH_V((k_vdown<DIM, T, TF, 7>), 7, n, s, c, lev, fsel, fptr, lp);
        }
        break;
    }
}

template <int DIM, typename T, typename TF, typename TO>
static void launch_up_v(int v, int n, hipStream_t s, const Ctx &c, int lev, int fsel, int osel, const void *fptr,
                        void *optr, const LvPair<T> &lp)
{
    switch (v) {
    case 0: LAUNCH_V((k_vup<DIM, T, TF, TO, 0>), 0, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    case 1: LAUNCH_V((k_vup<DIM, T, TF, TO, 1>), 1, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    case 2: LAUNCH_V((k_vup<DIM, T, TF, TO, 2>), 2, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    case 3: LAUNCH_V((k_vup<DIM, T, TF, TO, 3>), 3, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    case 4: LAUNCH_V((k_vup<DIM, T, TF, TO, 4>), 4, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    case 5: LAUNCH_V((k_vup<DIM, T, TF, TO, 5>), 5, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    case 6: LAUNCH_V((k_vup<DIM, T, TF, TO, 6>), 6, n, s, c, lev, fsel, osel, fptr, optr, lp); break;
    default:
        if constexpr (DIM == 3) {
            if (v == 7) LAUNCH_V((k_vup_z<T, TF, TO, 7>), 7, n, s, c, lev, fsel, osel, fptr, optr, lp);
            else LAUNCH_V((k_vup_z<T, TF, TO, 8>), 8, n, s, c, lev, fsel, osel, fptr, optr, lp);
        } else {
            LAUNCH_V((k_vup<DIM, T, TF, TO, 7>), 7, n, s, c, lev, fsel, osel, fptr, optr, lp);
        }
        break;
    }
}

// the streaming forms of the 2D FP32 finest-level legs (k_vdown / k_vup with
// ST = true), for levels of at least HH_STREAM_MIN unknowns; HH_STREAM=0
// keeps the plain forms (same values, bit for bit)
static bool stream_legs()
{
    const char *e = getenv("HH_STREAM");
    return !e || atoi(e) != 0;
}
static void launch_down_stream(int v, int n, hipStream_t s, const Ctx &c, int fsel, const void *fptr,
                               const LvPair<float> &lp)
{
    constexpr int DIM = 2;
    switch (v) {
    case 0: LAUNCH_V((k_vdown<2, float, double2, 0, true>), 0, n, s, c, 0, fsel, fptr, lp); break;
    case 1: LAUNCH_V((k_vdown<2, float, double2, 1, true>), 1, n, s, c, 0, fsel, fptr, lp); break;
    case 2: LAUNCH_V((k_vdown<2, float, double2, 2, true>), 2, n, s, c, 0, fsel, fptr, lp); break;
    case 3: LAUNCH_V((k_vdown<2, float, double2, 3, true>), 3, n, s, c, 0, fsel, fptr, lp); break;
    case 4: LAUNCH_V((k_vdown<2, float, double2, 4, true>), 4, n, s, c, 0, fsel, fptr, lp); break;
    case 5: LAUNCH_V((k_vdown<2, float, double2, 5, true>), 5, n, s, c, 0, fsel, fptr, lp); break;
    case 6: LAUNCH_V((k_vdown<2, float, double2, 6, true>), 6, n, s, c, 0, fsel, fptr, lp); break;
    default: LAUNCH_V((k_vdown<2, float, double2, 7, true>), 7, n, s, c, 0, fsel, fptr, lp); break;
    }
}
static void launch_up_stream(int v, int n, hipStream_t s, const Ctx &c, int fsel, int osel, const void *fptr, void *optr,
                             const LvPair<float> &lp)
{
    constexpr int DIM = 2;
    switch (v) {
    case 0: LAUNCH_V((k_vup<2, float, double2, float2, 0, true>), 0, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    case 1: LAUNCH_V((k_vup<2, float, double2, float2, 1, true>), 1, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    case 2: LAUNCH_V((k_vup<2, float, double2, float2, 2, true>), 2, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    case 3: LAUNCH_V((k_vup<2, float, double2, float2, 3, true>), 3, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    case 4: LAUNCH_V((k_vup<2, float, double2, float2, 4, true>), 4, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    case 5: LAUNCH_V((k_vup<2, float, double2, float2, 5, true>), 5, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    case 6: LAUNCH_V((k_vup<2, float, double2, float2, 6, true>), 6, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    default: LAUNCH_V((k_vup<2, float, double2, float2, 7, true>), 7, n, s, c, 0, fsel, osel, fptr, optr, lp); break;
    }
}

// host copies of one problem's level descriptors (null for a batch)
struct LvHost {
    const LevelDev<double> *d = nullptr;
    const LevelDev<float> *f = nullptr;
};
template <typename T> static const LevelDev<T> *lv_of(const LvHost &h);
template <> const LevelDev<double> *lv_of<double>(const LvHost &h) { return h.d; }
template <> const LevelDev<float> *lv_of<float>(const LvHost &h) { return h.f; }

// one launch of level lev's down- (leg 0) or up-leg (leg 1) with tile shape v
template <int DIM, typename T>
static void launch_leg(int leg, int v, int n, hipStream_t s, const Ctx &c, int lev, int fsel, int osel,
                       const void *fptr, void *optr, const LvHost &lh)
{
    using C = V2<T>;
    LvPair<T> lp;
    memset(&lp, 0, sizeof lp);
    if (const LevelDev<T> *L = lv_of<T>(lh)) {
        lp.f = L[lev];
        lp.c = L[lev + 1];
        lp.valid = 1;
    }
    if constexpr (DIM == 2 && std::is_same<T, float>::value) {
        if (lev == 0 && lp.valid && lp.f.N >= HH_STREAM_MIN && stream_legs()) {
            if (leg == 0) launch_down_stream(v, n, s, c, fsel, fptr, lp);
            else launch_up_stream(v, n, s, c, fsel, osel, fptr, optr, lp);
            return;
        }
    }
    if (leg == 0) {
        if (lev == 0) launch_down_v<DIM, T, double2>(v, n, s, c, lev, fsel, fptr, lp);
        else launch_down_v<DIM, T, C>(v, n, s, c, lev, fsel, fptr, lp);
    } else {
        if (lev == 0) launch_up_v<DIM, T, double2, C>(v, n, s, c, lev, fsel, osel, fptr, optr, lp);
        else launch_up_v<DIM, T, C, C>(v, n, s, c, lev, fsel, osel, fptr, optr, lp);
    }
}

static void launch_leg_any(int dim, bool fp32, int leg, int v, int n, hipStream_t s, const Ctx &c, int lev, int fsel,
                           int osel, const void *fptr, void *optr, const LvHost &lh)
{
    if (dim == 2) {
        if (fp32) launch_leg<2, float>(leg, v, n, s, c, lev, fsel, osel, fptr, optr, lh);
        else launch_leg<2, double>(leg, v, n, s, c, lev, fsel, osel, fptr, optr, lh);
    } else {
        if (fp32) launch_leg<3, float>(leg, v, n, s, c, lev, fsel, osel, fptr, optr, lh);
        else launch_leg<3, double>(leg, v, n, s, c, lev, fsel, osel, fptr, optr, lh);
    }
}

// ---------------------------------------------------------------------------
// tile autotuner: the fastest shape per (dimension, precision, leg, finest
// level or not, log2 of the level's unknowns), timed on the grid at hand the
// first time such a level is planned, then cached for the process.
// HH_TILE=v forces shape v everywhere; HH_TUNE=0 keeps shape 0.
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::array<int, 5>, int> g_tune;

static int tune_leg(const hh_grid *g, bool fp32, int leg, int l)
{
    if (const char *e = getenv("HH_TILE")) return std::min(std::max(atoi(e), 0), tile_shapes(g->hs.dim) - 1);
    if (const char *e = getenv("HH_TUNE"))
        if (atoi(e) == 0) return 0;
    const HostSetup &hs = g->hs;
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= hs.lev[l].N) ++lg;
    const std::array<int, 5> key{hs.dim, (int)fp32, leg, l == 0 ? 0 : 1, lg};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    // time every shape on this grid's level (inputs of level 0 from a
    // scratch buffer; the level arrays it writes are rewritten by every use).
    // Shapes are timed round-robin (a warm-up round, then NR timed rounds of
    // RL back-to-back launches each, no host wait in between) so that clock
    // and cache drift affect every shape alike; the median round decides.
    constexpr int NR = 5, RL = 3;
    int best = 0;
    const int64_t N0 = hs.lev[0].N;
    void *in = nullptr, *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev[HH_NTILE][NR][2] = {};
    bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (int v = 0; v < HH_NTILE && ok; ++v)
        for (int r = 0; r < NR && ok; ++r)
            ok = hipEventCreate(&ev[v][r][0]) == hipSuccess && hipEventCreate(&ev[v][r][1]) == hipSuccess;
    if (ok && l == 0)
        ok = hipMalloc(&in, sizeof(double2) * N0) == hipSuccess && hipMalloc(&out, sizeof(double2) * N0) == hipSuccess &&
             hipMemsetAsync(in, 0, sizeof(double2) * N0, st) == hipSuccess;
    if (ok) {
        Ctx c;
        c.P = g->pd_static_dev;
        c.tiles = nullptr;
        c.ctrl = nullptr;
        c.L = fp32 ? (const void *)g->L32 : (const void *)g->L64;
        c.omega = hs.omega;
        c.nu1 = hs.nu1;
        LvHost lh;
        lh.d = g->L64h;
        lh.f = g->L32h;
        const int ns = tile_shapes(hs.dim);
        int nt[HH_NTILE];
        for (int v = 0; v < ns; ++v) {
            int nd, nu;
            vtile_counts(hs.dim, v, hs.lev[l], hs.lev[l + 1], nd, nu);
            nt[v] = leg == 0 ? nd : nu;
        }
        for (int v = 0; v < ns; ++v)
            for (int q = 0; q < RL; ++q) launch_leg_any(hs.dim, fp32, leg, v, nt[v], st, c, l, VS_IN, VS_OUT, in, out, lh);
        for (int r = 0; r < NR && ok; ++r)
            for (int v = 0; v < ns && ok; ++v) {
                ok = hipEventRecord(ev[v][r][0], st) == hipSuccess;
                for (int q = 0; q < RL; ++q) launch_leg_any(hs.dim, fp32, leg, v, nt[v], st, c, l, VS_IN, VS_OUT, in, out, lh);
                ok = ok && hipEventRecord(ev[v][r][1], st) == hipSuccess;
            }
        ok = ok && hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess;
        float bt = 0.f, tv[HH_NTILE] = {};
        for (int v = 0; v < ns && ok; ++v) {
            float rep[NR];
            for (int r = 0; r < NR && ok; ++r) ok = hipEventElapsedTime(&rep[r], ev[v][r][0], ev[v][r][1]) == hipSuccess;
            if (!ok) break;
            std::sort(rep, rep + NR);
            tv[v] = rep[NR / 2] / RL;
            if (v == 0 || tv[v] < bt) {
                bt = tv[v];
                best = v;
            }
        }
        if (ok && getenv("HH_TUNE_LOG")) {
            fprintf(stderr, "hh tile tune: dim %d %s leg %s level %s 2^%d unknowns:", hs.dim, fp32 ? "c64" : "c128",
                    leg == 0 ? "down" : "up", l == 0 ? "finest" : "coarse", lg);
            for (int v = 0; v < ns; ++v) fprintf(stderr, " %.1f", tv[v] * 1e3f);
            fprintf(stderr, " us -> shape %d\n", best);
        }
    }
    if (st) (void)hipStreamSynchronize(st);
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
    for (int v = 0; v < HH_NTILE; ++v)
        for (int r = 0; r < NR; ++r)
            for (int q = 0; q < 2; ++q)
                if (ev[v][r][q]) (void)hipEventDestroy(ev[v][r][q]);
    if (st) (void)hipStreamDestroy(st);
    if (!ok) return 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return best;
}

// The shape tune_leg would use, without timing anything: forced, cached by
// an earlier plan of the same class, or shape 0 (shapes never change results).
static int tune_cached(const hh_grid *g, bool fp32, int leg, int l)
{
    if (const char *e = getenv("HH_TILE")) return std::min(std::max(atoi(e), 0), tile_shapes(g->hs.dim) - 1);
    const HostSetup &hs = g->hs;
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= hs.lev[l].N) ++lg;
    const std::array<int, 5> key{hs.dim, (int)fp32, leg, l == 0 ? 0 : 1, lg};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    return it != g_tune.end() ? it->second : 0;
}

// A one-problem V-cycle plan built on the host only: one-problem launches
// take the workgroup index as the tile index and read nothing from a plan's
// device lists, so no device memory, stream or timing is involved.  The level
// descriptors (device array L1, host copies lv64h/lv32h) are the caller's.
static void plan_host_one(Plan &pl, const hh_grid *g, bool fp32, const void *L1, const LevelDev<double> *lv64h,
                          const LevelDev<float> *lv32h)
{
    const HostSetup &hs = g->hs;
    pl.count = 1;
    pl.dim = hs.dim;
    pl.fp32 = fp32;
    const hh_grid *G[1] = {g};
    plan_merge(pl, G, 1, fp32);
    const int t = tail_level(hs, fp32);
    pl.Lmax = t;
    for (int l = 0; l < HH_MAXLEV; ++l) {
        pl.vdv[l] = pl.vuv[l] = 0;
        pl.down[l].n = pl.up[l].n = 0;
        if (l >= t || (pl.mK && l >= pl.mlev0)) continue;
        pl.vdv[l] = tune_cached(g, fp32, 0, l);
        if (!pl.mK || l < pl.mlev0u) pl.vuv[l] = tune_cached(g, fp32, 1, l);
    }
    for (int l = 0; l < t; ++l) {
        int nd, nu;
        vtile_counts(hs.dim, pl.vdv[l], hs.lev[l], hs.lev[l + 1], nd, nu);
        pl.down[l].n = nd;
        vtile_counts(hs.dim, pl.vuv[l], hs.lev[l], hs.lev[l + 1], nd, nu);
        pl.up[l].n = nu;
    }
    for (int q = 0; q < 5; ++q) pl.coarse[q].n = 0;
    const bool split = coarse_split(hs);
    if (split) {
        int lg = 0;
        while ((1 << lg) < coarse_seg(hs.Nc)) ++lg;
        pl.coarse[lg].n = ceil_div(fp32 ? coarse_waves<float>(hs.Nc) : coarse_waves<double>(hs.Nc), HH_WG / 64);
    }
    pl.tail_down = !split || t < hs.nlev - 1;
    pl.tail_up = split && t < hs.nlev - 1;
    pl.chunks.n = ceil_div(hs.lev[0].N, HH_SPAN);
    pl.nfin = 1;
    pl.probs = g->pd_static_dev;
    pl.ctrl = nullptr;
    pl.pd1 = g->pd_static;
    pl.galerkin = hs.coarse_op == HH_COARSE_GALERKIN;
    pl.ilu = hs.smoother == HH_SMOOTH_ILU0;
    pl.L1 = L1;
    pl.omega1 = hs.omega;
    pl.nu1_1 = hs.nu1;
    pl.lv64h = lv64h;
    pl.lv32h = lv32h;
}

// the merged down- (leg 0) or up-leg (leg 1) of a one-problem 2D plan
template <typename T, int K>
static void launch_merged_k(int leg, const Plan &pl, hipStream_t s, const LevelDev<T> *L)
{
    LvChain<T, K> lc;
    const int l0 = leg == 0 ? pl.mlev0 : pl.mlev0u;
    for (int k = 0; k <= K; ++k) lc.L[k] = L[l0 + k];
    const Ctx c = ctx_of(pl, pl.chunks);
    constexpr int NT = MergeTile<T>::NT;
    constexpr int UT = K == 4 ? MergeTile<T>::UT4 : MergeTile<T>::UT;
    if (leg == 0) {
        if constexpr (K <= 3) hipLaunchKernelGGL((k_vdown_m<T, K, MergeTile<T>::C, NT>), dim3(pl.mdn), dim3(NT), 0, s, c, lc);
    } else {
        hipLaunchKernelGGL((k_vup_m<T, K, UT, NT>), dim3(pl.mup), dim3(NT), 0, s, c, lc);
    }
}
template <typename T>
static void launch_merged(int leg, const Plan &pl, hipStream_t s, const LvHost &lh)
{
    const LevelDev<T> *L = lv_of<T>(lh);
    const int K = leg == 0 ? pl.mK : pl.mKup;
    if (K == 2) launch_merged_k<T, 2>(leg, pl, s, L);
    else if (K == 3) launch_merged_k<T, 3>(leg, pl, s, L);
    else launch_merged_k<T, 4>(leg, pl, s, L);
}

// the fused legs of Galerkin level l >= 1 of a one-problem 2D plan (leg 0
// down, 1 up), with the level descriptors' host copies
template <typename T> static void launch_gal_leg(int leg, const Plan &pl, int l, hipStream_t s, const LvHost &lh)
{
    const LevelDev<T> *L = lv_of<T>(lh);
    const LevelDev<T> &F = L[l], &Cs = L[l + 1];
    GalArgs<T> a;
    a.G = F.g;
    a.f = F.f;
    a.e = F.e;
    a.fc = Cs.f;
    a.ec = Cs.e;
    a.nfx = F.n[0];
    a.nfy = F.n[1];
    a.ncx = Cs.n[0];
    a.ncy = Cs.n[1];
    a.omega = (T)pl.omega1;
    a.pre = pl.nu1_1;
    const Ctx c = ctx_of(pl, pl.chunks);
    if (leg == 0) {
        const int n = ceil_div(a.ncx, GAL_C) * ceil_div(a.ncy, GAL_C);
        hipLaunchKernelGGL((k_gdown<T>), dim3(n), dim3(GAL_NT), 0, s, c, a);
    } else {
        const int n = ceil_div(a.nfx, 2 * GAL_C) * ceil_div(a.nfy, 2 * GAL_C);
        hipLaunchKernelGGL((k_gup<T>), dim3(n), dim3(GAL_NT), 0, s, c, a);
    }
}

// tail arguments of a one-problem plan, from its copy of the problem's static
// descriptor and host copies of its level descriptors
template <typename T> static TailArgs<T> tail_args(const Plan &pl)
{
    const ProbDev &h = pl.pd1;
    constexpr bool f32 = sizeof(T) == 4;
    const LevelDev<T> *lvh = (const LevelDev<T> *)(f32 ? (const void *)pl.lv32h : (const void *)pl.lv64h);
    TailArgs<T> a{};
    a.t0 = f32 ? h.tail32 : h.tail64;
    a.L = h.nlev;
    a.Nc = h.Nc;
    a.split = h.csplit;
    a.nu1 = h.nu1;
    a.omega = (T)h.omega;
    a.Lv = (const LevelDev<T> *)pl.L1;
    a.f_top = lvh[a.t0].f;
    a.e_top = lvh[a.t0].e;
    a.Minv = (const V2<T> *)(f32 ? (const void *)h.Minv32 : (const void *)h.Minv64);
    a.img = f32 ? h.timg32 : h.timg64;
    a.tab = f32 ? h.ttab32 : h.ttab64;
    a.n16 = (f32 ? h.timg_bytes32 : h.timg_bytes64) / 16;
    a.nseg = f32 ? h.tnseg32 : h.tnseg64;
    memcpy(a.seg, f32 ? h.tseg32 : h.tseg64, sizeof a.seg);
    return a;
}

template <int DIM, typename T>
static void vcycle_t(const Plan &pl, int fsel, int osel, const void *fptr, void *optr, hipStream_t s)
{
    if (pl.count == 1 && !fptr) {
        fptr = pl.host.at(0).vec[fsel];
        optr = pl.host.at(0).vec[osel];
    }
    LvHost lh;
    if (pl.count == 1) {
        lh.d = pl.lv64h;
        lh.f = pl.lv32h;
    }
    const int lsplit = pl.mK ? pl.mlev0 : pl.Lmax;   // first merged level
    for (int l = 0; l < lsplit; ++l) {
        if (pl.galerkin && l >= 1) launch_gal_leg<T>(0, pl, l, s, lh);
        else launch_leg<DIM, T>(0, pl.vdv[l], pl.down[l].n, s, ctx_of(pl, pl.down[l]), l, fsel, osel, fptr, optr, lh);
    }
    if (pl.mK) launch_merged<T>(0, pl, s, lh);
    {
        // coarse part: tail kernel (whole, or down-legs of split problems),
        // multi-workgroup coarsest solves, up-legs of split problems
        Ctx c = ctx_of(pl, pl.chunks);
        const int *probs = pl.count == 1 ? nullptr : pl.fin;
        if (pl.nfin > 0 && pl.tail_down) {
            if (pl.count == 1)
                hipLaunchKernelGGL((k_vtail<DIM, T, true>), dim3(1), dim3(TailCap<T>::WG), 0, s, c, nullptr, 0, tail_args<T>(pl));
            else
                hipLaunchKernelGGL((k_vtail<DIM, T, false>), dim3(pl.nfin), dim3(TailCap<T>::WG), 0, s, c, probs, 0, TailArgs<T>{});
        }
        LAUNCH((k_coarse<T, 1>), pl.coarse[0].n, s, ctx_of(pl, pl.coarse[0]));
        LAUNCH((k_coarse<T, 2>), pl.coarse[1].n, s, ctx_of(pl, pl.coarse[1]));
        LAUNCH((k_coarse<T, 4>), pl.coarse[2].n, s, ctx_of(pl, pl.coarse[2]));
        LAUNCH((k_coarse<T, 8>), pl.coarse[3].n, s, ctx_of(pl, pl.coarse[3]));
        LAUNCH((k_coarse<T, 16>), pl.coarse[4].n, s, ctx_of(pl, pl.coarse[4]));
        if (pl.nfin > 0 && pl.tail_up) {
            if (pl.count == 1)
                hipLaunchKernelGGL((k_vtail<DIM, T, true>), dim3(1), dim3(TailCap<T>::WG), 0, s, c, nullptr, 1, tail_args<T>(pl));
            else
                hipLaunchKernelGGL((k_vtail<DIM, T, false>), dim3(pl.nfin), dim3(TailCap<T>::WG), 0, s, c, probs, 1, TailArgs<T>{});
        }
    }
    if (pl.mK) launch_merged<T>(1, pl, s, lh);
    if constexpr (DIM == 2 && std::is_same<T, double>::value) {
        if (pl.ilu) {
            // ILU(0) up-legs (one problem): one workgroup per level
            const Ctx c = ctx_of(pl, pl.chunks);
            for (int l = pl.Lmax - 1; l >= 0; --l) {
                IluArgs a;
                a.fl = lh.d[l];
                a.cl = lh.d[l + 1];
                a.f = l == 0 ? (const double2 *)fptr : lh.d[l].f;
                a.u = l == 0 ? (double2 *)optr : lh.d[l].e;
                a.omega = pl.omega1;
                // the pipelined row form with the recent diagonals in LDS,
                // in bands where a level has more rows than the workgroup
                // threads (then its rows must fit the LDS halo), and w in its
                // step order; HH_ILU_GLOBAL: the global-memory form on every
                // level
                const bool rows = !getenv("HH_ILU_GLOBAL");
                const int nx = a.fl.n[0], ny = a.fl.n[1];
                const int form = !rows ? 0
                                 : a.fl.g ? (ny <= IluSet<true>::NT || nx <= IluSet<true>::HMAX ? 1 : 0)
                                          : (ny <= IluSet<false>::NT || nx <= IluSet<false>::HMAX ? 2 : 0);
                a.diag = form != 0;
                // levels of few rows take a workgroup of as few waves (the same
                // layout: one band either way)
                const int wg = form == 1 ? (ny <= 64 ? 64 : ny <= 128 ? 128 : IluSet<true>::NT)
                                         : form == 2 ? IluSet<false>::NT : HH_ILU_WG;
                // the pointwise phases run grid-wide except on levels of at
                // most HH_ILU_INNER_MAX points in a full-size workgroup
                // (HH_ILU_FUSED: inside the solve kernel always)
                a.inner = ((a.fl.N <= HH_ILU_INNER_MAX && wg >= 512) || getenv("HH_ILU_FUSED")) ? 1 : 0;
                const dim3 pg((unsigned)((a.fl.N + HH_ILU_PW - 1) / HH_ILU_PW));
                if (!a.inner) {
                    hipLaunchKernelGGL(k_ilu_prolong, pg, dim3(HH_ILU_PW), 0, s, c, a);
                    hipLaunchKernelGGL(k_ilu_resid, pg, dim3(HH_ILU_PW), 0, s, c, a);
                }
                // one band of more rows than threads: the multi-row instance
                const bool multi = form == 1 ? IluLayout<true>(nx, ny).nb == 1 && ny > IluSet<true>::NT
                                             : form == 2 && IluLayout<false>(nx, ny).nb == 1 && ny > IluSet<false>::NT;
                if (form == 1 && wg == 64)
                    hipLaunchKernelGGL((k_ilu_up_rows<true, 64, false>), dim3(1), dim3(64), 0, s, c, a);
                else if (form == 1 && wg == 128)
                    hipLaunchKernelGGL((k_ilu_up_rows<true, 128, false>), dim3(1), dim3(128), 0, s, c, a);
                else if (form == 1 && multi)
                    hipLaunchKernelGGL((k_ilu_up_rows<true, IluSet<true>::NT, true>), dim3(1), dim3(IluSet<true>::NT), 0, s, c, a);
                else if (form == 1)
                    hipLaunchKernelGGL((k_ilu_up_rows<true, IluSet<true>::NT, false>), dim3(1), dim3(IluSet<true>::NT), 0, s, c, a);
                else if (form == 2 && multi)
                    hipLaunchKernelGGL((k_ilu_up_rows<false, IluSet<false>::NT, true>), dim3(1), dim3(IluSet<false>::NT), 0, s, c, a);
                else if (form == 2)
                    hipLaunchKernelGGL((k_ilu_up_rows<false, IluSet<false>::NT, false>), dim3(1), dim3(IluSet<false>::NT), 0, s, c, a);
                else
                    hipLaunchKernelGGL(k_ilu_up, dim3(1), dim3(HH_ILU_WG), 0, s, c, a);
                if (!a.inner) hipLaunchKernelGGL(k_ilu_update, pg, dim3(HH_ILU_PW), 0, s, c, a);
            }
            return;
        }
    }
    for (int l = (pl.mK ? pl.mlev0u : pl.Lmax) - 1; l >= 0; --l) {
        if (pl.galerkin && l >= 1) launch_gal_leg<T>(1, pl, l, s, lh);
        else launch_leg<DIM, T>(1, pl.vuv[l], pl.up[l].n, s, ctx_of(pl, pl.up[l]), l, fsel, osel, fptr, optr, lh);
    }
}

void launch_vcycle(const Plan &pl, int fsel, int osel, const void *fptr, void *optr, hipStream_t s)
{
    if (pl.dim == 2) {
        if (pl.fp32) vcycle_t<2, float>(pl, fsel, osel, fptr, optr, s);
        else vcycle_t<2, double>(pl, fsel, osel, fptr, optr, s);
    } else {
        if (pl.fp32) vcycle_t<3, float>(pl, fsel, osel, fptr, optr, s);
        else vcycle_t<3, double>(pl, fsel, osel, fptr, optr, s);
    }
}

void launch_fin(const Plan &pl, const int *probs, int n, int kind, hipStream_t s)
{
    if (pl.count == 1 && !pl.host.empty()) {
        if (n > 0) hipLaunchKernelGGL(k_fin1, dim3(1), dim3(HH_WG), 0, s, kind, pl.host[0]);
        return;
    }
    const Ctx c = ctx_of(pl, pl.chunks);
    LAUNCH(k_fin, n, s, c, pl.count == 1 ? nullptr : probs, kind);
}

template <int DIM, typename SP>
static void bicg_iter_t(const Plan &pl, hipStream_t s)
{
    const Ctx c = ctx_of(pl, pl.chunks);
    const int n = pl.chunks.n;
    LAUNCH_K(k_bicg_p, n, s, c);
    launch_vcycle(pl, VS_P, VS_PH, nullptr, nullptr, s);
    LAUNCH_K((k_bicg_v<DIM, SP>), n, s, c);
    launch_fin(pl, pl.fin, pl.nfin, FIN_ALPHA, s);
    LAUNCH_K(k_bicg_s, n, s, c);
    // the half-step check on ||s|| runs in the omega finaliser
    launch_vcycle(pl, VS_R, VS_SH, nullptr, nullptr, s);
    LAUNCH_K((k_bicg_t<DIM, SP>), n, s, c);
    launch_fin(pl, pl.fin, pl.nfin, FIN_OMEGA, s);
    LAUNCH_K((k_bicg_xr<SP>), n, s, c);
    launch_fin(pl, pl.fin, pl.nfin, FIN_RHO, s);
}

void launch_bicg_iteration(const Plan &pl, hipStream_t s)
{
    if (pl.dim == 2) {
        if (pl.fp32) bicg_iter_t<2, float2>(pl, s);
        else bicg_iter_t<2, double2>(pl, s);
    } else {
        if (pl.fp32) bicg_iter_t<3, float2>(pl, s);
        else bicg_iter_t<3, double2>(pl, s);
    }
}

template <int DIM, typename SW>
static void idr_step_t(const Plan &pl, hipStream_t s)
{
    const Ctx c = ctx_of(pl, pl.chunks);
    const int n = pl.chunks.n;
    LAUNCH_K(k_idr_v, n, s, c);
    launch_vcycle(pl, VS_V, VS_W, nullptr, nullptr, s);
    LAUNCH_K((k_idr_t<DIM, SW>), n, s, c);
    launch_fin(pl, pl.fin, pl.nfin, FIN_IDR_OMEGA, s);
    LAUNCH_K((k_idr_up<DIM, SW>), n, s, c);
    launch_fin(pl, pl.fin, pl.nfin, FIN_IDR_STEP, s);
}

void launch_idr_step(const Plan &pl, hipStream_t s)
{
    if (pl.dim == 2) {
        if (pl.fp32) idr_step_t<2, float2>(pl, s);
        else idr_step_t<2, double2>(pl, s);
    } else {
        if (pl.fp32) idr_step_t<3, float2>(pl, s);
        else idr_step_t<3, double2>(pl, s);
    }
}

void launch_resid(const Plan &pl, const DevList &tiles, int mode, hipStream_t s)
{
    const Ctx c = ctx_of(pl, tiles);
    if (pl.dim == 2) LAUNCH_K(k_resid<2>, tiles.n, s, c, mode);
    else LAUNCH_K(k_resid<3>, tiles.n, s, c, mode);
}

void launch_norm(const Plan &pl, const DevList &tiles, int sel, hipStream_t s)
{
    LAUNCH_K(k_norm, tiles.n, s, ctx_of(pl, tiles), sel);
}

void launch_zero(const Plan &pl, const DevList &tiles, int sel, hipStream_t s)
{
    LAUNCH_K(k_zero, tiles.n, s, ctx_of(pl, tiles), sel);
}

// A grid from a finished host setup: copies the description (not phi) and
// uploads the hierarchy unless the description asks for a host-only grid.
hh_status grid_create(HostSetup &&hs, const hh_grid_desc *d, hh_grid **out)
{
    *out = nullptr;
    hh_grid *g = new hh_grid();
    g->hs = std::move(hs);
    g->desc = *d;
    g->desc.phi = nullptr;
    g->host_only = d->host_only != 0;
    if (!g->host_only) {
        hh_status st = grid_upload(g);
        if (st != HH_OK) {
            grid_release(g);
            return st;
        }
    }
    *out = g;
    return HH_OK;
}

// Upper bound of the device bytes one problem needs inside a batch: the grid
// (the arrays grid_upload carves, with the tail images bounded by the LDS
// capacity), the solve work space, b and x, the IDR shadow space, and its
// entries in a plan's tile lists and subset lists.
hh_status footprint_bytes(const hh_grid_desc *d, const hh_solve_opts *o, uint64_t &bytes, std::string &err)
{
    int nl = 0, nc = 0;
    hh_status st = desc_check(d, nl, nc, err);
    if (st != HH_OK) return st;
    if (d->centering != HH_CELL) {
        err = "a vertex-centred grid cannot be solved (operator apply only)";
        return HH_ERR_ARG;
    }
    if (!o) {
        err = "null options";
        return HH_ERR_ARG;
    }
    const int dim = d->dim;
    HostLevel L[HH_MAXLEV];
    for (int l = 0; l < nl; ++l) {
        L[l].N = 1;
        for (int a = 0; a < 3; ++a) {
            L[l].n[a] = a < dim ? d->n[a] >> l : 1;
            L[l].N *= L[l].n[a];
        }
    }
    const int64_t N = L[0].N;
    const bool fp32 = o->vcycle_prec == HH_C64;
    const int s = o->method == HH_METHOD_IDR ? o->s : 0;
    size_t g = 0;
    for (int a = 0; a < dim; ++a) g += 3 * align256(sizeof(double2) * L[0].n[a]);
    for (int l = 0; l < nl; ++l) {
        for (int a = 0; a < dim; ++a) g += 3 * align256(sizeof(double2) * L[l].n[a]) + 3 * align256(sizeof(float2) * L[l].n[a]);
        g += align256(sizeof(double) * L[l].N) + align256(sizeof(float) * L[l].N);
        if (l >= 1) g += 2 * align256(sizeof(double2) * L[l].N) + 2 * align256(sizeof(float2) * L[l].N);
        if (l >= 1 && d->coarse_op == HH_COARSE_GALERKIN)
            g += align256(sizeof(double2) * 25 * L[l].N) + align256(sizeof(float2) * 25 * L[l].N);
        if (l + 1 < nl && d->smoother == HH_SMOOTH_ILU0)
            g += align256(sizeof(double2) * 25 * L[l].N) + align256(sizeof(double2) * L[l].N);
    }
    g += align256(sizeof(double2) * (size_t)nc * nc) + align256(sizeof(float2) * (size_t)nc * nc);
    g += align256(TailCap<double>::BYTES) + align256(TailCap<float>::BYTES);
    g += 4 * align256(sizeof(LevelDev<double>) * HH_MAXLEV) + align256(sizeof(ProbDev));
    const int nch = ceil_div(N, HH_CHUNK), ngr = ceil_div(N, HH_SPAN);
    g += align256(sizeof(Tile) * nch);
    // a mixed-precision solve may continue with the FP64 V-cycle (larger work
    // space), so the FP64 work space is reserved either way
    size_t ws = solve_workspace_bytes(N, o->method, false, s, 0);
    size_t io = 2 * align256(sizeof(double2) * N) + (s > 0 ? align256(sizeof(double2) * (size_t)N * s) : 0);
    const bool split = nc > HH_SPLIT_NC || d->coarse_op == HH_COARSE_GALERKIN || d->smoother == HH_SMOOTH_ILU0;
    size_t tiles = ngr + (split ? ceil_div(coarse_waves<double>(nc), HH_WG / 64) : 0);
    for (int l = 0; l + 1 < nl; ++l) {
        int md = 0, mu = 0;
        for (int v = 0; v < HH_NTILE; ++v) {
            int nd, nu;
            vtile_counts(dim, v, L[l], L[l + 1], nd, nu);
            md = std::max(md, nd);
            mu = std::max(mu, nu);
        }
        tiles += md + mu;
    }
    size_t plan = sizeof(Tile) * (tiles + ngr) + sizeof(ProbDev) + sizeof(Ctrl) + 2 * sizeof(int) +
                  256 * (2 * HH_MAXLEV + 8);
    bytes = g + ws + io + plan;
    return HH_OK;
}

// ---------------------------------------------------------------------------
// C ABI: grids, apply, V-cycle
// ---------------------------------------------------------------------------
extern "C" {

const char *hh_last_error(void) { return g_err.c_str(); }
const char *hh_version(void) { return "hh 0.1 gfx950"; }

hh_status hh_setup_grid(const hh_grid_desc *d, hh_grid **out)
{
    if (!out) return hh_fail(HH_ERR_ARG, "out is null");
    *out = nullptr;
    HostSetup hs;
    std::string err;
    hh_status st = host_setup(d, hs, err);
    if (st != HH_OK) return hh_fail(st, "%s", err.c_str());
    return grid_create(std::move(hs), d, out);
}

hh_status hh_free_grid(hh_grid *g)
{
    if (!g) return HH_OK;
    grid_release(g);
    return HH_OK;
}

hh_status hh_grid_query(const hh_grid *g, hh_grid_info *info)
{
    if (!g || !info) return hh_fail(HH_ERR_ARG, "null argument");
    memset(info, 0, sizeof *info);
    info->dim = g->hs.dim;
    info->levels = g->hs.nlev;
    for (int l = 0; l < g->hs.nlev; ++l)
        for (int a = 0; a < 3; ++a) info->n[l][a] = g->hs.lev[l].n[a];
    info->unknowns = g->hs.lev[0].N;
    info->coarse_unknowns = g->hs.Nc;
    info->device_bytes = g->dbytes + g->ws.bytes + g->plan_bytes();
    return HH_OK;
}

hh_status hh_grid_export(const hh_grid *g, int32_t what, int32_t level, int32_t axis, void *host_dst, size_t bytes)
{
    if (!g || !host_dst) return hh_fail(HH_ERR_ARG, "null argument");
    const HostSetup &hs = g->hs;
    if (level < 0 || level >= hs.nlev) return hh_fail(HH_ERR_ARG, "level %d out of range", level);
    const void *src = nullptr;
    size_t need = 0;
    if (what >= 0 && what <= 5) {
        if (axis < 0 || axis >= hs.dim) return hh_fail(HH_ERR_ARG, "axis %d out of range", axis);
        if (what <= 2 && level != 0) return hh_fail(HH_ERR_ARG, "H coefficients exist on level 0 only");
        const std::vector<double2> *v = what == 0 ? &hs.aH[axis] : what == 1 ? &hs.cH[axis] : what == 2 ? &hs.dH[axis]
                                      : what == 3 ? &hs.lev[level].aM[axis] : what == 4 ? &hs.lev[level].cM[axis]
                                                  : &hs.lev[level].dM[axis];
        src = v->data();
        need = sizeof(double2) * v->size();
    } else if (what == 6) {
        src = hs.lev[level].phi.data();
        need = sizeof(double) * hs.lev[level].phi.size();
    } else if (what == 7) {
        src = hs.Minv.data();
        need = sizeof(double2) * hs.Minv.size();
    } else if (what == 8) {
        if (hs.lev[level].gal.empty()) return hh_fail(HH_ERR_ARG, "level %d has no Galerkin stencil", level);
        src = hs.lev[level].gal.data();
        need = sizeof(double2) * hs.lev[level].gal.size();
    } else if (what == 9) {
        if (hs.lev[level].ilu.empty()) return hh_fail(HH_ERR_ARG, "level %d has no ILU(0) factors", level);
        src = hs.lev[level].ilu.data();
        need = sizeof(double2) * hs.lev[level].ilu.size();
    } else {
        return hh_fail(HH_ERR_ARG, "unknown export %d", what);
    }
    if (bytes != need) return hh_fail(HH_ERR_ARG, "export needs %zu bytes, got %zu", need, bytes);
    memcpy(host_dst, src, need);
    return HH_OK;
}

hh_status hh_apply_operator(const hh_grid *g, hh_op op, hh_prec prec, const void *x, void *y, void *stream)
{
    if (!g || !x || !y) return hh_fail(HH_ERR_ARG, "null argument");
    if (g->host_only) return hh_fail(HH_ERR_ARG, "grid was built host-only");
    if (x == y) return hh_fail(HH_ERR_ARG, "x and y must not overlap");
    hipStream_t s = (hipStream_t)stream;
    const int n = g->nchunks;
    Ctx c;
    c.P = g->pd_static_dev;
    c.tiles = nullptr;
    c.ctrl = nullptr;
    c.L = prec == HH_C64 ? (const void *)g->L32 : (const void *)g->L64;
    c.omega = g->hs.omega;
    c.nu1 = g->hs.nu1;
    if (op == HH_OP_H) {
        if (prec != HH_C128) return hh_fail(HH_ERR_ARG, "H is applied in complex double only");
        const int nx = g->hs.lev[0].n[0], ny = g->hs.lev[0].n[1];
        if (g->hs.dim == 2 && nx % 256 == 0) LAUNCH(k_applyH_band, (nx / 256) * ((ny + 1) / 2), s, hview(&g->pd_static), x, y);
        else if (g->hs.dim == 2) LAUNCH(k_applyH<2>, n, s, c, x, y);
        else LAUNCH(k_applyH<3>, n, s, c, x, y);
    } else if (op == HH_OP_M) {
        if (prec == HH_C128) {
            if (g->hs.dim == 2) LAUNCH((k_applyM<2, double>), n, s, c, x, y);
            else LAUNCH((k_applyM<3, double>), n, s, c, x, y);
        } else if (prec == HH_C64) {
            if (g->hs.dim == 2) LAUNCH((k_applyM<2, float>), n, s, c, x, y);
            else LAUNCH((k_applyM<3, float>), n, s, c, x, y);
        } else {
            return hh_fail(HH_ERR_ARG, "unknown precision %d", (int)prec);
        }
    } else {
        return hh_fail(HH_ERR_ARG, "unknown operator %d", (int)op);
    }
    HIPCHK(hipGetLastError());
    return HH_OK;
}

hh_status hh_vcycle(const hh_grid *g, hh_prec prec, const void *f, void *u, void *stream)
{
    if (!g || !f || !u) return hh_fail(HH_ERR_ARG, "null argument");
    if (g->host_only) return hh_fail(HH_ERR_ARG, "grid was built host-only");
    if (f == u) return hh_fail(HH_ERR_ARG, "f and u must not overlap");
    if (prec != HH_C128 && prec != HH_C64) return hh_fail(HH_ERR_ARG, "unknown precision %d", (int)prec);
    if (g->hs.centering != HH_CELL) return hh_fail(HH_ERR_ARG, "a vertex-centred grid has no multigrid hierarchy");
    if (g->hs.smoother == HH_SMOOTH_ILU0 && prec == HH_C64)
        return hh_fail(HH_ERR_ARG, "ILU(0) smoothing runs in the FP64 V-cycle only (HH_C128)");
    hh_grid *gm = const_cast<hh_grid *>(g);
    hh_status st = grid_vplan(gm, prec == HH_C64);
    if (st != HH_OK) return st;
    const Plan &pl = prec == HH_C64 ? gm->vplan32 : gm->vplan64;
    launch_vcycle(pl, VS_IN, VS_OUT, f, u, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return HH_OK;
}

// The V-cycle of hh_vcycle with the coarse-level f and e in the device's
// static scratch array: no device allocation, no stream or event creation, no
// tile timing; the launches go to `stream` only.
hh_status hh_vcycle_noalloc(const hh_grid *g, hh_prec prec, const void *f, void *u, void *stream)
{
    if (!g || !f || !u) return hh_fail(HH_ERR_ARG, "null argument");
    if (g->host_only) return hh_fail(HH_ERR_ARG, "grid was built host-only");
    if (f == u) return hh_fail(HH_ERR_ARG, "f and u must not overlap");
    if (prec != HH_C128 && prec != HH_C64) return hh_fail(HH_ERR_ARG, "unknown precision %d", (int)prec);
    if (g->hs.centering != HH_CELL) return hh_fail(HH_ERR_ARG, "a vertex-centred grid has no multigrid hierarchy");
    if (!g->scratch_ok) return hh_fail(HH_ERR_HIP, "the scratch array of device %d was not found at grid setup", g->device);
    if (g->hs.smoother == HH_SMOOTH_ILU0 && prec == HH_C64)
        return hh_fail(HH_ERR_ARG, "ILU(0) smoothing runs in the FP64 V-cycle only (HH_C128)");
    const bool fp32 = prec == HH_C64;
    const size_t need = fp32 ? g->scratch_need32 : g->scratch_need64;
    if (need > HH_SCRATCH_BYTES)
        return hh_fail(HH_ERR_ARG,
                       "the coarse levels of this grid need %zu bytes of scratch in %s; the allocation-free V-cycle "
                       "has %zu (use hh_vcycle)", need, fp32 ? "complex float" : "complex double", HH_SCRATCH_BYTES);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != g->device)
        return hh_fail(HH_ERR_ARG, "current device %d is not the grid's device %d", dev, g->device);
    Plan pl;
    plan_host_one(pl, g, fp32, fp32 ? (const void *)g->L32s : (const void *)g->L64s, g->L64sh, g->L32sh);
    launch_vcycle(pl, VS_IN, VS_OUT, f, u, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return HH_OK;
}

// Times the grid's V-cycle and its finest level's fused legs with HIP events
// on `stream`: `reps` back-to-back cycles, then `reps` back-to-back launches of
// the finest down-leg and of the finest up-leg, each leg exactly as the cycle
// (and a solve's plan) launches it.
hh_status hh_profile_vcycle(const hh_grid *g, hh_prec prec, const void *f, void *u, int32_t reps,
                            hh_vcycle_profile *out, void *stream)
{
    if (!g || !f || !u || !out) return hh_fail(HH_ERR_ARG, "null argument");
    if (g->host_only) return hh_fail(HH_ERR_ARG, "grid was built host-only");
    if (f == u) return hh_fail(HH_ERR_ARG, "f and u must not overlap");
    if (prec != HH_C128 && prec != HH_C64) return hh_fail(HH_ERR_ARG, "unknown precision %d", (int)prec);
    if (g->hs.centering != HH_CELL) return hh_fail(HH_ERR_ARG, "a vertex-centred grid has no multigrid hierarchy");
    if (reps < 1) return hh_fail(HH_ERR_ARG, "reps must be at least 1");
    if (g->hs.smoother == HH_SMOOTH_ILU0)
        return hh_fail(HH_ERR_ARG, "the profile times the weighted-Jacobi legs; an ILU(0) grid has none");
    const bool fp32 = prec == HH_C64;
    hh_grid *gm = const_cast<hh_grid *>(g);
    hh_status st = grid_vplan(gm, fp32);
    if (st != HH_OK) return st;
    const Plan &pl = fp32 ? gm->vplan32 : gm->vplan64;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[6] = {};
    for (int i = 0; i < 6; ++i) {
        hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) {
            for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
            return hh_fail(HH_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    LvHost lh;
    lh.d = pl.lv64h;
    lh.f = pl.lv32h;
    const Ctx cd = ctx_of(pl, pl.down[0]), cu = ctx_of(pl, pl.up[0]);
    launch_vcycle(pl, VS_IN, VS_OUT, f, u, s);   // warm-up; leaves every level's f and e valid
    hipError_t e = hipEventRecord(ev[0], s);
    for (int r = 0; r < reps; ++r) launch_vcycle(pl, VS_IN, VS_OUT, f, u, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventRecord(ev[2], s);
    for (int r = 0; r < reps; ++r)
        launch_leg_any(g->hs.dim, fp32, 0, pl.vdv[0], pl.down[0].n, s, cd, 0, VS_IN, VS_OUT, f, u, lh);
    if (e == hipSuccess) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) e = hipEventRecord(ev[4], s);
    for (int r = 0; r < reps; ++r)
        launch_leg_any(g->hs.dim, fp32, 1, pl.vuv[0], pl.up[0].n, s, cu, 0, VS_IN, VS_OUT, f, u, lh);
    if (e == hipSuccess) e = hipEventRecord(ev[5], s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
    float ms[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms[i], ev[2 * i], ev[2 * i + 1]);
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return hh_fail(HH_ERR_HIP, "V-cycle profile: %s", hipGetErrorString(e));
    out->vcycle_us = 1e3 * ms[0] / reps;
    out->down_us = 1e3 * ms[1] / reps;
    out->up_us = 1e3 * ms[2] / reps;
    out->down_shape = pl.vdv[0];
    out->up_shape = pl.vuv[0];
    out->down_groups = pl.down[0].n;
    out->up_groups = pl.up[0].n;
    return HH_OK;
}

} // extern "C"

hh_status grid_vplan(hh_grid *g, bool fp32)
{
    Plan &pl = fp32 ? g->vplan32 : g->vplan64;
    if (pl.mem) return HH_OK;
    std::vector<const hh_grid *> G{g};
    hh_status st = plan_build(pl, G, fp32);
    if (st != HH_OK) return st;
    // standalone cycles: the static descriptor, no control block (always run)
    pl.probs = g->pd_static_dev;
    pl.ctrl = nullptr;
    pl.host.assign(1, g->pd_static);
    return HH_OK;
}
