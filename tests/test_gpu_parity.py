"""GPU parity of the HIP path against the CPU FP64 oracle, through the C ABI.

FP64 paths follow the same fixed operation order as the oracle, so operator
applies, V-cycles and whole Bi-CGSTAB solves are compared value for value
(iteration counts equal).  Mixed precision (complex-FP32 V-cycle) is judged by
the FP64 true residual and the solution error against the oracle.
Tolerance of the method (fixed by the target): relative solution error
<= 1e-6 at an FP64 relative residual of 1e-8, iteration counts within +-1.
"""
import math

import numpy as np
import pytest

from paper_0912_0180_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP32 V-cycle against the oracle's FP64 cycle, relative error in norm.  FP32
# unit roundoff u = 2^-24 = 6.0e-8; the measured error of the rediscretised
# cycle is 1.1e-7 .. 1.4e-7 (about 2u) on every parity case, so the bound is
# 1e-6 (about 17u, 7x the largest measured).
FP32_VCYCLE_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def hh_mod(torch_dev):
    from paper_0912_0180_amd import hh
    hh.lib()
    return hh


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda") if dtype is None else t.to("cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def same(a, b):
    """value-for-value equality of complex arrays (+0 == -0)"""
    return np.array_equal(np.asarray(a), np.asarray(b))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# problem shapes: full configs' geometry at sizes the oracle finishes in
# seconds, spanning several tiles and ragged tails
def ragged_2d():
    d = W.base_desc(2, (96, 80), (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=3)
    rng = np.random.default_rng(21)
    phi = (30.0 ** 2) * (1 + 0.3 * rng.uniform(size=96 * 80))
    return {"desc": d, "phi": phi}


def ragged_3d():
    d = W.base_desc(3, (24, 16, 40), (-0.2, -0.25, -0.1), (1.2, 1.3, 1.15), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), levels=3)
    rng = np.random.default_rng(22)
    phi = (12.0 ** 2) * (1 + 0.3 * rng.uniform(size=24 * 16 * 40))
    return {"desc": d, "phi": phi}


CASES = {
    "c1": lambda: W.c1(),
    "c1_interior": lambda: W.c1(mode=1),
    "c2_256": lambda: W.c2(n=256, levels=6),
    "ragged_2d": ragged_2d,
    "ragged_3d": ragged_3d,
    "c3_32": lambda: W.c3(n=32, layer=4, method="bicgstab"),
    # coarsest grid 10 x 10 = 100 unknowns: the tail's two-segment coarse solve
    "c2_80": lambda: W.c2(n=80, levels=4),
}


def rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("name", list(CASES))
def test_operator_apply_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    x = rand_c(np.random.default_rng(1), g.N)
    xd = dev(torch, x)
    yH = host(g.apply(xd, "H"))
    yM = host(g.apply(xd, "M"))
    yM32 = host(g.apply(xd.to(torch.complex64), "M", prec="c64"))
    torch.cuda.synchronize()
    assert same(yH, o.apply(x, "H"))
    assert same(yM, o.apply(x, "M"))
    assert rel(yM32, o.apply(x.astype(np.complex64).astype(np.complex128), "M")) < 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    f = rand_c(np.random.default_rng(2), g.N)
    fd = dev(torch, f)
    u64 = host(g.vcycle(fd, "c128"))
    u32 = host(g.vcycle(fd, "c64"))
    torch.cuda.synchronize()
    ref = o.vcycle(f)
    assert same(u64, ref)
    err = rel(u32.astype(np.complex128), ref)
    assert err < FP32_VCYCLE_TOL, err


@pytest.mark.parametrize("name", ["c1", "c1_interior", "ragged_2d", "ragged_3d", "c3_32", "c2_80"])
def test_bicgstab_fp64_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c.get("b")
    if b is None:
        b = rand_c(np.random.default_rng(3), g.N)
    xo, io = o.solve(b, tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, b), tol=1e-8, vcycle_prec="c128", history=True)
    xg = host(xg)
    assert io["status"] == 0 and ig["status"] == 0
    assert abs(ig["matvecs"] - io["matvecs"]) <= 1
    assert ig["rel_res_true"] < 1e-8
    assert rel(xg, xo) <= 1e-6
    # the arithmetic contract makes the whole iteration reproduce the oracle
    assert ig["matvecs"] == io["matvecs"] and ig["iterations"] == io["iterations"]
    assert same(xg, xo)
    assert np.array_equal(ig["history"], io["history"])


@pytest.mark.parametrize("name", ["c1", "c2_256", "ragged_3d", "c3_32", "c2_80"])
def test_bicgstab_mixed_precision(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c.get("b")
    if b is None:
        b = rand_c(np.random.default_rng(4), g.N)
    xo, io = o.solve(b, tol=1e-8)
    xg, ig = g.solve(dev(torch, b), tol=1e-8, vcycle_prec="c64")
    xg = host(xg)
    assert ig["status"] == 0 and ig["rel_res_true"] < 1e-8
    assert ig["fp64_fallback"] == 0          # the FP32 V-cycle carried the whole solve
    assert rel(xg, xo) <= 1e-6
    print(name, "matvecs fp64", io["matvecs"], "mixed", ig["matvecs"], "err", rel(xg, xo))


def test_mixed_drift_falls_back_to_fp64(torch_dev, hh_mod, monkeypatch):
    """The drift guard (forced here by a 3-matvec stall limit) stops a mixed
    solve and the solve finishes from its iterate with the FP64 V-cycle: it
    reaches the tolerance and the FP64 solution, and batched problems give
    what they give alone."""
    torch = torch_dev
    cs = [W.c2(n=256, levels=6), ragged_2d()]
    rng = np.random.default_rng(12)
    grids, bs, x64s = [], [], []
    for c in cs:
        g = hh_mod.Grid(c["desc"], c["phi"])
        b = c.get("b")
        b = dev(torch, b if b is not None else rand_c(rng, g.N))
        x64, i64 = g.solve(b, tol=1e-8, vcycle_prec="c128")
        assert i64["status"] == 0 and i64["fp64_fallback"] == 0
        grids.append(g)
        bs.append(b)
        x64s.append(host(x64))
    monkeypatch.setenv("HH_DRIFT_STALL", "3")
    monkeypatch.setenv("HH_MIXED_STAGE", "0")   # the guard alone, without stage restarts
    alone = []
    for g, b, x64 in zip(grids, bs, x64s):
        xm, im = g.solve(b, tol=1e-8, vcycle_prec="c64", history=True)
        assert im["status"] == 0 and im["fp64_fallback"] == 1, im
        assert im["rel_res_true"] < 1e-8
        assert rel(host(xm), x64) <= 1e-6
        h = im["history"]
        assert len(h) == im["matvecs"] and np.all(np.isfinite(h)) and h[-1] < 1e-8
        alone.append((host(xm), im))
    xs, infos = hh_mod.solve_batch(grids, bs, tol=1e-8, vcycle_prec="c64")
    for (xa, ia), x, i in zip(alone, xs, infos):
        assert i["fp64_fallback"] == 1 and i["matvecs"] == ia["matvecs"]
        assert same(host(x), xa)


def test_underresolved_mixed_solve_is_correct(torch_dev, hh_mod):
    """An under-resolved problem (5.4 points per wavelength, 512^2) sits near
    the FP32 V-cycle's accuracy floor; with or without the FP64 fallback the
    mixed solve must reach the tolerance and the FP64 solution."""
    torch = torch_dev
    p = W.c4(64)[27]
    assert p["desc"]["n"][:2] == [512, 512] and p["ppw"] < 5.5
    g = hh_mod.Grid(p["desc"], p["phi"])
    b = dev(torch, p["b"])
    x64, i64 = g.solve(b, tol=1e-8, vcycle_prec="c128")
    xm, im = g.solve(b, tol=1e-8, vcycle_prec="c64")
    print("5.4 ppw 512^2: fp64 matvecs", i64["matvecs"], "mixed", im["matvecs"], "fallback", im["fp64_fallback"])
    assert i64["status"] == 0 and im["status"] == 0 and im["rel_res_true"] < 1e-8
    assert rel(host(xm), host(x64)) <= 1e-6


def big_2d(n, ppw, seed):
    g = W.rng(seed)
    d = W.base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0))
    h = 1.5 / n
    k0 = 2 * math.pi / (ppw * h)
    phi = W.bump_k(d, k0, g.uniform(0.15, 0.85, size=(8, 2)))
    b = W.gaussian_sources(d, g.uniform(0.1, 0.9, size=(3, 2)))
    return {"desc": d, "phi": phi, "b": b}


@pytest.mark.parametrize("n,ppw,seed", [(1280, 10.0, 7), (1536, 10.0, 7)])
def test_staged_mixed_solve_needs_no_fp64_fallback(torch_dev, hh_mod, monkeypatch, n, ppw, seed):
    """2D grids of 1216^2 and more at 10 points per wavelength used to drift
    in mixed precision and fall back to the FP64 V-cycle.  Run in stages, each
    restarting from the FP64 true residual after a tenfold reduction, the mixed
    Bi-CGSTAB solve reaches 1e-8 without the fallback and agrees with the FP64
    solve; with stages off it is the old unstaged iteration."""
    torch = torch_dev
    c = big_2d(n, ppw, seed)
    print("case staged mixed", n, ppw, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    b = dev(torch, c["b"])
    x64, i64 = g.solve(b, tol=1e-8, vcycle_prec="c128")
    xm, im = g.solve(b, tol=1e-8, vcycle_prec="c64")
    assert i64["status"] == 0 and i64["stages"] == 0
    assert im["status"] == 0 and im["fp64_fallback"] == 0 and im["stages"] > 1 and im["rel_res_true"] < 1e-8
    assert rel(host(xm), host(x64)) <= 1e-6
    monkeypatch.setenv("HH_MIXED_STAGE", "0")
    xu, iu = g.solve(b, tol=1e-8, vcycle_prec="c64")
    assert iu["stages"] == 0 and iu["status"] == 0 and iu["rel_res_true"] < 1e-8
    print(n, "matvecs fp64", i64["matvecs"], "staged mixed", im["matvecs"], "stages", im["stages"],
          "unstaged mixed", iu["matvecs"], "fallback", iu["fp64_fallback"], flush=True)


def test_batch_equals_single(torch_dev, hh_mod):
    """Problems solved together give exactly the results they give alone."""
    torch = torch_dev
    cs = [W.c1(), W.c2(n=256, levels=6), ragged_2d(), W.c1(mode=1)]
    rng = np.random.default_rng(5)
    grids, bs = [], []
    for c in cs:
        g = hh_mod.Grid(c["desc"], c["phi"])
        grids.append(g)
        b = c.get("b")
        bs.append(dev(torch, b if b is not None else rand_c(rng, g.N)))
    single = [g.solve(b, tol=1e-8) for g, b in zip(grids, bs)]
    for prec in ("c128", "c64"):
        xs, infos = hh_mod.solve_batch(grids, bs, tol=1e-8, vcycle_prec=prec)
        for q in range(len(cs)):
            xq, iq = grids[q].solve(bs[q], tol=1e-8, vcycle_prec=prec)
            assert infos[q]["status"] == 0
            assert infos[q]["matvecs"] == iq["matvecs"]
            assert same(host(xs[q]), host(xq))
    for q in range(len(cs)):
        assert single[q][1]["status"] == 0


def test_solve_is_deterministic(torch_dev, hh_mod):
    torch = torch_dev
    c = W.c2(n=256, levels=6)
    g = hh_mod.Grid(c["desc"], c["phi"])
    b = dev(torch, c["b"])
    ref, ir = g.solve(b, tol=1e-8, vcycle_prec="c64")
    ref = host(ref)
    for _ in range(3):
        x, i = g.solve(b, tol=1e-8, vcycle_prec="c64")
        assert i["matvecs"] == ir["matvecs"] and same(host(x), ref)


def test_edge_cases(torch_dev, hh_mod, oracle_mod):
    torch = torch_dev
    c = W.c1()
    g = hh_mod.Grid(c["desc"], c["phi"])
    z = torch.zeros(g.N, dtype=torch.complex128, device="cuda")
    x, info = g.solve(z)
    assert info["status"] == 0 and info["matvecs"] == 0 and torch.count_nonzero(x).item() == 0
    b = dev(torch, c["b"])
    x, info = g.solve(b, max_matvec=1, max_restarts=0)
    xo, io = oracle_mod.Grid(c["desc"], c["phi"]).solve(c["b"], max_matvec=1, max_restarts=0)
    assert info["status"] == -4 == io["status"] and info["matvecs"] == 1
    assert same(host(x), xo)
    bad = c["b"].copy()
    bad[5] = np.nan
    x, info = g.solve(dev(torch, bad))
    assert info["status"] == -6
    # warm start (resume from a saved iterate) follows the oracle exactly
    x0, i0 = g.solve(b, tol=1e-8, max_matvec=40, max_restarts=0)
    assert i0["status"] == -4
    x1, i1 = g.solve(b, x=x0.clone(), x0_given=True, tol=1e-8)
    xo1, io1 = oracle_mod.Grid(c["desc"], c["phi"]).solve(c["b"], x0=host(x0), tol=1e-8)
    assert i1["status"] == 0 == io1["status"] and i1["matvecs"] == io1["matvecs"]
    assert same(host(x1), xo1)


@pytest.mark.parametrize("name,s", [("c1", 4), ("ragged_2d", 4), ("ragged_3d", 4), ("c3_32", 4), ("c1_interior", 1),
                                    ("c1", 2), ("c1", 8)])
def test_idr_fp64_matches_oracle(torch_dev, hh_mod, oracle_mod, name, s):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, "s", s, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c.get("b")
    if b is None:
        b = rand_c(np.random.default_rng(13), g.N)
    P = W.shadow_space(g.N, s, 1000 + s)
    xo, io = o.solve(b, method="idr", s=s, P=P, tol=1e-8, history=True)
    Pd = hh_mod.shadow_to_device(P)
    xg, ig = g.solve(dev(torch, b), method="idr", s=s, P=Pd, tol=1e-8, vcycle_prec="c128", history=True)
    xg = host(xg)
    assert io["status"] == 0 and ig["status"] == 0
    assert ig["rel_res_true"] < 1e-8 and rel(xg, xo) <= 1e-6
    assert ig["matvecs"] == io["matvecs"] and ig["iterations"] == io["iterations"]
    assert same(xg, xo)
    assert np.array_equal(ig["history"], io["history"])


def small_problem(n=(16, 16), k=20.0):
    d = W.base_desc(2, n, (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0), levels=2)
    N = int(np.prod(n))
    rng = np.random.default_rng(7)
    phi = k * k * (1 + 0.2 * rng.uniform(size=N))
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return d, phi, b


@pytest.mark.parametrize("s", [1, 4])
def test_idr_breakdown_and_restarts_match_oracle(torch_dev, hh_mod, oracle_mod, s):
    """A zero shadow space gives a zero G at the end of each start-up: a
    breakdown, a restart from the true residual, and after max_restarts the
    breakdown status.  Status, restarts, counts, history and iterate equal
    the oracle's."""
    torch = torch_dev
    d, phi, b = small_problem()
    print("case idr P=0 s", s, flush=True)
    g = hh_mod.Grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    P = np.zeros((g.N, s), complex)
    xo, io = o.solve(b, method="idr", s=s, P=P, max_restarts=2, history=True)
    xg, ig = g.solve(dev(torch, b), method="idr", s=s, P=hh_mod.shadow_to_device(P), max_restarts=2,
                     vcycle_prec="c128", history=True)
    assert io["status"] == -5 == ig["status"]
    assert ig["restarts"] == io["restarts"] == 2 and ig["matvecs"] == io["matvecs"] == 3 * s
    assert np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo) and ig["rel_res_true"] == io["rel_res_true"]


@pytest.mark.parametrize("method,n,tol,restarts", [("bicgstab", (32, 32), 1e-15, 1), ("bicgstab", (16, 16), 2e-15, 2),
                                                   ("idr", (32, 32), 1e-15, 1), ("idr", (24, 16), 1e-15, 2),
                                                   ("bicgstab", (16, 16), 1e-15, 3)])
def test_restart_from_true_residual_matches_oracle(torch_dev, hh_mod, oracle_mod, method, n, tol, restarts):
    """Tolerances near FP64 rounding force restarts from the true residual
    (then convergence, or the restarts run out: not converged); the GPU
    reproduces the oracle's status, restarts, matvecs, history and iterate."""
    torch = torch_dev
    d, phi, b = small_problem(n=n)
    print("case restart", method, n, tol, flush=True)
    g = hh_mod.Grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    P = W.shadow_space(g.N, 4, 11)
    xo, io = o.solve(b, method=method, tol=tol, s=4, P=P, max_restarts=3, history=True)
    xg, ig = g.solve(dev(torch, b), method=method, tol=tol, s=4, P=hh_mod.shadow_to_device(P), max_restarts=3,
                     vcycle_prec="c128", history=True)
    assert io["restarts"] == restarts == ig["restarts"]
    assert ig["status"] == io["status"] and ig["matvecs"] == io["matvecs"]
    assert ig["iterations"] == io["iterations"]
    assert np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)


@pytest.mark.parametrize("name", ["c1", "ragged_3d", "c3_32"])
def test_idr_mixed_precision(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c.get("b")
    if b is None:
        b = rand_c(np.random.default_rng(14), g.N)
    P = W.shadow_space(g.N, 4, 1004)
    xo, io = o.solve(b, method="idr", s=4, P=P, tol=1e-8)
    xg, ig = g.solve(dev(torch, b), method="idr", s=4, P=hh_mod.shadow_to_device(P), tol=1e-8, vcycle_prec="c64")
    assert ig["status"] == 0 and ig["rel_res_true"] < 1e-8
    assert rel(host(xg), xo) <= 1e-6
    print(name, "IDR(4) matvecs fp64", io["matvecs"], "mixed", ig["matvecs"])


def test_idr_batch_equals_single(torch_dev, hh_mod):
    torch = torch_dev
    cs = [W.c1(), ragged_2d(), W.c2(n=256, levels=6)]
    rng = np.random.default_rng(15)
    grids, bs, Ps = [], [], []
    for c in cs:
        g = hh_mod.Grid(c["desc"], c["phi"])
        grids.append(g)
        b = c.get("b")
        bs.append(dev(torch, b if b is not None else rand_c(rng, g.N)))
    # one shared options set: all problems use s = 4 with their own P
    xs_single = []
    for g, b in zip(grids, bs):
        P = hh_mod.shadow_to_device(W.shadow_space(g.N, 4, 77))
        Ps.append(P)
        x, i = g.solve(b, method="idr", s=4, P=P, tol=1e-8, vcycle_prec="c64")
        assert i["status"] == 0
        xs_single.append((host(x), i["matvecs"]))
    L = hh_mod.lib()
    import ctypes
    n = len(grids)
    opts = (hh_mod.SolveOpts * n)()
    for q in range(n):
        o, _ = hh_mod.make_opts(method="idr", s=4, P=Ps[q], tol=1e-8, vcycle_prec="c64")
        opts[q] = o
    infos = (hh_mod.SolveInfo * n)()
    xs = [torch.zeros_like(b) for b in bs]
    G = (ctypes.c_void_p * n)(*[g.h.value for g in grids])
    B = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
    X = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    st = L.hh_solve_batch(G, n, opts, B, X, infos, None)
    torch.cuda.synchronize()
    assert st == 0
    for q in range(n):
        assert infos[q].matvecs == xs_single[q][1]
        assert same(host(xs[q]), xs_single[q][0])


def test_graph_replay_equals_eager(torch_dev, hh_mod, monkeypatch):
    """Iterations replayed from a captured graph (K per check) give exactly the
    eager-launch results, over several solves in a row, for both methods."""
    torch = torch_dev
    c = W.c2(n=256, levels=6)
    g = hh_mod.Grid(c["desc"], c["phi"])
    b = dev(torch, c["b"])
    P = hh_mod.shadow_to_device(W.shadow_space(g.N, 4, 5))
    runs = {}
    for mode in ("eager", "graph4", "graph1", "graph7"):
        monkeypatch.delenv("HH_NO_GRAPH", raising=False)
        if mode == "eager":
            monkeypatch.setenv("HH_NO_GRAPH", "1")
            monkeypatch.setenv("HH_ITERS_PER_CHECK", "1")
        else:
            monkeypatch.setenv("HH_ITERS_PER_CHECK", mode[5:])
        out = []
        for rep in range(2):
            x1, i1 = g.solve(b, tol=1e-8, vcycle_prec="c64")
            x2, i2 = g.solve(b, tol=1e-8, vcycle_prec="c128", method="idr", s=4, P=P)
            torch.cuda.synchronize()
            out.append((host(x1), i1["matvecs"], host(x2), i2["matvecs"]))
        runs[mode] = out
    ref = runs["eager"][0]
    for mode, out in runs.items():
        for r in out:
            assert r[1] == ref[1] and r[3] == ref[3], mode
            assert same(r[0], ref[0]) and same(r[2], ref[2]), mode


def test_long_partial_arrays_match_oracle(torch_dev, hh_mod, oracle_mod):
    """4096 x 2560 unknowns make 40960 reduction chunks (10240 groups of
    four), more than one finaliser block (8192 partials): the first FP64
    matvecs give the oracle's residual history and iterate value for value."""
    torch = torch_dev
    d = W.base_desc(2, (4096, 2560), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0), levels=9)
    h = 1.5 / 4096
    phi = W.bump_k(d, 2 * np.pi / (10 * h), W.rng(2).uniform(0.15, 0.85, size=(8, 2)))
    g = hh_mod.Grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    b = rand_c(np.random.default_rng(17), g.N)
    print("long partials: N", g.N, flush=True)
    xo, io = o.solve(b, tol=1e-14, max_matvec=4, history=True)
    xg, ig = g.solve(dev(torch, b), tol=1e-14, max_matvec=4, vcycle_prec="c128", history=True)
    assert ig["matvecs"] == io["matvecs"] == 4
    assert np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)
    assert ig["rel_res_true"] == io["rel_res_true"]


def test_full_size_2d_solve(torch_dev, hh_mod, oracle_mod):
    """The 1024^2 point-source problem, solved as bench.py times it.  The
    oracle takes too long for a whole solve here, so its first 24 FP64
    matvecs are compared: the residual history and the iterate agree value
    for value.  The whole FP64 and mixed solves must then reach a true
    residual below 1e-8, evaluated with the oracle's operator, and agree
    with each other to 1e-6."""
    torch = torch_dev
    c = W.c2()
    print("case c2 1024^2", flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c["b"]
    bd = dev(torch, b)
    xo, io = o.solve(b, tol=1e-8, max_matvec=24, history=True)
    xg, ig = g.solve(bd, tol=1e-8, max_matvec=24, vcycle_prec="c128", history=True)
    assert io["status"] == ig["status"] == -4
    assert ig["matvecs"] == io["matvecs"] == 24
    assert np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)
    nb = np.linalg.norm(b)
    x64, i64 = g.solve(bd, tol=1e-8, vcycle_prec="c128")
    x32, i32 = g.solve(bd, tol=1e-8, vcycle_prec="c64")
    x64, x32 = host(x64), host(x32)
    for x, info in ((x64, i64), (x32, i32)):
        assert info["status"] == 0
        assert np.linalg.norm(b - o.apply(x, "H")) / nb < 1e-8
    assert i32["fp64_fallback"] == 0
    assert rel(x32, x64) <= 1e-6
    print("c2 matvecs fp64", i64["matvecs"], "mixed", i32["matvecs"], "diff", rel(x32, x64), flush=True)


def test_full_size_3d_solve(torch_dev, hh_mod, oracle_mod):
    """The 128^3 problem with 16-cell layers (2.1 M unknowns, five levels),
    solved as bench.py times it.  The first 8 FP64 matvecs of Bi-CGSTAB and
    of IDR(4) give the oracle's residual history and iterate value for value.
    The whole mixed Bi-CGSTAB and IDR(4) solves must reach a true residual
    below 1e-8, evaluated with the oracle's operator, and agree with the
    whole FP64 Bi-CGSTAB solve to 1e-6."""
    torch = torch_dev
    c = W.c3(n=128, layer=16, method="idr", s=4)
    print("case c3 128^3", flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b, P = c["b"], c["P"]
    bd, Pd = dev(torch, b), hh_mod.shadow_to_device(P)
    for ko, kg in (({}, {}), ({"method": "idr", "s": 4, "P": P}, {"method": "idr", "s": 4, "P": Pd})):
        xo, io = o.solve(b, tol=1e-8, max_matvec=8, history=True, **ko)
        xg, ig = g.solve(bd, tol=1e-8, max_matvec=8, vcycle_prec="c128", history=True, **kg)
        assert io["status"] == ig["status"] == -4, ko
        assert ig["matvecs"] == io["matvecs"] == 8 and ig["iterations"] == io["iterations"], ko
        assert np.array_equal(ig["history"], io["history"]), ko
        assert same(host(xg), xo), ko
    nb = np.linalg.norm(b)
    x64, i64 = g.solve(bd, tol=1e-8, vcycle_prec="c128")
    x64 = host(x64)
    runs = {"bicgstab_fp64": (x64, i64)}
    x, i = g.solve(bd, tol=1e-8, vcycle_prec="c64")
    runs["bicgstab_mixed"] = (host(x), i)
    x, i = g.solve(bd, tol=1e-8, vcycle_prec="c64", method="idr", s=4, P=Pd)
    runs["idr4_mixed"] = (host(x), i)
    for name, (x, info) in runs.items():
        assert info["status"] == 0, name
        assert np.linalg.norm(b - o.apply(x, "H")) / nb < 1e-8, name
        assert rel(x, x64) <= 1e-6, name
        print(name, "matvecs", info["matvecs"], "diff to fp64", rel(x, x64), flush=True)


def test_full_size_batch(torch_dev, hh_mod, oracle_mod):
    """The 64-problem batch (sides 256 to 1024, 5 to 12 points per
    wavelength, 1 to 4 Gaussian sources), solved in mixed precision as
    bench.py times it.  Every problem must reach a true residual below 1e-8,
    evaluated with the oracle's operator.  Problems whose FP32 V-cycle
    drifted finish with the FP64 one and report it.  Problems taken from the
    batch must give alone exactly what they gave in it."""
    torch = torch_dev
    probs = W.c4(count=64)
    print("case c4: 64 problems", flush=True)
    grids = [hh_mod.Grid(c["desc"], c["phi"]) for c in probs]
    bs = [dev(torch, c["b"]) for c in probs]
    xs, infos = hh_mod.solve_batch(grids, bs, tol=1e-8, vcycle_prec="c64")
    fell = [q for q in range(len(probs)) if infos[q]["fp64_fallback"]]
    for q, c in enumerate(probs):
        assert infos[q]["status"] == 0, q
        o = oracle_mod.Grid(c["desc"], c["phi"])
        r = np.linalg.norm(c["b"] - o.apply(host(xs[q]), "H")) / np.linalg.norm(c["b"])
        assert r < 1e-8, (q, r)
        del o
    for q in [0, 1, 2] + fell[:1]:
        xq, iq = grids[q].solve(bs[q], tol=1e-8, vcycle_prec="c64")
        assert iq["matvecs"] == infos[q]["matvecs"] and iq["fp64_fallback"] == infos[q]["fp64_fallback"], q
        assert same(host(xq), host(xs[q])), q
    print("c4: fallbacks", fell, "matvecs max", max(i["matvecs"] for i in infos), flush=True)
    for g in grids:
        g.close()


# problems of 1 to 4 reduction chunks (256 unknowns each), ragged and exact:
# a Krylov workgroup of several chunks stops its group sum at the padded chunk
# count; 24 x 24 also takes the many-workgroup coarse solve (144 unknowns)
TINY = [(16, 12), (16, 16), (24, 16), (24, 24), (32, 28)]


@pytest.mark.parametrize("n", TINY)
def test_tiny_problems_match_oracle(torch_dev, hh_mod, oracle_mod, n):
    torch = torch_dev
    d = W.base_desc(2, n, (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=2)
    N = n[0] * n[1]
    phi = 25.0 * (1 + 0.3 * np.random.default_rng(N).uniform(size=N))
    g = hh_mod.Grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    b = rand_c(np.random.default_rng(N + 1), N)
    print("tiny", n, "chunks", -(-N // 256), flush=True)
    xo, io = o.solve(b, tol=1e-12, max_matvec=60, history=True)
    xg, ig = g.solve(dev(torch, b), tol=1e-12, max_matvec=60, vcycle_prec="c128", history=True)
    assert ig["status"] == io["status"] and ig["matvecs"] == io["matvecs"] > 0
    assert np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)
    assert ig["rel_res_true"] == io["rel_res_true"]
    if n == (24, 24):
        P = W.shadow_space(N, 2, 5)
        xo, io = o.solve(b, tol=1e-12, max_matvec=60, method="idr", s=2, P=P, history=True)
        xg, ig = g.solve(dev(torch, b), tol=1e-12, max_matvec=60, method="idr", s=2, P=hh_mod.shadow_to_device(P),
                         vcycle_prec="c128", history=True)
        assert ig["status"] == io["status"] and ig["matvecs"] == io["matvecs"] > 0
        assert np.array_equal(ig["history"], io["history"])
        assert same(host(xg), xo)


def ragged_merge():
    d = W.base_desc(2, (352, 224), (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=6)
    rng = np.random.default_rng(23)
    phi = (100.0 ** 2) * (1 + 0.3 * rng.uniform(size=352 * 224))
    return {"desc": d, "phi": phi}


# 2D problems whose last levels above the tail run as one merged down- and
# one merged up-leg launch: two levels (256^2), three (512^2), three with
# ragged tiles on every level (352 x 224), three above a 576-unknown coarsest
# grid solved by k_coarse between the tail's down- and up-legs (384^2), three
# down and four up (1024^2)
MERGE_CASES = {
    "c2_256": lambda: W.c2(n=256, levels=6),
    "c2_512": lambda: W.c2(n=512, levels=7),
    "ragged_merge": ragged_merge,
    "c2_384_split": lambda: W.c2(n=384, levels=5),
    "c2_1024": lambda: W.c2(),
}


@pytest.mark.parametrize("name", list(MERGE_CASES))
def test_merged_coarse_legs_match(torch_dev, hh_mod, oracle_mod, monkeypatch, name):
    """Merged coarse legs give the oracle's FP64 V-cycle value for value, and
    the same FP32 cycle as the level-by-level kernels (same arithmetic)."""
    torch = torch_dev
    c = MERGE_CASES[name]()
    print("case", name, flush=True)
    o = oracle_mod.Grid(c["desc"], c["phi"])
    f = rand_c(np.random.default_rng(9), o.N)
    ref = o.vcycle(f)
    fd = dev(torch, f)
    out = {}
    for merge in ("1", "0"):
        monkeypatch.setenv("HH_MERGE", merge)
        g = hh_mod.Grid(c["desc"], c["phi"])
        assert same(host(g.vcycle(fd, "c128")), ref), (name, merge)
        out[merge] = host(g.vcycle(fd, "c64"))
        g.close()
    assert same(out["1"], out["0"])
    assert rel(out["1"], ref) < FP32_VCYCLE_TOL, rel(out["1"], ref)


@pytest.mark.parametrize("name", ["c2_256", "ragged_2d", "ragged_3d", "c3_32"])
def test_every_tile_shape_gives_the_same_cycle(torch_dev, hh_mod, oracle_mod, monkeypatch, name):
    """The autotuner may pick any tile shape: every shape must give the FP64
    V-cycle of the oracle value for value, and one FP32 result for all."""
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    o = oracle_mod.Grid(c["desc"], c["phi"])
    f = rand_c(np.random.default_rng(8), o.N)
    ref = o.vcycle(f)
    fd = dev(torch, f)
    u32 = None
    # tile shapes: 7 box shapes; in 3D two more, the z-streaming kernels, in
    # 2D one more box of 1024 threads
    for v in range(9 if c["desc"]["dim"] == 3 else 8):
        monkeypatch.setenv("HH_TILE", str(v))
        g = hh_mod.Grid(c["desc"], c["phi"])
        assert same(host(g.vcycle(fd, "c128")), ref), (name, v)
        u = host(g.vcycle(fd, "c64"))
        if u32 is None:
            u32 = u
        assert same(u, u32), (name, v)
        g.close()


def test_streaming_legs_equal_plain_legs(torch_dev, hh_mod, oracle_mod, monkeypatch):
    """Finest 2D levels of at least 8M unknowns run the FP32 legs with
    non-temporal per-point accesses (interior tiles).  The arithmetic is the
    plain legs', so the cycle equals theirs bit for bit (HH_STREAM=0), and it
    stays within the FP32 bound of the oracle's FP64 cycle."""
    torch = torch_dev
    n = 2944
    c = W.c2(n=n, levels=8)
    assert n * n >= 8 << 20
    print("case c2_%d" % n, flush=True)
    f = rand_c(np.random.default_rng(10), n * n)
    fd = dev(torch, f)
    out = {}
    for st in ("1", "0"):
        monkeypatch.setenv("HH_STREAM", st)
        g = hh_mod.Grid(c["desc"], c["phi"])
        out[st] = host(g.vcycle(fd, "c64"))
        g.close()
    assert same(out["1"], out["0"])
    del fd
    o = oracle_mod.Grid(c["desc"], c["phi"])
    ref = o.vcycle(f)
    err = rel(out["1"], ref)
    print("FP32 cycle vs oracle", err, flush=True)
    assert err < FP32_VCYCLE_TOL, err


def test_c2_full_solve_against_oracle_fixture(torch_dev, hh_mod):
    """The whole headline solve at 1024^2 against the oracle's own
    (tests/golden/c2_1024_oracle_solve.json, written from the oracle alone by
    tests/golden/make_c2_oracle_fixture.py): the FP64 GPU solve reproduces its
    matvec and iteration counts, its whole residual history and its sampled
    solution entries value for value; the mixed solve reaches 1e-8 with the
    sampled entries within 1e-6 of the oracle's (relative)."""
    import json
    import os
    torch = torch_dev
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_1024_oracle_solve.json")
    fx = json.load(open(path))
    c = W.c2()
    g = hh_mod.Grid(c["desc"], c["phi"])
    b = dev(torch, c["b"])
    idx = np.array(fx["sample_index"])
    xo = np.array(fx["sample_re"]) + 1j * np.array(fx["sample_im"])
    print("case c2 fp64", flush=True)
    x64, i64 = g.solve(b, tol=1e-8, vcycle_prec="c128", history=True)
    assert i64["status"] == 0 and fx["status"] == 0
    assert i64["matvecs"] == fx["matvecs"] and i64["iterations"] == fx["iterations"]
    assert np.array_equal(i64["history"], np.array(fx["history"]))
    x64 = host(x64)
    assert same(x64[idx], xo)
    assert abs(np.linalg.norm(x64) - fx["x_norm"]) <= 1e-14 * fx["x_norm"]
    print("case c2 mixed", flush=True)
    xm, im = g.solve(b, tol=1e-8, vcycle_prec="c64")
    assert im["status"] == 0 and im["rel_res_true"] < 1e-8
    assert rel(host(xm)[idx], xo) <= 1e-6
