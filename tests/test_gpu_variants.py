"""GPU parity of the paper's other problem and preconditioner settings against
the CPU FP64 oracle, through the C ABI:

* model problems 2 and 3 (Sec. 4, eqs. (MP2), (MP3), (BC)): Dirichlet south
  and west, ECS layers north and east only, analytic wave numbers;
* the Sommerfeld variant of MP2 (eq. (sommerfeld1) on the north and east
  edges, a negative CSG angle as in the paper's Sommerfeld rows), and a 3D grid
  with one Sommerfeld face;
* the CSL preconditioner (Sec. 5.2, eq. (helmctucsl)) with a shift of
  modulus above one;
* a smooth ECS contour (Sec. 6.2, remark: the layer turns in equal angle
  steps).

The kernels are the same as for the headline problem (only the setup's
coefficients differ), so the FP64 operator, V-cycle and whole Bi-CGSTAB and
IDR(s) solves equal the oracle value for value, with identical counts and
histories; mixed precision is held to the method's tolerance (relative
solution error <= 1e-6 at a true residual below 1e-8).
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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def csl_c1():
    c = W.c1()
    c["desc"].update(csg_mode=2, csl_shift=[1.0, 0.35])
    return c


def smooth_c2():
    c = W.c2(n=128, levels=4)
    c["desc"].update(contour_steps=32)
    return c


def sommerfeld_3d():
    c = W.c3(n=32, layer=4, method="bicgstab")
    d = c["desc"]
    d["a"][2] = d["lo"][2]
    d["bc"][2] = [1, 0]
    d["k_bc"] = 12.0
    return c


# same resolution as the paper's grids (h = r / n_int), smaller domains
VARIANTS = {
    "mp2_nu7k2": lambda: W.mp2(n_int=96, n_lay=32, r=12.5),
    "mp2_nu1k4": lambda: W.mp2(nu=1.0, k=4.0, n_int=96, n_lay=32, r=12.5),
    "mp3_r90k2": lambda: W.mp3(n_int=96, n_lay=32, r=90.0 * 96 / 1024),
    "mp2_sommerfeld": lambda: W.mp2(n_int=128, n_lay=0, r=50.0 / 3, bc="sommerfeld", theta_csg=-math.pi / 8),
    "csl_c1": csl_c1,
    "smooth_c2": smooth_c2,
    "sommerfeld_3d": sommerfeld_3d,
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variant_operators_and_vcycle_match_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = VARIANTS[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    rng = np.random.default_rng(41)
    x = rng.standard_normal(g.N) + 1j * rng.standard_normal(g.N)
    xd = dev(torch, x)
    assert same(host(g.apply(xd, "H")), o.apply(x, "H"))
    assert same(host(g.apply(xd, "M")), o.apply(x, "M"))
    ref = o.vcycle(x)
    assert same(host(g.vcycle(xd, "c128")), ref)
    err = rel(host(g.vcycle(xd, "c64")).astype(np.complex128), ref)
    assert err < FP32_VCYCLE_TOL, err


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variant_bicgstab_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = VARIANTS[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    xo, io = o.solve(c["b"], tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, c["b"]), tol=1e-8, vcycle_prec="c128", history=True)
    assert io["status"] == 0 == ig["status"] and ig["rel_res_true"] < 1e-8
    assert ig["matvecs"] == io["matvecs"] and ig["iterations"] == io["iterations"]
    assert np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)
    xm, im = g.solve(dev(torch, c["b"]), tol=1e-8, vcycle_prec="c64")
    assert im["status"] == 0 and im["rel_res_true"] < 1e-8
    assert rel(host(xm), xo) <= 1e-6
    print(name, "matvecs fp64", io["matvecs"], "mixed", im["matvecs"], "err %.2e" % rel(host(xm), xo), flush=True)


@pytest.mark.parametrize("name,s", [("mp2_nu1k4", 4), ("mp2_nu1k4", 8), ("mp3_r90k2", 4), ("mp3_r90k2", 8),
                                    ("mp2_sommerfeld", 4)])
def test_variant_idr_matches_oracle(torch_dev, hh_mod, oracle_mod, name, s):
    torch = torch_dev
    c = VARIANTS[name]()
    print("case", name, "s", s, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    P = W.shadow_space(g.N, s, 2000 + s)
    xo, io = o.solve(c["b"], method="idr", s=s, P=P, tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, c["b"]), method="idr", s=s, P=hh_mod.shadow_to_device(P), tol=1e-8,
                     vcycle_prec="c128", history=True)
    assert io["status"] == 0 == ig["status"] and ig["rel_res_true"] < 1e-8
    assert ig["matvecs"] == io["matvecs"] and np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)


def test_mp2_full_size_matches_oracle(torch_dev, hh_mod, oracle_mod):
    """MP2 at the paper's size (384 interior + 128 layer cells per axis, r =
    50, nu = 7, k = 2): the whole FP64 Bi-CGSTAB solve equals the oracle's
    value for value; the mixed solve meets the tolerance against it."""
    torch = torch_dev
    c = W.mp2()
    print("case mp2 512^2", flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    xo, io = o.solve(c["b"], tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, c["b"]), tol=1e-8, vcycle_prec="c128", history=True)
    assert io["status"] == 0 == ig["status"]
    assert ig["matvecs"] == io["matvecs"] and np.array_equal(ig["history"], io["history"])
    assert same(host(xg), xo)
    xm, im = g.solve(dev(torch, c["b"]), tol=1e-8, vcycle_prec="c64")
    assert im["status"] == 0 and im["rel_res_true"] < 1e-8 and rel(host(xm), xo) <= 1e-6
    print("mp2 512^2 matvecs fp64", io["matvecs"], "mixed", im["matvecs"], flush=True)


def test_mp3_full_size(torch_dev, hh_mod, oracle_mod):
    """MP3 at the paper's size (1024 interior + 256 layer cells, r = 90, k =
    2): the first 24 FP64 matvecs equal the oracle's (history and iterate);
    the whole FP64 and mixed solves reach a true residual below 1e-8 measured
    with the oracle's operator and agree to 1e-6."""
    torch = torch_dev
    c = W.mp3()
    print("case mp3 1280^2", flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = dev(torch, c["b"])
    xo, io = o.solve(c["b"], tol=1e-8, max_matvec=24, max_restarts=0, history=True)
    xg, ig = g.solve(b, tol=1e-8, max_matvec=24, max_restarts=0, vcycle_prec="c128", history=True)
    assert io["status"] == ig["status"] and ig["matvecs"] == io["matvecs"] == 24
    assert np.array_equal(ig["history"], io["history"]) and same(host(xg), xo)
    bn = np.linalg.norm(c["b"])
    x64, i64 = g.solve(b, tol=1e-8, vcycle_prec="c128")
    xm, im = g.solve(b, tol=1e-8, vcycle_prec="c64")
    for x, i in ((x64, i64), (xm, im)):
        assert i["status"] == 0
        xh = host(x)
        assert np.linalg.norm(c["b"] - o.apply(xh, "H")) / bn < 1e-8
    assert rel(host(xm), host(x64)) <= 1e-6
    print("mp3 1280^2 matvecs fp64", i64["matvecs"], "mixed", im["matvecs"], "fallback", im["fp64_fallback"], flush=True)


@pytest.mark.parametrize("name,which,start,cycles", [("c1", "csg", math.pi / 4, 20), ("mp2_nu7k2", "csg", math.pi / 4, 30),
                                                     ("c1", "csl", 2.0, 20),
                                                     ("mp2_sommerfeld", "csg", -math.pi / 4, 20)])
def test_preconditioner_selection_matches_oracle(torch_dev, hh_mod, oracle_mod, name, which, start, cycles):
    """Sec. 6.2, remark on choosing the CSL and CSG parameters: the library's
    search (FP64 V-cycles and operator applies, norms in the contract's order)
    picks the oracle's value, with the same cycle counts and the same
    residuals for every candidate."""
    torch = torch_dev
    c = VARIANTS[name]() if name in VARIANTS else W.c1()
    print("case selection", name, which, flush=True)
    ro, to = oracle_mod.select_preconditioner(c["desc"], c["phi"], c["b"], which=which, start=start,
                                              max_cycles=cycles)
    rg, tg = hh_mod.select_preconditioner(c["desc"], dev(torch, c["b"]), phi=c["phi"], which=which, start=start,
                                          max_cycles=cycles)
    assert rg["status"] == ro["status"] == 0 and rg["tried"] == ro["tried"]
    assert rg["value"] == ro["value"] and rg["cycles"] == ro["cycles"]
    assert np.array_equal(tg, to)
    print(name, which, "chose %.4f after %d candidates, %d cycles" % (rg["value"], rg["tried"], rg["cycles"]), flush=True)


def _v01(c):
    c["desc"]["nu1"] = 0
    return c


# every kernel path of the cycle: box-tile legs, merged 2D legs (256^2, the
# full 1024^2), the one-workgroup tail, the split coarsest solve, 3D box and
# z-streaming legs, a ragged 3D grid
V01_CASES = {
    "c1": lambda: _v01(W.c1()),
    "c2_256": lambda: _v01(W.c2(n=256, levels=6)),
    "c2_1024": lambda: _v01(W.c2()),
    "c2_384_split": lambda: _v01(W.c2(n=384, levels=5)),
    "c3_32": lambda: _v01(W.c3(n=32, layer=4, method="bicgstab")),
    "c3_64": lambda: _v01(W.c3(n=64, layer=8, method="bicgstab")),
    "mp2_nu7k2": lambda: _v01(W.mp2(n_int=96, n_lay=32, r=12.5)),
}


@pytest.mark.parametrize("name", list(V01_CASES))
def test_v01_cycle_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    """The paper's V(0,1) cycle (Sec. 6.1: no pre-smoothing, one post-smoothing
    step) equals the oracle's value for value in FP64, in every kernel path."""
    torch = torch_dev
    c = V01_CASES[name]()
    print("case v01", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    rng = np.random.default_rng(51)
    f = rng.standard_normal(g.N) + 1j * rng.standard_normal(g.N)
    fd = dev(torch, f)
    ref = o.vcycle(f)
    assert same(host(g.vcycle(fd, "c128")), ref)
    err = rel(host(g.vcycle(fd, "c64")).astype(np.complex128), ref)
    assert err < FP32_VCYCLE_TOL, err
    assert same(host(g.vcycle_noalloc(fd, "c128")), ref)


@pytest.mark.parametrize("name,method", [("c1", "bicgstab"), ("mp2_nu7k2", "bicgstab"), ("mp2_nu7k2", "idr"),
                                         ("c3_32", "bicgstab")])
def test_v01_solves_match_oracle(torch_dev, hh_mod, oracle_mod, name, method):
    torch = torch_dev
    c = V01_CASES[name]()
    print("case v01 solve", name, method, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    P = W.shadow_space(g.N, 4, 4004)
    xo, io = o.solve(c["b"], method=method, s=4, P=P, tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, c["b"]), method=method, s=4, P=hh_mod.shadow_to_device(P), tol=1e-8,
                     vcycle_prec="c128", history=True)
    assert io["status"] == 0 == ig["status"] and ig["matvecs"] == io["matvecs"]
    assert np.array_equal(ig["history"], io["history"]) and same(host(xg), xo)
    print(name, method, "V(0,1) matvecs", io["matvecs"], flush=True)
