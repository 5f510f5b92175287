"""GPU parity of the Galerkin coarse operators (Sec. 6.1; 2D, cell-centred)
against the CPU FP64 oracle, through the C ABI.

The library builds M_{l+1} = R M_l P on the host (the same values as the
oracle's column-by-column definition, tested bitwise on the CPU); the device
V-cycle applies the 25-point stencils in the oracle's operation order, so
FP64 V-cycles and whole FP64 Bi-CGSTAB solves equal the oracle's value for
value.  The FP32 cycle is held to 1e-5 in norm: its measured error is up to
1.0e-6 (the 25-point stencils cancel more than the 5-point ones, whose FP32
cycle stays near 1.4e-7), and the bound keeps a 10x margin.
"""
import math

import numpy as np
import pytest

from paper_0912_0180_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def c1_gal(nu1=1, mode=0):
    c = W.c1(mode=mode)
    d = dict(c["desc"])
    d["coarse_op"] = 1
    d["nu1"] = nu1
    return {"desc": d, "phi": c["phi"], "b": c["b"]}


def ragged_gal(nu1=1):
    d = W.base_desc(2, (96, 80), (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=4, nu1=nu1, coarse_op=1)
    rng = np.random.default_rng(71)
    phi = (30.0 ** 2) * (1 + 0.3 * rng.uniform(size=96 * 80))
    return {"desc": d, "phi": phi}


def paper_gal(nu1=0):
    """C1-paper (192^2, k = 80) in the paper's own configuration: Galerkin
    coarse operators and a V(0,1) cycle (with weighted Jacobi)."""
    c = W.c1_paper()
    d = dict(c["desc"])
    d["coarse_op"] = 1
    d["nu1"] = nu1
    return {"desc": d, "phi": c["phi"], "b": c["b"]}


CASES = {"c1_v11": lambda: c1_gal(1), "c1_v01": lambda: c1_gal(0), "c1_interior": lambda: c1_gal(1, mode=1),
         "ragged_v11": lambda: ragged_gal(1), "ragged_v01": lambda: ragged_gal(0), "paper_v01": lambda: paper_gal(0)}


@pytest.mark.parametrize("name", list(CASES))
def test_galerkin_vcycle_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    for lev in range(1, g.levels):
        assert np.array_equal(g.export("galerkin", lev), o.galerkin(lev)), lev
    f = rand_c(np.random.default_rng(5), g.N)
    fd = dev(torch, f)
    u64 = host(g.vcycle(fd, "c128"))
    u32 = host(g.vcycle(fd, "c64"))
    torch.cuda.synchronize()
    ref = o.vcycle(f)
    assert np.array_equal(u64, ref)
    err = rel(u32.astype(np.complex128), ref)
    assert err < 1e-5, err


@pytest.mark.parametrize("name", ["c1_v11", "ragged_v01", "paper_v01"])
def test_galerkin_bicgstab_fp64_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c.get("b")
    if b is None:
        b = rand_c(np.random.default_rng(6), g.N)
    xo, io = o.solve(b, tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, b), tol=1e-8, vcycle_prec="c128", history=True)
    assert io["status"] == 0 and ig["status"] == 0
    assert ig["matvecs"] == io["matvecs"] and ig["iterations"] == io["iterations"]
    assert np.array_equal(host(xg), xo)
    assert np.array_equal(ig["history"], io["history"])


def test_galerkin_mixed_precision_solve(torch_dev, hh_mod, oracle_mod):
    torch = torch_dev
    c = CASES["paper_v01"]()
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    xg, ig = g.solve(dev(torch, c["b"]), tol=1e-8, vcycle_prec="c64")
    xo, io = o.solve(c["b"], tol=1e-8)
    assert ig["status"] == 0 and ig["rel_res_true"] < 1e-8
    assert rel(host(xg), xo) < 1e-6


def test_galerkin_noalloc_equals_vcycle(torch_dev, hh_mod):
    torch = torch_dev
    c = CASES["ragged_v11"]()
    g = hh_mod.Grid(c["desc"], c["phi"])
    f = dev(torch, rand_c(np.random.default_rng(8), g.N))
    for prec in ("c128", "c64"):
        a = host(g.vcycle(f, prec))
        b = host(g.vcycle_noalloc(f, prec))
        torch.cuda.synchronize()
        assert np.array_equal(a, b), prec


def test_galerkin_batches_rejected(torch_dev, hh_mod):
    torch = torch_dev
    c = CASES["c1_v11"]()
    grids = [hh_mod.Grid(c["desc"], c["phi"]) for _ in range(2)]
    bs = [dev(torch, c["b"]) for _ in range(2)]
    with pytest.raises(hh_mod.HHError) as ei:
        hh_mod.solve_batch(grids, bs, tol=1e-8, vcycle_prec="c128")
    assert "Galerkin" in str(ei.value)
    sv = hh_mod.Server(budget=0, max_slots=2)
    try:
        with pytest.raises(hh_mod.HHError) as ei:
            sv.submit(c["desc"], c["b"], phi=c["phi"])
        assert "Galerkin" in str(ei.value)
    finally:
        sv.close()
