"""GPU parity of the ILU(0) smoother (Sec. 6.1, the paper's multigrid: ILU(0)
post-smoothing in a V(0,1) cycle, on Galerkin or rediscretised coarse
operators; 2D, cell-centred, FP64) against the CPU FP64 oracle, through the
C ABI.

The library factors every smoothing level on the host (the same values as the
oracle's, tested bitwise on the CPU); the device's up-legs solve with the
factors along anti-diagonals, every per-point operation in the oracle's
order, so V-cycles and whole FP64 Bi-CGSTAB and IDR(s) solves equal the
oracle's value for value.
"""
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


def ilu_case(c, coarse_op, omega=1.0):
    d = dict(c["desc"])
    d.update(coarse_op=coarse_op, smoother=1, nu1=0, omega=omega)
    return {"desc": d, "phi": c["phi"], "b": c.get("b")}


def ragged(coarse_op):
    d = W.base_desc(2, (96, 80), (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=4)
    rng = np.random.default_rng(74)
    phi = (30.0 ** 2) * (1 + 0.3 * rng.uniform(size=96 * 80))
    return ilu_case({"desc": d, "phi": phi}, coarse_op, omega=0.9)


def tall(coarse_op):
    """48 x 2096 cells, 5 levels: more rows than the row form's workgroup on
    the levels 0 (2096 rows), 1 (1048) and 2 (524, Galerkin), each solved in
    one pass with a thread owning rows t, t + NT, ...; the pointwise phases of
    every smoothing level run grid-wide (the c1 cases and HH_ILU_FUSED cover
    them inside the solve kernel)."""
    h = 1.0 / 64
    n = (48, 2096)
    hi = (-0.2 + n[0] * h, -0.3 + n[1] * h)
    d = W.base_desc(2, n, (-0.2, -0.3), hi, (0.0, 0.0), (hi[0] - 0.2, hi[1] - 0.35), levels=5)
    rng = np.random.default_rng(75)
    phi = (8.0 ** 2) * (1 + 0.3 * rng.uniform(size=n[0] * n[1]))
    return ilu_case({"desc": d, "phi": phi}, coarse_op, omega=0.9)


def wide_redisc():
    """1088^2 cells, 7 levels, rediscretised 5-point operators: the finest
    level is wider than the one-pass form allows (1088 > 1024 columns) and
    taller than its workgroup, so it runs in 2 bands of 544 rows."""
    n = (1088, 1088)
    h = 1.0 / 1024
    hi = (-0.01 + n[0] * h, -0.01 + n[1] * h)
    d = W.base_desc(2, n, (-0.01, -0.01), hi, (0.0, 0.0), (hi[0] - 0.02, hi[1] - 0.02), levels=7)
    rng = np.random.default_rng(76)
    phi = (40.0 ** 2) * (1 + 0.3 * rng.uniform(size=n[0] * n[1]))
    return ilu_case({"desc": d, "phi": phi}, 0, omega=0.9)


CASES = {"c1_gal": lambda: ilu_case(W.c1(), 1), "c1_redisc": lambda: ilu_case(W.c1(), 0),
         "c1_interior_gal": lambda: ilu_case(W.c1(mode=1), 1), "ragged_gal": lambda: ragged(1),
         "ragged_redisc": lambda: ragged(0), "paper_gal": lambda: ilu_case(W.c1_paper(), 1),
         "tall_gal": lambda: tall(1), "tall_redisc": lambda: tall(0), "wide_redisc": wide_redisc}


@pytest.mark.parametrize("name", list(CASES))
def test_ilu_vcycle_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    for lev in range(g.levels - 1):
        assert np.array_equal(g.export("ilu", lev), o.ilu(lev)), lev
    f = rand_c(np.random.default_rng(15), g.N)
    fd = dev(torch, f)
    u = host(g.vcycle(fd, "c128"))
    torch.cuda.synchronize()
    assert np.array_equal(u, o.vcycle(f))
    # a second call from the same f gives the same cycle (the work space is rewritten)
    assert np.array_equal(host(g.vcycle(fd, "c128")), u)


@pytest.mark.parametrize("name", ["c1_gal", "c1_redisc", "ragged_gal", "paper_gal", "tall_gal", "tall_redisc"])
def test_ilu_bicgstab_fp64_matches_oracle(torch_dev, hh_mod, oracle_mod, name):
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    b = c["b"] if c["b"] is not None else rand_c(np.random.default_rng(16), g.N)
    xo, io = o.solve(b, tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, b), tol=1e-8, vcycle_prec="c128", history=True)
    print("matvecs", io["matvecs"], ig["matvecs"], flush=True)
    assert io["status"] == 0 and ig["status"] == 0
    assert ig["matvecs"] == io["matvecs"] and ig["iterations"] == io["iterations"]
    assert np.array_equal(host(xg), xo)
    assert np.array_equal(ig["history"], io["history"])


@pytest.mark.parametrize("s", [4, 8])
def test_ilu_idr_fp64_matches_oracle(torch_dev, hh_mod, oracle_mod, s):
    torch = torch_dev
    c = CASES["c1_gal"]()
    print("case c1_gal s", s, flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    P = W.shadow_space(g.N, s, 2000 + s)
    xo, io = o.solve(c["b"], method="idr", s=s, P=P, tol=1e-8, history=True)
    xg, ig = g.solve(dev(torch, c["b"]), method="idr", s=s, P=hh_mod.shadow_to_device(P), tol=1e-8,
                     vcycle_prec="c128", history=True)
    assert io["status"] == 0 and ig["status"] == 0
    assert ig["matvecs"] == io["matvecs"] and ig["iterations"] == io["iterations"]
    assert np.array_equal(host(xg), xo)
    assert np.array_equal(ig["history"], io["history"])


def test_ilu_noalloc_equals_vcycle(torch_dev, hh_mod):
    torch = torch_dev
    c = CASES["ragged_gal"]()
    g = hh_mod.Grid(c["desc"], c["phi"])
    f = dev(torch, rand_c(np.random.default_rng(17), g.N))
    a = host(g.vcycle(f, "c128"))
    b = host(g.vcycle_noalloc(f, "c128"))
    torch.cuda.synchronize()
    assert np.array_equal(a, b)


def test_ilu_rejections(torch_dev, hh_mod):
    """ILU(0) runs in the FP64 cycle of single solves and V-cycle calls."""
    torch = torch_dev
    c = CASES["c1_gal"]()
    g = hh_mod.Grid(c["desc"], c["phi"])
    b = dev(torch, c["b"])
    for call in (lambda: g.vcycle(b, "c64"), lambda: g.vcycle_noalloc(b, "c64"),
                 lambda: g.solve(b, tol=1e-8, vcycle_prec="c64"), lambda: g.profile_vcycle(b, "c128", reps=1)):
        with pytest.raises(hh_mod.HHError):
            call()
    c = CASES["c1_redisc"]()   # rediscretised: the ILU(0) check, not the Galerkin one, answers
    grids = [hh_mod.Grid(c["desc"], c["phi"]) for _ in range(2)]
    with pytest.raises(hh_mod.HHError) as ei:
        hh_mod.solve_batch(grids, [b, b.clone()], tol=1e-8, vcycle_prec="c128")
    assert "ILU(0)" in str(ei.value)
    sv = hh_mod.Server(budget=0, max_slots=2)
    try:
        with pytest.raises(hh_mod.HHError) as ei:
            sv.submit(c["desc"], c["b"], phi=c["phi"])
        assert "ILU(0)" in str(ei.value)
    finally:
        sv.close()


@pytest.mark.parametrize("layers,csl", [(True, False), (False, False), (False, True)])
def test_ilu_mp1_table_problem_matches_oracle(torch_dev, hh_mod, oracle_mod, layers, csl):
    """Table MP1's problem at the paper's size (256 interior points per axis:
    384^2 with ECS layers, 256^2 with the Sommerfeld condition) and tolerance
    (1e-6), in the paper's multigrid configuration: the GPU's Bi-CGSTAB solve
    equals the oracle's value for value (whose matvec counts are held against
    the table on the CPU)."""
    torch = torch_dev
    c = W.mp1(layers=layers)
    if csl:   # the table's CSL row, beta^2 = 1 + 0.2i (printed shift -1 + 0.2i with the Sommerfeld condition)
        d = dict(c["desc"])
        d["csg_mode"] = 2
        d["csl_shift"] = [1.0, -0.2]
        c = dict(c, desc=d)
    print("case mp1", "ecs" if layers else "sommerfeld", "csl" if csl else "csg", flush=True)
    g = hh_mod.Grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    xo, io = o.solve(c["b"], tol=1e-6, history=True)
    xg, ig = g.solve(dev(torch, c["b"]), tol=1e-6, vcycle_prec="c128", history=True)
    print("matvecs", io["matvecs"], ig["matvecs"], flush=True)
    assert io["status"] == 0 and ig["status"] == 0
    assert ig["matvecs"] == io["matvecs"]
    assert np.array_equal(host(xg), xo)
    assert np.array_equal(ig["history"], io["history"])


@pytest.mark.parametrize("name", ["c1_gal", "ragged_redisc", "tall_gal", "wide_redisc"])
def test_ilu_up_leg_forms_are_equal(torch_dev, hh_mod, oracle_mod, monkeypatch, name):
    """The up-leg's forms: the pipelined row form (in bands where a level has
    more rows than its workgroup), the global-memory form (HH_ILU_GLOBAL=1 on
    every level), and the pointwise phases inside the sweep kernel
    (HH_ILU_FUSED=1) instead of grid-wide on large levels.  Every combination
    gives the oracle's cycle value for value."""
    torch = torch_dev
    c = CASES[name]()
    print("case", name, flush=True)
    o = oracle_mod.Grid(c["desc"], c["phi"])
    f = rand_c(np.random.default_rng(18), o.N)
    ref = o.vcycle(f)
    fd = dev(torch, f)
    for glob in (False, True):
        for fused in (False, True):
            for var, on in (("HH_ILU_GLOBAL", glob), ("HH_ILU_FUSED", fused)):
                monkeypatch.setenv(var, "1") if on else monkeypatch.delenv(var, raising=False)
            g = hh_mod.Grid(c["desc"], c["phi"])
            assert np.array_equal(host(g.vcycle(fd, "c128")), ref), (glob, fused)
            g.close()
