"""CPU tests of the C-ABI library: it loads, exports every symbol include/hh.h
declares, validates descriptions, and its host-side setup (node maps,
Shortley-Weller coefficients, coarse phi, coarsest inverse) equals the
oracle's value for value.  No GPU compute call is made here."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_0912_0180_amd import hh
from paper_0912_0180_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hh.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(hh.EXPORTS)
    assert b"gfx950" in L.hh_version()


def host_grid(desc, phi=None):
    return hh.Grid(desc, phi, host_only=True)


@pytest.mark.parametrize("cfg", ["c1", "c1_interior", "c3_small", "c2_small"])
def test_host_setup_equals_oracle_bitwise(oracle_mod, cfg):
    if cfg == "c1":
        c = W.c1()
    elif cfg == "c1_interior":
        c = W.c1(mode=1)
    elif cfg == "c2_small":
        c = W.c2(n=128, levels=4)
    else:
        c = W.c3(n=32, layer=4, method="bicgstab")
    g = host_grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    assert g.levels == o.nlev and g.Nc == o.Nc
    for lev in range(g.levels):
        assert g.level_dims[lev][: g.dim] == o.level_dims(lev)[: g.dim]
        for ax in range(g.dim):
            names = ["aM", "cM", "dM"] + (["aH", "cH", "dH"] if lev == 0 else [])
            for w in names:
                a, b = g.export(w, lev, ax), o.coeffs(lev, ax, w)
                assert np.array_equal(a.view(np.float64), b.view(np.float64)), (lev, ax, w)
        assert np.array_equal(g.export("phi", lev), o.phi(lev))
    assert np.array_equal(g.export("Minv").view(np.float64), o.coarse_inverse().view(np.float64))


def bad(desc, **kw):
    d = dict(desc)
    d.update(kw)
    return d


def test_invalid_descriptions_are_rejected():
    c = W.c1()
    d = c["desc"]
    cases = [bad(d, dim=4), bad(d, theta_ecs=0.0), bad(d, theta_csg=2.0), bad(d, levels=9),
             bad(d, n=[130, 128]), bad(d, nu1=2), bad(d, a=[-0.5, 0.0]), bad(d, levels=1), bad(d, omega=0.0),
             bad(d, csg_mode=5), bad(d, n=[16, 16], levels=0)]
    for dd in cases:
        with pytest.raises(hh.HHError) as e:
            host_grid(dd, c["phi"])
        assert e.value.status == -1
    phi = c["phi"].copy()
    phi[7] = np.nan
    with pytest.raises(hh.HHError):
        host_grid(d, phi)


def test_host_only_grid_refuses_compute():
    c = W.c1()
    g = host_grid(c["desc"], c["phi"])
    L = hh.lib()
    assert L.hh_apply_operator(g.h, 0, 0, 1, 2, None) == -1
    assert "host-only" in hh.last_error()
    assert L.hh_vcycle(g.h, 0, 1, 2, None) == -1


def test_auto_levels_rule():
    for n, want in [(128, 4), (1024, 7), (384, 6), (768, 7), (2048, 8)]:
        d = W.base_desc(2, (n, n), (0, 0), (1, 1), (0, 0), (1, 1), levels=0)
        g = host_grid(d, np.ones(n * n))
        assert g.levels == want, (n, g.levels)
        assert g.level_dims[-1][0] <= 16


def test_fastdiv_host_emulation(tmp_path):
    """The 32-bit division by a runtime constant used for index decomposition
    agrees with integer division (host build of the same inline function)."""
    src = tmp_path / "fd.cpp"
    src.write_text(r'''
#include "hh_common.h"
#include <cstdio>
#include <random>
int main() {
  std::mt19937 r(1);
  unsigned ds[] = {1,2,3,5,7,12,16,17,96,100,128,129,255,256,384,1000,1023,1024,2048,4095,65536,1048576,16777216};
  for (unsigned d : ds) {
    FastDiv f = make_fastdiv(d);
    for (int t = 0; t < 200000; ++t) {
      unsigned n = (t < 1000) ? t : (r() & 0x7fffffff);
      if (fdiv(n, f) != n / d) { printf("FAIL %u %u\n", n, d); return 1; }
    }
    unsigned n = 0x7fffffff; if (fdiv(n, f) != n / d) { printf("FAIL max %u\n", d); return 1; }
  }
  printf("ok\n"); return 0; }
''')
    exe = tmp_path / "fd"
    inc = os.path.join(ROOT, "paper_0912_0180_amd", "csrc")
    subprocess.check_call(["hipcc", "-O1", "-std=c++17", "-I", inc, str(src), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    assert subprocess.check_output([str(exe)]).strip() == b"ok"


def test_request_footprint_bounds():
    """The admission footprint covers the solve's vectors, hierarchy and lists
    and is not loose: it sits between the vector bytes alone and 1.5x them."""
    d2 = W.base_desc(2, (1024, 1024), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0))
    N = 1024 * 1024
    f_mixed = hh.request_footprint(d2, method="bicgstab", vcycle_prec="c64")
    f_fp64 = hh.request_footprint(d2, method="bicgstab", vcycle_prec="c128")
    f_idr = hh.request_footprint(d2, method="idr", s=4, vcycle_prec="c64")
    lower = N * (7 * 16 + 2 * 16 + 12)              # r rh p v t p^ s^ (FP64), b x, phi
    assert lower < f_mixed < 1.5 * lower
    assert f_fp64 == f_mixed                         # a mixed solve may continue in FP64
    assert f_idr - f_mixed >= N * (4 * 16)           # dR, dX and P outgrow rh/p/ph/sh
    d3 = W.base_desc(3, (64, 64, 64), (-0.2,) * 3, (1.2,) * 3, (0.0,) * 3, (1.0,) * 3)
    f3 = hh.request_footprint(d3, method="bicgstab", vcycle_prec="c64")
    assert 64 ** 3 * (7 * 16 + 2 * 16 + 12) < f3
    bad = dict(d2, n=(1000, 1024))
    bad["levels"] = 8
    with pytest.raises(hh.HHError) as e:
        hh.request_footprint(bad)
    assert e.value.status == -1


@pytest.mark.parametrize("dim", [2, 3])
def test_vertex_grid_host_setup_equals_oracle(oracle_mod, dim):
    """The vertex-centred grid of Sec. 3 (eq. (ecsgrid)): one level, node
    widths (hi - lo)/(n + 1); its H and M coefficients equal the oracle's."""
    n = {2: (12, 10), 3: (6, 5, 7)}[dim]
    d = W.base_desc(dim, n, (-0.3,) * dim, (1.3,) * dim, (0.0,) * dim, (1.0,) * dim, centering=1, levels=1)
    phi = np.random.default_rng(dim).uniform(10.0, 20.0, size=int(np.prod(n)))
    g = host_grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    assert g.levels == 1 == o.nlev
    for ax in range(dim):
        for w in ("aM", "cM", "dM", "aH", "cH", "dH"):
            assert np.array_equal(g.export(w, 0, ax).view(np.float64), o.coeffs(0, ax, w).view(np.float64)), (ax, w)
    assert np.array_equal(g.export("phi", 0), o.phi(0))


def test_vertex_grid_validation():
    d = W.base_desc(2, (12, 10), (0.0, 0.0), (1.0, 1.0), (0.0, 0.0), (1.0, 1.0), centering=1, levels=2)
    with pytest.raises(hh.HHError):
        host_grid(d)
    d["levels"] = 0
    g = host_grid(d)
    assert g.levels == 1 and g.Nc == 0
    d["centering"] = 2
    with pytest.raises(hh.HHError):
        host_grid(d)
    d["centering"] = 1
    with pytest.raises(hh.HHError) as ei:
        hh.request_footprint(d)
    assert "vertex" in str(ei.value)


def _variant(name):
    if name == "csl":
        c = W.c1()
        c["desc"].update(csg_mode=2, csl_shift=[1.0, 0.2])
        return c
    if name == "csl_interior_angle":
        c = W.c1(mode=1)
        c["desc"].update(contour_steps=8)
        return c
    if name == "smooth":
        c = W.c2(n=128, levels=4)
        c["desc"].update(contour_steps=32)
        return c
    if name == "mp2":
        return W.mp2(n_int=96, n_lay=32, r=12.5)
    if name == "mp3":
        return W.mp3(n_int=96, n_lay=32, r=90.0 * 96 / 1024)
    if name == "mp2_sommerfeld":
        return W.mp2(n_int=128, n_lay=0, r=50.0 / 3, bc="sommerfeld", theta_csg=-math.pi / 20)
    if name == "sommerfeld_3d":
        c = W.c3(n=32, layer=4, method="bicgstab")
        d = c["desc"]
        d["a"][2] = d["lo"][2]                      # no layer on the low z side: Sommerfeld there
        d["bc"][2] = [1, 0]
        d["k_bc"] = 12.0
        return c
    raise KeyError(name)


@pytest.mark.parametrize("name", ["csl", "csl_interior_angle", "smooth", "mp2", "mp3", "mp2_sommerfeld", "sommerfeld_3d"])
def test_host_setup_variants_equal_oracle_bitwise(oracle_mod, name):
    """CSL shift, smooth contours, one-sided layers and Sommerfeld sides: the
    library's node maps, coefficients, coarse phi and coarsest inverse equal
    the oracle's value for value."""
    c = _variant(name)
    g = host_grid(c["desc"], c["phi"])
    o = oracle_mod.Grid(c["desc"], c["phi"])
    assert g.levels == o.nlev and g.Nc == o.Nc
    for lev in range(g.levels):
        for ax in range(g.dim):
            names = ["aM", "cM", "dM"] + (["aH", "cH", "dH"] if lev == 0 else [])
            for w in names:
                a, b = g.export(w, lev, ax), o.coeffs(lev, ax, w)
                assert np.array_equal(a.view(np.float64), b.view(np.float64)), (name, lev, ax, w)
        assert np.array_equal(g.export("phi", lev), o.phi(lev))
    assert np.array_equal(g.export("Minv").view(np.float64), o.coarse_inverse().view(np.float64))


def test_variant_validation():
    base = W.c1()["desc"]

    def bad(**kw):
        d = dict(base)
        d.update(kw)
        with pytest.raises(hh.HHError):
            host_grid(d)

    bad(csg_mode=3)
    bad(csg_mode=2, csl_shift=[0.0, 0.0])
    bad(theta_csg=1.6)
    bad(contour_steps=-1)
    bad(bc=[[1, 0], [0, 0]], k_bc=3.0)             # Sommerfeld on a side with a layer
    d = dict(base)
    d.update(a=[-0.25, 0.0], bc=[[1, 0], [0, 0]], k_bc=0.0)
    with pytest.raises(hh.HHError):
        host_grid(d)                                # no k_bc
    d.update(k_bc=5.0)
    assert host_grid(d).levels == 4
    d2 = dict(base)
    d2.update(theta_csg=-math.pi / 20)              # negative angles are the Sommerfeld tables' choice
    assert host_grid(d2).levels == 4


def test_paper_cycle_v01_accepted():
    d = dict(W.c1()["desc"])
    d["nu1"] = 0
    assert host_grid(d).levels == 4
    for nu1, nu2 in ((0, 0), (1, 2), (2, 1)):
        d.update(nu1=nu1, nu2=nu2)
        with pytest.raises(hh.HHError):
            host_grid(d)


@pytest.mark.parametrize("cfg", ["c1", "c1_interior", "ragged", "paper"])
def test_galerkin_host_setup_equals_oracle_bitwise(oracle_mod, cfg):
    """The library's Galerkin stencils (built on the cells each column reaches)
    and the coarsest inverse equal the oracle's column-by-column R (M (P e_J))
    value for value."""
    if cfg == "ragged":
        d = W.base_desc(2, (96, 80), (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=4, coarse_op=1)
        phi = 900.0 * (1 + 0.3 * np.random.default_rng(72).uniform(size=96 * 80))
    else:
        c = W.c1_paper() if cfg == "paper" else W.c1(mode=1 if cfg == "c1_interior" else 0)
        d, phi = dict(c["desc"]), c["phi"]
        d["coarse_op"] = 1
    g = host_grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    assert g.levels == o.nlev
    for lev in range(1, g.levels):
        assert np.array_equal(g.export("galerkin", lev), o.galerkin(lev)), lev
    assert np.array_equal(g.export("Minv"), o.coarse_inverse())
    with pytest.raises(hh.HHError):
        g.export("galerkin", 0)


def test_galerkin_validation():
    base = dict(n=(32, 32), lo=(0.0, 0.0), hi=(1.0, 1.0), a=(0.0, 0.0), b=(1.0, 1.0))
    for kw, msg in ((dict(coarse_op=2), "coarse_op"), (dict(coarse_op=1, centering=1, levels=1), "2D cell-centred")):
        d = W.base_desc(2, base["n"], base["lo"], base["hi"], base["a"], base["b"], **kw)
        with pytest.raises(hh.HHError) as ei:
            host_grid(d, np.zeros(32 * 32))
        assert msg in str(ei.value)
    d3 = W.base_desc(3, (16,) * 3, (0.0,) * 3, (1.0,) * 3, (0.0,) * 3, (1.0,) * 3, coarse_op=1)
    with pytest.raises(hh.HHError) as ei:
        host_grid(d3, np.zeros(16 ** 3))
    assert "2D cell-centred" in str(ei.value)


@pytest.mark.parametrize("coarse_op", [0, 1])
@pytest.mark.parametrize("cfg", ["c1", "ragged", "paper"])
def test_ilu0_host_setup_equals_oracle_bitwise(oracle_mod, cfg, coarse_op):
    """The library's ILU(0) factors of every smoothing level (built on the host
    by the row-wise incomplete elimination) equal the oracle's value for
    value, on rediscretised and Galerkin hierarchies; the coarsest level has
    none."""
    if cfg == "ragged":
        d = W.base_desc(2, (96, 80), (-0.2, -0.3), (1.3, 1.1), (0.0, 0.0), (1.0, 0.9), levels=4)
        phi = 900.0 * (1 + 0.3 * np.random.default_rng(73).uniform(size=96 * 80))
    else:
        c = W.c1_paper() if cfg == "paper" else W.c1()
        d, phi = dict(c["desc"]), c["phi"]
    d.update(coarse_op=coarse_op, smoother=1, nu1=0, omega=1.0)
    g = host_grid(d, phi)
    o = oracle_mod.Grid(d, phi)
    assert g.levels == o.nlev
    for lev in range(g.levels - 1):
        assert np.array_equal(g.export("ilu", lev), o.ilu(lev)), lev
    with pytest.raises(hh.HHError):
        g.export("ilu", g.levels - 1)


def test_ilu0_validation():
    base = dict(n=(32, 32), lo=(0.0, 0.0), hi=(1.0, 1.0), a=(0.0, 0.0), b=(1.0, 1.0))
    cases = ((dict(smoother=2), "smoother"), (dict(smoother=1, nu1=1), "V(0,1)"),
             (dict(smoother=1, nu1=0, centering=1, levels=1), "2D cell-centred"),
             (dict(smoother=1, nu1=0, levels=5), "at least 5 cells"))
    for kw, msg in cases:
        d = W.base_desc(2, base["n"], base["lo"], base["hi"], base["a"], base["b"], **kw)
        with pytest.raises(hh.HHError) as ei:
            host_grid(d, np.zeros(32 * 32))
        assert msg in str(ei.value), (kw, str(ei.value))
    d3 = W.base_desc(3, (16,) * 3, (0.0,) * 3, (1.0,) * 3, (0.0,) * 3, (1.0,) * 3, smoother=1, nu1=0)
    with pytest.raises(hh.HHError) as ei:
        host_grid(d3, np.zeros(16 ** 3))
    assert "2D cell-centred" in str(ei.value)
