"""The allocation-free V-cycle (hh_vcycle_noalloc) against hh_vcycle, through
the C ABI.

Both run the same kernels over the same levels; only where the coarse levels'
restricted right-hand sides and solutions live differs (the library's static
scratch array instead of memory the grid allocates).  Results must be equal
value for value in complex double and in complex float, on consecutive calls
over grids of decreasing size (the scratch keeps the previous call's
contents), before and after hh_vcycle has planned (and tuned) the same grid.
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


def same(torch, a, b):
    torch.cuda.synchronize()
    return bool(torch.equal(torch.view_as_real(a), torch.view_as_real(b)))


def rhs(torch, N, seed):
    g = np.random.default_rng(seed)
    f = g.standard_normal(N) + 1j * g.standard_normal(N)
    return torch.from_numpy(f).to("cuda")


# largest first: the full-size 1024^2 problem (merged coarse legs), a 384^2
# grid whose 576-unknown coarsest solve is spread over workgroups, the 128^2
# C1 problem, a 3D grid with z-streaming legs
SEQUENCE = [
    ("c2_1024", lambda: W.c2()),
    ("c2_384_split", lambda: W.c2(n=384, levels=5)),
    ("c1", lambda: W.c1()),
    ("c3_32", lambda: W.c3(n=32, layer=4, method="bicgstab")),
]


def test_noalloc_equals_vcycle_on_consecutive_grids(torch_dev, hh_mod):
    torch = torch_dev
    for name, make in SEQUENCE:
        c = make()
        g = hh_mod.Grid(c["desc"], c["phi"])
        f = rhs(torch, g.N, 7)
        for prec in ("c128", "c64"):
            print("case", name, prec, flush=True)
            # first on a grid no plan has seen, then the planned cycle, then again
            u0 = g.vcycle_noalloc(f, prec)
            u1 = g.vcycle(f, prec)
            u2 = g.vcycle_noalloc(f, prec)
            assert same(torch, u0, u1), (name, prec)
            assert same(torch, u2, u1), (name, prec)
        g.close()


def test_noalloc_rejects_grids_beyond_the_scratch(torch_dev, hh_mod):
    """2048^2 with 8 levels: the coarse levels need about 45 MB in complex
    double (over the 32 MiB array) and 22 MB in complex float."""
    torch = torch_dev
    n = 2048
    d = W.base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0), levels=8)
    phi = np.full(n * n, (0.625 * n / 1.5) ** 2)
    g = hh_mod.Grid(d, phi)
    f = rhs(torch, g.N, 8)
    print("case 2048 c128 rejected", flush=True)
    with pytest.raises(hh_mod.HHError) as ei:
        g.vcycle_noalloc(f, "c128")
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    print("case 2048 c64", flush=True)
    u = g.vcycle_noalloc(f, "c64")
    assert same(torch, u, g.vcycle(f, "c64"))
    # a smaller grid after it still matches
    c = W.c1()
    g2 = hh_mod.Grid(c["desc"], c["phi"])
    f2 = rhs(torch, g2.N, 9)
    assert same(torch, g2.vcycle_noalloc(f2, "c128"), g2.vcycle(f2, "c128"))
    g.close()
    g2.close()


def test_noalloc_argument_errors(torch_dev, hh_mod):
    torch = torch_dev
    import ctypes
    c = W.c1()
    g = hh_mod.Grid(c["desc"], c["phi"])
    f = rhs(torch, g.N, 10)
    L = hh_mod.lib()
    p = ctypes.c_void_p(f.data_ptr())
    assert L.hh_vcycle_noalloc(g.h, hh_mod.C128, p, p, None) == -1          # f == u
    assert L.hh_vcycle_noalloc(g.h, 7, p, ctypes.c_void_p(1), None) == -1  # unknown precision
    assert L.hh_vcycle_noalloc(None, hh_mod.C128, p, p, None) == -1
    g.close()
