"""Full-size closed-form pins of the HIP operator apply, independent of the
oracle.

On the vertex-centred grid of Sec. 3 (eq. (ecsgrid)) without layers the
Helmholtz operator is the textbook 2d+1-point Dirichlet matrix: its
eigenvectors are tensor products of sin(j pi i/(n+1)) and its eigenvalues
sum_a (4/h_a^2) sin^2(j_a pi/(2(n_a+1))) - k^2.  The uniform CSG of Sec. 5.3
(eq. (CSL-CSG)) multiplies every width by beta, so the preconditioner M has
the same eigenvectors with eigenvalues lambda_L/beta^2 - k^2.  Both are
checked at the full sizes of the 2D and 3D workloads (1024^2, 128^3), for low,
middle and high modes, with the error measured against the operator's scale:
||A v - lambda v|| <= 1e-13 * ||A||_inf * ||v||, ||A||_inf = sum_a 4/h_a^2 * 2
+ k^2 bounding every row sum of |A| (the rounding of one stencil is a few ulps
of that scale).
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


def sine_mode(ns, js):
    v = None
    for n, j in zip(ns, js):
        s = np.sin(j * np.pi * np.arange(1, n + 1) / (n + 1))
        v = s if v is None else np.kron(s, v)   # x fastest
    return v


@pytest.mark.parametrize("dim,n", [(2, 1024), (3, 128)])
def test_dirichlet_and_uniform_csg_eigenpairs_full_size(torch_dev, hh_mod, dim, n):
    torch = torch_dev
    lo, hi = 0.0, 1.5
    theta_b = math.pi / 8
    ns = (n,) * dim
    d = W.base_desc(dim, ns, (lo,) * dim, (hi,) * dim, (lo,) * dim, (hi,) * dim, theta_csg=theta_b,
                    centering=1, levels=1)
    h = (hi - lo) / (n + 1)
    k2 = (0.625 / h) ** 2 * 0.7
    d["phi_const"] = k2
    print("case vertex", dim, n, flush=True)
    g = hh_mod.Grid(d)
    assert g.levels == 1 and g.N == n ** dim
    beta2 = complex(math.cos(2 * theta_b), math.sin(2 * theta_b))
    scale = dim * 8.0 / h ** 2 + k2
    worst = {"H": 0.0, "M": 0.0}
    for js in [(1,) * dim, (2, 3, 5)[:dim], (n // 2, n // 3, 7)[:dim], (n,) * dim, (n - 1, 1, n // 4)[:dim]]:
        v = sine_mode(ns, js)
        lamL = sum(4.0 / h ** 2 * math.sin(j * math.pi / (2 * (n + 1))) ** 2 for j in js)
        vd = torch.from_numpy(v.astype(np.complex128)).to("cuda")
        for op, lam in (("H", lamL - k2), ("M", lamL / beta2 - k2)):
            y = g.apply(vd, op).cpu().numpy()
            err = np.linalg.norm(y - lam * v) / (scale * np.linalg.norm(v))
            worst[op] = max(worst[op], err)
            assert err <= 1e-13, (op, js, err)
    print("vertex eigenpairs", dim, n, "worst scaled error H %.2e M %.2e" % (worst["H"], worst["M"]), flush=True)


def test_vertex_grid_rejects_multigrid_calls(torch_dev, hh_mod):
    torch = torch_dev
    d = W.base_desc(2, (64, 64), (0.0, 0.0), (1.0, 1.0), (0.0, 0.0), (1.0, 1.0), centering=1, levels=1)
    d["phi_const"] = 100.0
    g = hh_mod.Grid(d)
    f = torch.ones(g.N, dtype=torch.complex128, device="cuda")
    for call in (lambda: g.vcycle(f), lambda: g.vcycle_noalloc(f), lambda: g.solve(f)):
        with pytest.raises(hh_mod.HHError) as ei:
            call()
        assert ei.value.status == -1 and "vertex" in str(ei.value)
