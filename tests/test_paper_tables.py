"""The paper's own multigrid (Sec. 6.1: ILU(0) smoothing in a V(0,1) cycle
on Galerkin coarse operators) reproduces Table MP1 (Sec. 6.2), whose figures
are stored in tests/golden/mp1_table.json with their citation.

This pins the whole preconditioner chain (the ECS/CSG geometry, the
Shortley-Weller operator, the transfers, the Galerkin products, the ILU(0)
factors and the Krylov solvers) against numbers the paper prints, not
against the oracle itself.  The discretisations are not identical: this
build's grids are cell-centred (the paper's are vertex-centred), its point
source sits in the cell past the centre (a cell-centred grid has no centre
node), and its IDR(s) shadow spaces are its own seeded random ones.  So the
bounds are bands, not equalities: the multigrid factor within 0.05 and its
cycle count within 4 of the table's; every matvec count within 10% of the
table's with the Sommerfeld condition (measured: 74/74/71 against 74/70/72
with the CSG, 76/71/74 against 79/72/76 with the CSL), the CSG Bi-CGSTAB count
within 5% (it is equal), and within 25% with ECS layers, whose cell-centred
layers put this build 10-24% above the table (67/69/63 against 58/62/56 with
the CSG, 73/70/66 against 59/62/60 with the CSL).  The CSL rows use the
table's first shift (printed -1 -+ 0.2i, the negated beta^2); its other shift,
-e^{+-2i pi/28}, makes the CSL a multiple of the CSG of angle pi/28 (eq.
(CSL-CSG)), so those rows repeat the CSG counts here.
"""
import json
import os

import numpy as np
import pytest

from paper_0912_0180_amd import workloads as W

TABLE = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mp1_table.json")))


ROWS = ["ecs", "sommerfeld", "ecs_csl", "sommerfeld_csl"]


def mp1_row(row):
    """The grid description of a table row: CSG (angle +-pi/28) or the CSL with
    beta^2 = 1 -+ 0.2i."""
    c = W.mp1(layers=row.startswith("ecs"))
    if row.endswith("_csl"):
        d = dict(c["desc"])
        d["csg_mode"] = 2
        d["csl_shift"] = [1.0, 0.2 if row == "ecs_csl" else -0.2]
        c = dict(c, desc=d)
    return c


@pytest.mark.parametrize("bc", ROWS)
def test_mp1_multigrid_factor_matches_table(oracle_mod, bc):
    """The V(0,1) cycle as a standalone solver of the preconditioner problem
    M u = f (u <- u + V(f - M u) from u = 0) until the residual drops by
    seven orders; average factor per cycle against the table's."""
    c = mp1_row(bc)
    o = oracle_mod.Grid(c["desc"], c["phi"])
    f = c["b"]
    u = np.zeros(o.N, dtype=complex)
    r, r0, it = f.copy(), np.linalg.norm(f), 0
    while np.linalg.norm(r) > 1e-7 * r0 and it < 40:
        u = u + o.vcycle(r)
        r = f - o.apply(u, "M")
        it += 1
    factor = (np.linalg.norm(r) / r0) ** (1.0 / it)
    want = TABLE[bc]
    print(bc, "cycles", it, "factor", factor)
    assert abs(factor - want["mg_factor"]) <= 0.05, factor
    assert abs(it - want["mg_cycles"]) <= 4, it


@pytest.mark.parametrize("bc", ROWS)
def test_mp1_matvecs_match_table(oracle_mod, bc):
    """Bi-CGSTAB, IDR(4) and IDR(8) preconditioned by one V(0,1) cycle, to a
    relative residual of 1e-6 (the paper's tolerance)."""
    c = mp1_row(bc)
    o = oracle_mod.Grid(c["desc"], c["phi"])
    want = TABLE[bc]
    got = {}
    for key, kw in (("bicgstab", {}), ("idr4", dict(method="idr", s=4, P=W.shadow_space(o.N, 4, 504))),
                    ("idr8", dict(method="idr", s=8, P=W.shadow_space(o.N, 8, 508)))):
        _, info = o.solve(c["b"], tol=1e-6, **kw)
        assert info["status"] == 0, (key, info)
        got[key] = info["matvecs"]
    print(bc, got)
    band = 0.25 if bc.startswith("ecs") else 0.10
    for key in got:
        assert abs(got[key] - want[key]) <= band * want[key], (key, got[key], want[key])
    if bc == "sommerfeld":
        assert abs(got["bicgstab"] - want["bicgstab"]) <= 0.05 * want["bicgstab"], got
