"""Writes csg_interior_1d_scaled_matrix.json: rows of the scaled 1D operator
-h^2 M_h of the interior-only complex stretched grid (Sec. 5.3, eq.
(lapctucsg) and fig. ctucsg): the interior mesh width h becomes beta*h, the
contour keeps its width gamma*h, and the grid stays connected at the turning
points.  Shortley-Weller rows (Sec. 3, eq. (shortwell)) on those widths:
a node with left width hl and right width hr has the row
  ( -2/(hl (hl+hr)),  2/(hl (hl+hr)) + 2/(hr (hl+hr)),  -2/(hr (hl+hr)) ),
so an interior row is (-1, 2, -1)/beta^2, a contour row (-1, 2, -1)/gamma^2,
and a turning-point row mixes beta and gamma.  Calls nothing but the standard
library: the values are the paper's widths put into that formula, not any
implementation's output.

Two vertex-centred grids (Sec. 3, eq. (ecsgrid)) with h = 1/n_int:
  "right":     interior [0, 1] (n_int intervals), a layer of m_lay intervals
               on the right only, Dirichlet at both ends;
  "two_sided": interior [1, 2] (n_int intervals) with m_lay-interval layers
               on both sides, so the interior does not start at the origin.
"""
import cmath
import json
import math
import os

n_int, m_lay = 6, 4
theta_g, theta_b = math.pi / 6, math.pi / 8
g = cmath.exp(1j * theta_g)
b = cmath.exp(1j * theta_b)


def c(z):
    return [z.real, z.imag]


def row(node, hl, hr, what, last=False, first=False):
    """Row of -h^2 M_h at a node with left/right widths hl*h, hr*h."""
    s = hl + hr
    return {"node": node, "formula": what,
            "lower": c(0j if first else -2 / (hl * s)),
            "diag": c(2 / (hl * s) + 2 / (hr * s)),
            "upper": c(0j if last else -2 / (hr * s))}


right = {
    "lo": 0.0, "a": 0.0, "b": 1.0, "hi": 1.0 + m_lay / n_int, "unknowns": n_int + m_lay - 1,
    "rows": [
        row(1, b, b, "first interior row (-1, 2, -1)/beta^2 (Dirichlet neighbour at 0)", first=True),
        row(3, b, b, "interior row (-1, 2, -1)/beta^2"),
        row(n_int, b, g, "turning point: left width beta h, right width gamma h"),
        row(n_int + 1, g, g, "contour row (-1, 2, -1)/gamma^2"),
        row(n_int + m_lay - 1, g, g, "last contour row, Dirichlet end", last=True),
    ],
}
two = {
    "lo": 1.0 - m_lay / n_int, "a": 1.0, "b": 2.0, "hi": 2.0 + m_lay / n_int, "unknowns": n_int + 2 * m_lay - 1,
    "rows": [
        row(1, g, g, "first left-contour row (-1, 2, -1)/gamma^2", first=True),
        row(m_lay, g, b, "left turning point: left width gamma h, right width beta h"),
        row(m_lay + 2, b, b, "interior row (-1, 2, -1)/beta^2"),
        row(m_lay + n_int, b, g, "right turning point: left width beta h, right width gamma h"),
        row(m_lay + n_int + 1, g, g, "right contour row (-1, 2, -1)/gamma^2"),
    ],
}
fx = {"source": "paper, Sec. 5.3, eq. (lapctucsg) and fig. ctucsg: interior widths beta*h, contour widths gamma*h; "
                "Sec. 3, eq. (shortwell) for the rows",
      "n_interior": n_int, "m_layer": m_lay, "theta_ecs": theta_g, "theta_csg": theta_b,
      "gamma": c(g), "beta": c(b), "grids": {"right": right, "two_sided": two}}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csg_interior_1d_scaled_matrix.json"), "w") as fh:
    json.dump(fx, fh, indent=1)
