"""Writes ecs_1d_scaled_matrix.json: rows of the scaled 1D ECS operator
-h^2 L_h exactly as printed (symbolically) in the proof of Lemma 3.1 of the
paper, evaluated at gamma = e^{i theta}.  Calls nothing but the standard
library: the values are the paper's formulas, not any implementation's."""
import cmath
import json
import math
import os

n_int, m_lay, theta = 6, 4, math.pi / 6
g = cmath.exp(1j * theta)


def c(z):
    return [z.real, z.imag]


rows = [
    {"node": 1, "formula": "(-1, 2, -1) interior row", "lower": c(-1 + 0j), "diag": c(2 + 0j), "upper": c(-1 + 0j)},
    {"node": n_int, "formula": "turning point: -2/(1+g), 2(1+1/g)/(1+g), -2/(g(1+g))",
     "lower": c(-2 / (1 + g)), "diag": c(2 * (1 + 1 / g) / (1 + g)), "upper": c(-2 / (g * (1 + g)))},
    {"node": n_int + 1, "formula": "contour row (-1, 2, -1)/g^2", "lower": c(-1 / g ** 2), "diag": c(2 / g ** 2),
     "upper": c(-1 / g ** 2)},
    {"node": n_int + m_lay - 1, "formula": "last contour row (-1, 2)/g^2 (Dirichlet end)", "lower": c(-1 / g ** 2),
     "diag": c(2 / g ** 2), "upper": c(0j)},
]
fx = {"source": "paper, Sec. 3, proof of Lemma 3.1: the scaled operator -h^2 L_h on the ECS grid of eq. (ecsgrid)",
      "n_interior": n_int, "m_layer": m_lay, "theta": theta, "gamma": c(g), "rows": rows}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ecs_1d_scaled_matrix.json"), "w") as fh:
    json.dump(fx, fh, indent=1)
