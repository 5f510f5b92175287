"""Seeded synthetic inputs: grid descriptions, wave-number fields, right-hand
sides and IDR shadow spaces for the benchmark and test problems.

This module holds none of the solver's arithmetic.  It produces the *inputs*
both the device library and the CPU oracle receive: the geometry parameters,
phi = k(x)^2 sampled at the real cell centres, source vectors, and the random
shadow space of IDR(s).  All randomness comes from
numpy.random.Generator(PCG64(seed)).

Problem family (Sec. 4 of the paper, eq. (Helgen)): -(Lap + phi) u = chi on a
box whose interior [a, b] per axis is surrounded by exterior-complex-scaled
layers out to [lo, hi]; Dirichlet at lo and hi.  The paper's own model
problems are analytic (MP1 point source with constant k; MP2/MP3 analytic
potentials); the larger workloads here follow the same recipe with seeded
Gaussian-bump wave numbers and Gaussian sources, at 10 (or the stated)
points per wavelength, kh < 0.625 (Sec. 4).
"""
import math

import numpy as np

PI = math.pi


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def base_desc(dim, n, lo, hi, a, b, theta_ecs=PI / 6, theta_csg=PI / 8, csg_mode=0, levels=0,
              nu1=1, nu2=1, omega=0.8, centering=0, csl_shift=(0.0, 0.0), contour_steps=0, bc=None, k_bc=0.0,
              coarse_op=0, smoother=0):
    """Grid description (the keys of the library's hh_grid_desc).  bc: per axis
    [low side, high side], 0 Dirichlet / contour end, 1 Sommerfeld (wave number
    k_bc); csg_mode 2 is the CSL preconditioner with the shift csl_shift;
    coarse_op 1 takes Galerkin coarse operators (2D); smoother 1 takes ILU(0)
    smoothing (2D, V(0,1), omega its relaxation factor)."""
    return {"dim": dim, "n": list(n), "lo": list(lo), "hi": list(hi), "a": list(a), "b": list(b),
            "theta_ecs": float(theta_ecs), "theta_csg": float(theta_csg), "csg_mode": int(csg_mode),
            "centering": int(centering), "levels": int(levels), "nu1": int(nu1), "nu2": int(nu2),
            "omega": float(omega), "csl_shift": [float(csl_shift[0]), float(csl_shift[1])],
            "contour_steps": int(contour_steps), "bc": [list(v) for v in (bc or [[0, 0]] * dim)],
            "k_bc": float(k_bc), "coarse_op": int(coarse_op), "smoother": int(smoother)}


def cell_centres(n, lo, hi):
    """Real coordinates of the n cell centres of [lo, hi]."""
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


def grid_coords(desc):
    """Per-axis cell-centre coordinate arrays (x fastest in the flattened layout)."""
    return [cell_centres(desc["n"][d], desc["lo"][d], desc["hi"][d]) for d in range(desc["dim"])]


def flat(field):
    """Flatten an array indexed [x, y, z] to the x-fastest layout."""
    return np.ascontiguousarray(np.asarray(field).transpose().reshape(-1))


def mesh(desc):
    xs = grid_coords(desc)
    return np.meshgrid(*xs, indexing="ij")


def bump_k(desc, k0, centres, sigma=0.05, amp=0.3):
    """k(x) = k0 (1 + amp * sum_i exp(-|x - c_i|^2 / (2 sigma^2))) at the real
    cell centres; returns phi = k^2, flattened x fastest."""
    X = mesh(desc)
    s = np.zeros(X[0].shape)
    for c in centres:
        r2 = sum((X[d] - c[d]) ** 2 for d in range(desc["dim"]))
        s += np.exp(-r2 / (2.0 * sigma * sigma))
    k = k0 * (1.0 + amp * s)
    return flat(k * k)


def point_source(desc, idx, value=1.0):
    """Unit source at one node, idx = (i, j[, k]) 0-based (Sec. 4, MP1)."""
    N = int(np.prod(desc["n"][: desc["dim"]]))
    b = np.zeros(N, dtype=np.complex128)
    n = desc["n"]
    p = idx[0] + n[0] * (idx[1] + (n[1] * idx[2] if desc["dim"] == 3 else 0)) if desc["dim"] >= 2 else idx[0]
    b[p] = value
    return b


def gaussian_sources(desc, centres, sigma=0.02, amp=1.0):
    X = mesh(desc)
    s = np.zeros(X[0].shape)
    for c in centres:
        r2 = sum((X[d] - c[d]) ** 2 for d in range(desc["dim"]))
        s += amp * np.exp(-r2 / (2.0 * sigma * sigma))
    return flat(s).astype(np.complex128)


def shadow_space(N, s, seed):
    """IDR(s) shadow space: s seeded complex-Gaussian columns, orthonormalised
    (QR); returned as an N x s complex array (column-major ready)."""
    g = rng(seed)
    Z = g.standard_normal((N, s)) + 1j * g.standard_normal((N, s))
    Q, _ = np.linalg.qr(Z)
    return np.asfortranarray(Q.astype(np.complex128))


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def c1(mode=0, theta_csg=PI / 8):
    """2D, 128 x 128 cells in total over [-0.25, 1.25]^2 (interior [0,1]^2 and
    an ECS layer of width 0.25 per side, angle pi/6), constant k with
    kh = 0.625, unit point source at node (64, 64), CSG pi/8, 4 levels."""
    n = 128
    d = base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0),
                  theta_csg=theta_csg, csg_mode=mode, levels=4)
    h = 1.5 / n
    k = 0.625 / h
    d["phi_const"] = k * k
    phi = np.full(n * n, k * k)
    return {"name": "c1", "desc": d, "phi": phi, "b": point_source(d, (64, 64)), "k0": k,
            "method": "bicgstab", "tol": 1e-8}


def c1_paper():
    """The paper's multigrid-component setting (Sec. 6.1): 128 interior cells
    plus 2 x 32 layer cells per axis (192^2), k = 80, point source at the centre."""
    n = 192
    d = base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0), levels=4)
    k = 80.0
    phi = np.full(n * n, k * k)
    return {"name": "c1_paper", "desc": d, "phi": phi, "b": point_source(d, (96, 96)), "k0": k,
            "method": "bicgstab", "tol": 1e-8}


def mp1(k=160.0, n_int=256, layers=True, theta_csg=None, levels=6, smoother=1, coarse_op=1):
    """Model problem 1 (Sec. 4, eq. (MP1)) as in Table MP1: the unit square
    with n_int interior cells per axis (h = 1/n_int), constant k, unit point
    source at the cell just past the centre (a cell-centred grid has no centre
    node).  layers: ECS layers of n_int/4 cells (width 0.25, angle pi/6) on
    every side; else first-order Sommerfeld sides (wave number k) on the bare
    square.  CSG angle pi/28 (layers) or -pi/28 (Sommerfeld), the table's; the
    paper's multigrid by default: ILU(0) V(0,1) on Galerkin coarse
    operators, relaxation 1."""
    if layers:
        nl = n_int // 4
        n = n_int + 2 * nl
        lo, hi = -nl / n_int, 1.0 + nl / n_int
        th = PI / 28 if theta_csg is None else theta_csg
        d = base_desc(2, (n, n), (lo, lo), (hi, hi), (0.0, 0.0), (1.0, 1.0), theta_csg=th, levels=levels,
                      nu1=0, omega=1.0, coarse_op=coarse_op, smoother=smoother)
    else:
        n = n_int
        th = -PI / 28 if theta_csg is None else theta_csg
        d = base_desc(2, (n, n), (0.0, 0.0), (1.0, 1.0), (0.0, 0.0), (1.0, 1.0), theta_csg=th, levels=levels,
                      nu1=0, omega=1.0, coarse_op=coarse_op, smoother=smoother, bc=[[1, 1], [1, 1]], k_bc=k)
    phi = np.full(n * n, k * k)
    return {"name": "mp1", "desc": d, "phi": phi, "b": point_source(d, (n // 2, n // 2)), "k0": k,
            "method": "bicgstab", "tol": 1e-6}


def c2(n=1024, levels=8, seed=2):
    """2D n x n (default 1024^2) over the C1 geometry, k0 at 10 points per
    wavelength, k(x) = k0 (1 + 0.3 sum of 8 Gaussian bumps of width 0.05 with
    centres uniform in [0.15, 0.85]^2), unit point source at (n/2, n/2)."""
    d = base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0), levels=levels)
    h = 1.5 / n
    k0 = 2 * PI / (10 * h)
    cen = rng(seed).uniform(0.15, 0.85, size=(8, 2))
    phi = bump_k(d, k0, cen)
    return {"name": "c2", "desc": d, "phi": phi, "b": point_source(d, (n // 2, n // 2)), "k0": k0,
            "method": "bicgstab", "tol": 1e-8}


def c3(n=128, layer=16, seed=3, method="idr", s=4):
    """3D n^3 (default 128^3) with `layer` ECS cells on all six faces (interior
    [0,1]^3 of n - 2*layer cells), k0 at 8 points per wavelength with the bump
    law of c2 (8 bumps, seed 3), unit point source at (n/2,n/2,n/2) plus 4
    unit sources at seeded uniform interior nodes; 5 levels for 128^3."""
    ni = n - 2 * layer
    h = 1.0 / ni
    lo, hi = -layer * h, 1.0 + layer * h
    levels = 0
    d = base_desc(3, (n, n, n), (lo,) * 3, (hi,) * 3, (0.0,) * 3, (1.0,) * 3, levels=levels)
    k0 = 2 * PI / (8 * h)
    g = rng(seed)
    cen = g.uniform(0.15, 0.85, size=(8, 3))
    phi = bump_k(d, k0, cen)
    b = point_source(d, (n // 2, n // 2, n // 2))
    for _ in range(4):
        idx = g.integers(layer, n - layer, size=3)
        b += point_source(d, tuple(int(v) for v in idx))
    out = {"name": "c3", "desc": d, "phi": phi, "b": b, "k0": k0, "method": method, "tol": 1e-8, "s": s}
    if method == "idr":
        out["P"] = shadow_space(n ** 3, s, 1003)
    return out


def c4(count=64, seed=4, sides=(256, 384, 512, 768, 1024)):
    """Batched 2D: `count` independent problems, side uniform from `sides`
    (C1 geometry), points per wavelength uniform in [5, 12], bump wave number
    of c2 with per-problem seeded centres, 1-4 Gaussian sources (sigma 0.02)
    with centres uniform in [0.1, 0.9]^2, auto levels."""
    g = rng(seed)
    probs = []
    for q in range(count):
        n = int(g.choice(sides))
        ppw = g.uniform(5.0, 12.0)
        d = base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0), levels=0)
        h = 1.5 / n
        k0 = 2 * PI / (ppw * h)
        cen = g.uniform(0.15, 0.85, size=(8, 2))
        phi = bump_k(d, k0, cen)
        ns = int(g.integers(1, 5))
        src = g.uniform(0.1, 0.9, size=(ns, 2))
        b = gaussian_sources(d, src)
        probs.append({"name": "c4_%d" % q, "desc": d, "phi": phi, "b": b, "k0": k0, "ppw": ppw,
                      "method": "bicgstab", "tol": 1e-8})
    return probs


def mp_grid(n_int, n_lay, r, theta_csg=PI / 8, levels=0, bc="ecs", k=0.0):
    """The grid of the paper's model problems 2 and 3 (Sec. 4, eq. (BC)): the
    square (0, r)^2 with n_int cells of width h = r / n_int per axis,
    homogeneous Dirichlet on the south and west edges (x = 0, y = 0: no layer,
    a = lo = 0), and on the north and east edges either an ECS layer of n_lay
    cells (bc "ecs") or the Sommerfeld condition du/dn = -i k u (bc
    "sommerfeld", no layer)."""
    h = r / n_int
    if bc == "sommerfeld":
        return base_desc(2, (n_int, n_int), (0.0, 0.0), (r, r), (0.0, 0.0), (r, r), theta_csg=theta_csg,
                         levels=levels, bc=[[0, 1], [0, 1]], k_bc=k)
    n = n_int + n_lay
    hi = r + n_lay * h
    return base_desc(2, (n, n), (0.0, 0.0), (hi, hi), (0.0, 0.0), (r, r), theta_csg=theta_csg, levels=levels)


def mp2(nu=7.0, k=2.0, n_int=384, n_lay=128, r=50.0, theta_csg=PI / 8, levels=0, bc="ecs"):
    """Model problem 2 (Sec. 4, eq. (MP2)): phi = nu (e^{-x^2} + e^{-y^2}) + k^2,
    chi = e^{-(x^2 + y^2)}, on the mp_grid; the paper's sizes are 384 interior
    + 128 layer cells for r = 50 (nu = 7, k = 2 and nu = 1, k = 4).  phi and
    chi are sampled at the real cell centres (layer cells included)."""
    d = mp_grid(n_int, n_lay, r, theta_csg, levels, bc, k)
    X, Y = mesh(d)
    phi = flat(nu * (np.exp(-X * X) + np.exp(-Y * Y)) + k * k)
    b = flat(np.exp(-(X * X + Y * Y))).astype(np.complex128)
    return {"name": "mp2", "desc": d, "phi": phi, "b": b, "k0": k, "nu": nu, "r": r,
            "method": "bicgstab", "tol": 1e-8}


def mp3(r=90.0, k=2.0, n_int=1024, n_lay=256, theta_csg=PI / 8, levels=0, bc="ecs"):
    """Model problem 3 (Sec. 4, eq. (MP3)): phi = 1/x + 1/y + k^2, chi =
    e^{-(x^2 + y^2)}, on the mp_grid; the paper's sizes are 1024 interior +
    256 layer cells for r = 90, k = 2 (2048 + 512 for r = 150, k = 4).  The
    cell centres never reach the singularity at the origin: the largest phi
    is at the first centre (h/2, h/2), as in the paper's mesh-width bound."""
    d = mp_grid(n_int, n_lay, r, theta_csg, levels, bc, k)
    X, Y = mesh(d)
    phi = flat(1.0 / X + 1.0 / Y + k * k)
    b = flat(np.exp(-(X * X + Y * Y))).astype(np.complex128)
    return {"name": "mp3", "desc": d, "phi": phi, "b": b, "k0": k, "r": r, "method": "bicgstab", "tol": 1e-8}


def mp_max_mesh_width(problem, k, nu=0.0):
    """Largest mesh width with kh < 0.625 at the largest discrete wave number
    (Sec. 6.2): MP2 takes phi's supremum at the origin, 2 nu + k^2; MP3 takes
    phi at the first cell centre (h/2, h/2), 4/h + k^2, which gives the
    quadratic k^2 h^2 + 4 h - 0.625^2 = 0."""
    c = 0.625
    if problem == "mp2":
        return c / math.sqrt(2.0 * nu + k * k)
    return (-4.0 + math.sqrt(16.0 + 4.0 * k * k * c * c)) / (2.0 * k * k)


def serving_request(g, frac3d=0.25):
    """One request of the serving mix: 75% 2D with side in {256, 320, ...,
    2048}, 25% 3D with side in {64, 96, 128, 160} and layers of side/8;
    points per wavelength uniform in [8, 12]; bump k(x); 1-4 Gaussian sources."""
    if g.uniform() < frac3d:
        n = int(g.choice([64, 96, 128, 160]))
        layer = n // 8
        ni = n - 2 * layer
        h = 1.0 / ni
        lo, hi = -layer * h, 1.0 + layer * h
        d = base_desc(3, (n, n, n), (lo,) * 3, (hi,) * 3, (0.0,) * 3, (1.0,) * 3)
        dim = 3
    else:
        n = int(g.choice(np.arange(256, 2049, 64)))
        d = base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0))
        h = 1.5 / n
        dim = 2
    ppw = g.uniform(8.0, 12.0)
    k0 = 2 * PI / (ppw * h)
    cen = g.uniform(0.15, 0.85, size=(8, dim))
    phi = bump_k(d, k0, cen)
    ns = int(g.integers(1, 5))
    src = g.uniform(0.1, 0.9, size=(ns, dim))
    b = gaussian_sources(d, src)
    return {"desc": d, "phi": phi, "b": b, "k0": k0, "ppw": ppw, "method": "bicgstab", "tol": 1e-8}


def poisson_arrivals(rate, count, seed):
    """Arrival times (s) of a seeded Poisson stream."""
    g = rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, size=count))
