"""ctypes binding of the CPU FP64 oracle (hh_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the cpu_baseline leg of bench.py, never by the product package.  It shares no
code with the HIP path; both receive the same seeded inputs from
paper_0912_0180_amd.workloads, which holds no arithmetic of the method.

Vectors are numpy complex128 arrays, x fastest (index i + nx*(j + ny*k)).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hh_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99"]

OK, ERR_ARG, ERR_NOCONV, ERR_BREAKDOWN, ERR_NONFINITE = 0, -1, -4, -5, -6


def build(verbose=False):
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    cmd = ["gcc"] + GCC_FLAGS + ["-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB


class _Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("s", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_matvec", ctypes.c_int), ("max_restarts", ctypes.c_int), ("x0_given", ctypes.c_int),
                ("P", ctypes.c_void_p), ("history", ctypes.c_void_p), ("history_len", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("matvecs", ctypes.c_int), ("iterations", ctypes.c_int),
                ("restarts", ctypes.c_int), ("rel_res_recurrence", ctypes.c_double),
                ("rel_res_true", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P, D, I = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
        L.og_create.restype = P
        L.og_create.argtypes = [I, P, P, P, P, P, D, D, I, I, I, I, I, D, P, D, D, I, P, D, I, I]
        L.og_free.argtypes = [P]
        L.og_levels.argtypes = [P]
        L.og_level_dims.argtypes = [P, I, P]
        L.og_coarse_size.restype = ctypes.c_long
        L.og_coarse_size.argtypes = [P]
        L.og_coeffs.argtypes = [P, I, I, I, P]
        L.og_phi.argtypes = [P, I, P]
        L.og_coarse_inverse.argtypes = [P, P]
        L.og_galerkin.argtypes = [P, I, P]
        L.og_ilu.argtypes = [P, I, P]
        L.og_ilu_sweep.argtypes = [P, I, P, P]
        L.og_apply.argtypes = [P, I, I, P, P]
        L.og_vcycle.argtypes = [P, P, P]
        L.og_restrict.argtypes = [P, I, P, P]
        L.og_prolong.argtypes = [P, I, P, P]
        L.og_jacobi.argtypes = [P, I, P, P]
        L.og_coarse_solve.argtypes = [P, P, P]
        L.og_dotc.argtypes = [P, P, ctypes.c_long, P]
        L.og_nrm2.restype = D
        L.og_nrm2.argtypes = [P, ctypes.c_long]
        L.og_solve.argtypes = [P, P, P, P, P]
        L.og_num_threads.restype = I
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(x):
    return np.ascontiguousarray(x, dtype=np.complex128)


def _three(v, fill):
    v = list(v)
    return v + [fill] * (3 - len(v))


class Grid:
    """One discretised problem: geometry, coefficients of H (ECS) and M (CSG)
    on every level, coarse phi, the explicit coarsest inverse.

    desc keys (same meaning as the library's grid descriptor): dim, n, lo, hi,
    a, b, theta_ecs, theta_csg, csg_mode (0 uniform CSG, 1 interior CSG, 2
    CSL), centering (0 cell, 1 vertex), levels (0 auto), nu1, nu2, omega,
    csl_shift ([re, im] of beta^2 for the CSL), contour_steps (ECS contour
    parts, 0/1 linear), bc ([[lo, hi]] per axis, 1 = Sommerfeld), k_bc (its
    wave number), coarse_op (0 rediscretised coarse operators, 1 Galerkin,
    2D only), smoother (0 weighted Jacobi, 1 ILU(0): 2D, cell-centred,
    nu1 = 0, omega its relaxation factor); phi is the real array k(x)^2 on the finest grid (shape
    prod(n)), or phi_const."""

    def __init__(self, desc, phi=None):
        L = lib()
        d = dict(desc)
        dim = int(d["dim"])
        n = [int(v) for v in d["n"]][:dim]
        N = int(np.prod(n))
        if phi is None:
            phi = d.get("phi")
        if phi is None:
            phi = np.full(N, float(d.get("phi_const", 0.0)))
        phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
        assert phi.size == N, (phi.size, N)
        bc = np.zeros(6, dtype=np.int32)
        for ax, sides in enumerate(d.get("bc", [])[:dim]):
            bc[2 * ax], bc[2 * ax + 1] = int(sides[0]), int(sides[1])
        self._keep = [np.array(_three(n, 1), dtype=np.int32),
                      np.array(_three(d["lo"], 0.0)), np.array(_three(d["hi"], 1.0)),
                      np.array(_three(d["a"], 0.0)), np.array(_three(d["b"], 1.0)), phi, bc]
        ni, lo, hi, a, b, _, _ = self._keep
        shift = d.get("csl_shift", [0.0, 0.0])
        self.h = L.og_create(dim, _ptr(ni), _ptr(lo), _ptr(hi), _ptr(a), _ptr(b),
                             float(d.get("theta_ecs", np.pi / 6)), float(d.get("theta_csg", np.pi / 8)),
                             int(d.get("csg_mode", 0)), int(d.get("centering", 0)), int(d.get("levels", 0)),
                             int(d.get("nu1", 1)), int(d.get("nu2", 1)), float(d.get("omega", 0.8)), _ptr(phi),
                             float(shift[0]), float(shift[1]), int(d.get("contour_steps", 0)), _ptr(bc),
                             float(d.get("k_bc", 0.0)), int(d.get("coarse_op", 0)), int(d.get("smoother", 0)))
        if not self.h:
            raise ValueError("oracle rejected the grid description")
        self.dim = dim
        self.n = n
        self.N = N
        self.nlev = L.og_levels(self.h)
        self.Nc = int(L.og_coarse_size(self.h))

    def __del__(self):
        if getattr(self, "h", None):
            lib().og_free(self.h)
            self.h = None

    def level_dims(self, lev):
        out = np.zeros(3, dtype=np.int32)
        lib().og_level_dims(self.h, lev, _ptr(out))
        return [int(v) for v in out]

    def level_size(self, lev):
        return int(np.prod(self.level_dims(lev)))

    def coeffs(self, lev, axis, which):
        """which in {'aH','cH','dH','aM','cM','dM'}"""
        w = ["aH", "cH", "dH", "aM", "cM", "dM"].index(which)
        n = self.level_dims(lev)[axis]
        out = np.zeros(n, dtype=np.complex128)
        rc = lib().og_coeffs(self.h, lev, axis, w, _ptr(out))
        assert rc == n
        return out

    def phi(self, lev):
        out = np.zeros(self.level_size(lev))
        lib().og_phi(self.h, lev, _ptr(out))
        return out

    def ilu(self, lev):
        """ILU(0) factors of level lev (a smoothing level) as (25, N), in the
        Galerkin stencil layout: rows s < 12 (columns below the diagonal) hold
        L (unit diagonal not stored), s >= 12 hold U; zero off the pattern."""
        N = self.level_size(lev)
        out = np.zeros(25 * N, dtype=np.complex128)
        rc = lib().og_ilu(self.h, lev, _ptr(out))
        if rc != 0:
            raise ValueError("level %d has no ILU(0) factors" % lev)
        return out.reshape(25, N)

    def ilu_sweep(self, lev, f, u):
        """One ILU(0) smoothing sweep on level lev: returns u + omega (LU)^-1 (f - M u)."""
        f = _c128(f)
        u = _c128(u).copy()
        rc = lib().og_ilu_sweep(self.h, lev, _ptr(f), _ptr(u))
        if rc != 0:
            raise ValueError("level %d has no ILU(0) factors" % lev)
        return u

    def galerkin(self, lev):
        """Galerkin stencil of level lev >= 1 as (25, N): row s = (dx+2) + 5(dy+2)
        holds the matrix entries M[p, p + dx + nx*dy], |dx|, |dy| <= 2."""
        N = self.level_size(lev)
        out = np.zeros(25 * N, dtype=np.complex128)
        rc = lib().og_galerkin(self.h, lev, _ptr(out))
        if rc != 0:
            raise ValueError("level %d has no Galerkin stencil" % lev)
        return out.reshape(25, N)

    def coarse_inverse(self):
        out = np.zeros((self.Nc, self.Nc), dtype=np.complex128)
        lib().og_coarse_inverse(self.h, _ptr(out))
        return out

    def apply(self, x, op="H", lev=0):
        x = _c128(x).reshape(-1)
        y = np.empty_like(x)
        lib().og_apply(self.h, 0 if op == "H" else 1, lev, _ptr(x), _ptr(y))
        return y

    def matrix(self, op="H", lev=0):
        """Dense matrix of the operator (column q = A e_q); tiny grids only."""
        N = self.level_size(lev)
        A = np.zeros((N, N), dtype=np.complex128)
        e = np.zeros(N, dtype=np.complex128)
        for q in range(N):
            e[q] = 1.0
            A[:, q] = self.apply(e, op, lev)
            e[q] = 0.0
        return A

    def vcycle(self, f):
        f = _c128(f).reshape(-1)
        u = np.empty_like(f)
        lib().og_vcycle(self.h, _ptr(f), _ptr(u))
        return u

    def restrict(self, r, lev=0):
        r = _c128(r).reshape(-1)
        out = np.empty(self.level_size(lev + 1), dtype=np.complex128)
        lib().og_restrict(self.h, lev, _ptr(r), _ptr(out))
        return out

    def prolong(self, e, lev=0):
        e = _c128(e).reshape(-1)
        out = np.empty(self.level_size(lev), dtype=np.complex128)
        lib().og_prolong(self.h, lev, _ptr(e), _ptr(out))
        return out

    def jacobi(self, f, u, lev=0):
        f = _c128(f).reshape(-1)
        u = _c128(u).reshape(-1).copy()
        lib().og_jacobi(self.h, lev, _ptr(f), _ptr(u))
        return u

    def coarse_solve(self, f):
        f = _c128(f).reshape(-1)
        e = np.empty_like(f)
        lib().og_coarse_solve(self.h, _ptr(f), _ptr(e))
        return e

    def solve(self, b, method="bicgstab", tol=1e-8, max_matvec=10000, max_restarts=3, x0=None,
              s=4, P=None, history=False):
        b = _c128(b).reshape(-1)
        x = np.zeros_like(b) if x0 is None else _c128(x0).reshape(-1).copy()
        o = _Opts()
        o.method = 0 if method == "bicgstab" else 1
        o.s = int(s)
        o.tol = float(tol)
        o.max_matvec = int(max_matvec)
        o.max_restarts = int(max_restarts)
        o.x0_given = 0 if x0 is None else 1
        Pk = None
        if o.method == 1:
            Pk = np.asfortranarray(_c128(P).reshape(self.N, s, order="F")) if P is not None else None
            if Pk is None:
                raise ValueError("IDR(s) needs the shadow space P")
            o.P = Pk.ctypes.data
        hist = np.full(max_matvec, np.nan) if history else None
        if hist is not None:
            o.history = hist.ctypes.data
            o.history_len = max_matvec
        info = _Info()
        lib().og_solve(self.h, ctypes.byref(o), _ptr(b), _ptr(x), ctypes.byref(info))
        res = {"status": info.status, "matvecs": info.matvecs, "iterations": info.iterations,
               "restarts": info.restarts, "rel_res_recurrence": info.rel_res_recurrence,
               "rel_res_true": info.rel_res_true}
        if hist is not None:
            res["history"] = hist[: info.matvecs]
        return x, res


def dotc(x, y):
    x, y = _c128(x).reshape(-1), _c128(y).reshape(-1)
    out = np.zeros(2)
    lib().og_dotc(_ptr(x), _ptr(y), x.size, _ptr(out))
    return complex(out[0], out[1])


def nrm2(x):
    x = _c128(x).reshape(-1)
    return float(lib().og_nrm2(_ptr(x), x.size))


def num_threads():
    return int(lib().og_num_threads())


def select_preconditioner(desc, phi, f, which="csg", start=np.pi / 4, factor=0.8, min_value=1e-3, max_cycles=20,
                          reduction=1e-7, max_steps=30):
    """Sec. 6.2, remark on choosing the CSL and CSG parameters: multigrid alone
    on M u = f (u_k = u_{k-1} + V(f - M u_{k-1}), u_0 = 0) for the candidates
    start, start*factor, ...; a candidate converges when ||f - M u_k||/||f||
    drops below `reduction` within `max_cycles` cycles; the search stops at the
    first that does not and returns the last that did.  which "csg" sets the
    CSG angle (a CSL description becomes uniform CSG), "csl" the shift
    1 + i*value.  Returns (result dict, trace rows (value, cycles or 0, last
    relative residual)).  Stops a candidate early once its residual exceeds
    1e3 or is not finite."""
    d = dict(desc)
    d["csl_shift"] = list(d.get("csl_shift", [0.0, 0.0]))
    if which == "csg":
        d["csg_mode"] = 0 if int(d.get("csg_mode", 0)) == 2 else int(d.get("csg_mode", 0))
    else:
        d["csg_mode"] = 2
    f = _c128(f).reshape(-1)
    fn = nrm2(f)
    value, res, trace = float(start), None, []
    for _ in range(max_steps):
        if abs(value) < min_value:
            break
        if which == "csg":
            d["theta_csg"] = value
        else:
            d["csl_shift"] = [1.0, value]
        g = Grid(d, phi)
        u = np.zeros_like(f)
        r = f.copy()
        cycles, rel = 0, 1.0
        for k in range(1, max_cycles + 1):
            v = g.vcycle(r)
            u = u + v
            r = f - g.apply(u, "M")
            rel = nrm2(r) / fn
            if rel < reduction:
                cycles = k
                break
            if not np.isfinite(rel) or rel > 1e3:
                break
        trace.append((value, cycles, rel))
        if cycles == 0:
            break
        res = {"value": value, "cycles": cycles, "factor": rel ** (1.0 / cycles)}
        value = value * factor
    out = {"status": 0 if res else -4, "tried": len(trace)}
    if res:
        out.update(res)
    return out, np.array(trace, dtype=float).reshape(-1, 3)
