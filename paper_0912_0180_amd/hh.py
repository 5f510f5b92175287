"""Python binding of libhh.so (the gfx950 Helmholtz solver), argument
marshalling only: every step of the method runs in the library's HIP kernels.

PyTorch supplies device memory (torch.complex128 / complex64 tensors on
cuda:N) and the current stream.  There is no CPU fallback: if the library is
missing or no GPU is usable, every call raises.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhh.so")

OK, PENDING = 0, 1
ERR = {-1: "HH_ERR_ARG", -2: "HH_ERR_OOM", -3: "HH_ERR_HIP", -4: "HH_ERR_NOCONV", -5: "HH_ERR_BREAKDOWN",
       -6: "HH_ERR_NONFINITE", -7: "HH_ERR_BUSY", -8: "HH_ERR_TICKET"}
C128, C64 = 0, 1
OP_H, OP_M = 0, 1
BICGSTAB, IDR = 0, 1

# every symbol include/hh.h declares
EXPORTS = ["hh_setup_grid", "hh_free_grid", "hh_grid_query", "hh_grid_export", "hh_apply_operator", "hh_vcycle",
           "hh_vcycle_noalloc", "hh_profile_vcycle", "hh_solve", "hh_solve_batch", "hh_server_create", "hh_submit", "hh_poll", "hh_server_destroy",
           "hh_server_query", "hh_request_footprint", "hh_select_preconditioner", "hh_last_error", "hh_version"]


class HHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (ERR.get(status, "?"), status, msg))
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("a", ctypes.c_double * 3), ("b", ctypes.c_double * 3),
                ("theta_ecs", ctypes.c_double), ("theta_csg", ctypes.c_double), ("csg_mode", ctypes.c_int32),
                ("centering", ctypes.c_int32), ("levels", ctypes.c_int32), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("omega", ctypes.c_double), ("phi", ctypes.c_void_p), ("phi_const", ctypes.c_double),
                ("host_only", ctypes.c_int32), ("csl_shift", ctypes.c_double * 2), ("contour_steps", ctypes.c_int32),
                ("bc", (ctypes.c_int32 * 2) * 3), ("k_bc", ctypes.c_double), ("coarse_op", ctypes.c_int32),
                ("smoother", ctypes.c_int32)]


class GridInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("levels", ctypes.c_int32), ("n", (ctypes.c_int32 * 3) * 16),
                ("unknowns", ctypes.c_int64), ("coarse_unknowns", ctypes.c_int32), ("device_bytes", ctypes.c_uint64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("s", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_matvec", ctypes.c_int32), ("max_restarts", ctypes.c_int32), ("vcycle_prec", ctypes.c_int32),
                ("x0_given", ctypes.c_int32), ("idr_P", ctypes.c_void_p), ("history", ctypes.c_void_p),
                ("history_len", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("rel_res_recurrence", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("seconds", ctypes.c_double), ("fp64_fallback", ctypes.c_int32),
                ("stages", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class VcycleProfile(ctypes.Structure):
    _fields_ = [("vcycle_us", ctypes.c_double), ("down_us", ctypes.c_double), ("up_us", ctypes.c_double),
                ("down_shape", ctypes.c_int32), ("up_shape", ctypes.c_int32), ("down_groups", ctypes.c_int32),
                ("up_groups", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SelectOpts(ctypes.Structure):
    _fields_ = [("which", ctypes.c_int32), ("start", ctypes.c_double), ("factor", ctypes.c_double),
                ("min_value", ctypes.c_double), ("max_cycles", ctypes.c_int32), ("reduction", ctypes.c_double),
                ("max_steps", ctypes.c_int32)]


class SelectResult(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("cycles", ctypes.c_int32), ("factor", ctypes.c_double),
                ("tried", ctypes.c_int32), ("status", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32), ("device", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("grid", GridDesc), ("opts", SolveOpts), ("b_host", ctypes.c_void_p), ("x_host", ctypes.c_void_p),
                ("idr_P_host", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("info", SolveInfo), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64), ("bytes_budget", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("actual_in_use", ctypes.c_uint64), ("peak_actual", ctypes.c_uint64),
                ("active_slots", ctypes.c_int32), ("queued", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Loads libhh.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhh.so is not built: run `python -m paper_0912_0180_amd.build` "
                               "(or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        V, P, I = ctypes.c_void_p, ctypes.POINTER, ctypes.c_int32
        L.hh_setup_grid.argtypes = [P(GridDesc), P(V)]
        L.hh_free_grid.argtypes = [V]
        L.hh_grid_query.argtypes = [V, P(GridInfo)]
        L.hh_grid_export.argtypes = [V, I, I, I, V, ctypes.c_size_t]
        L.hh_apply_operator.argtypes = [V, I, I, V, V, V]
        L.hh_vcycle.argtypes = [V, I, V, V, V]
        L.hh_vcycle_noalloc.argtypes = [V, I, V, V, V]
        L.hh_profile_vcycle.argtypes = [V, I, V, V, I, P(VcycleProfile), V]
        L.hh_solve.argtypes = [V, P(SolveOpts), V, V, P(SolveInfo), V]
        L.hh_solve_batch.argtypes = [P(V), I, P(SolveOpts), P(V), P(V), P(SolveInfo), V]
        L.hh_server_create.argtypes = [P(ServerOpts), P(V)]
        L.hh_submit.argtypes = [V, P(Request), P(ctypes.c_uint64)]
        L.hh_poll.argtypes = [V, ctypes.c_uint64, P(Result)]
        L.hh_server_destroy.argtypes = [V]
        L.hh_server_query.argtypes = [V, P(ServerStats)]
        L.hh_request_footprint.argtypes = [P(GridDesc), P(SolveOpts), P(ctypes.c_uint64)]
        L.hh_select_preconditioner.argtypes = [P(GridDesc), P(SelectOpts), V, P(SelectResult), V, V]
        L.hh_last_error.restype = ctypes.c_char_p
        L.hh_version.restype = ctypes.c_char_p
        for name in ["hh_setup_grid", "hh_free_grid", "hh_grid_query", "hh_grid_export", "hh_apply_operator",
                     "hh_vcycle", "hh_vcycle_noalloc", "hh_profile_vcycle", "hh_solve", "hh_solve_batch", "hh_server_create", "hh_submit", "hh_poll",
                     "hh_server_destroy", "hh_server_query", "hh_request_footprint", "hh_select_preconditioner"]:
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def last_error():
    return lib().hh_last_error().decode()


def check(status, allow=(OK,)):
    if status not in allow:
        raise HHError(status, last_error())
    return status


def make_desc(desc, phi=None, host_only=False):
    d = GridDesc()
    dim = int(desc["dim"])
    d.dim = dim
    def pick(key, a, fill):
        v = desc[key]
        return v[a] if a < min(dim, len(v)) else fill

    for a in range(3):
        d.n[a] = int(pick("n", a, 1))
        d.lo[a] = float(pick("lo", a, 0.0))
        d.hi[a] = float(pick("hi", a, 1.0))
        d.a[a] = float(pick("a", a, 0.0))
        d.b[a] = float(pick("b", a, 1.0))
    d.theta_ecs = float(desc.get("theta_ecs", math.pi / 6))
    d.theta_csg = float(desc.get("theta_csg", math.pi / 8))
    d.csg_mode = int(desc.get("csg_mode", 0))
    d.centering = int(desc.get("centering", 0))
    d.levels = int(desc.get("levels", 0))
    d.nu1 = int(desc.get("nu1", 1))
    d.nu2 = int(desc.get("nu2", 1))
    d.omega = float(desc.get("omega", 0.8))
    keep = None
    if phi is not None:
        keep = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
        d.phi = keep.ctypes.data
    else:
        d.phi = None
        d.phi_const = float(desc.get("phi_const", 0.0))
    d.host_only = 1 if host_only else 0
    shift = desc.get("csl_shift", (0.0, 0.0))
    d.csl_shift[0], d.csl_shift[1] = float(shift[0]), float(shift[1])
    d.contour_steps = int(desc.get("contour_steps", 0))
    for a, sides in enumerate(desc.get("bc", [])[:dim]):
        d.bc[a][0], d.bc[a][1] = int(sides[0]), int(sides[1])
    d.k_bc = float(desc.get("k_bc", 0.0))
    d.coarse_op = int(desc.get("coarse_op", 0))
    d.smoother = int(desc.get("smoother", 0))
    return d, keep


def _torch():
    import torch
    return torch


def _stream(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _need(t, dtype, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise TypeError("%s must be a contiguous %s tensor of %d elements" % (name, dtype, n))


class Grid:
    """A discretised problem on the device (hh_setup_grid)."""

    def __init__(self, desc, phi=None, host_only=False):
        L = lib()
        d, keep = make_desc(desc, phi if phi is not None else desc.get("phi"), host_only)
        h = ctypes.c_void_p()
        check(L.hh_setup_grid(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.desc = dict(desc)
        info = GridInfo()
        check(L.hh_grid_query(self.h, ctypes.byref(info)))
        self.dim = info.dim
        self.levels = info.levels
        self.level_dims = [[info.n[l][a] for a in range(3)] for l in range(info.levels)]
        self.N = int(info.unknowns)
        self.Nc = int(info.coarse_unknowns)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().hh_free_grid(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self):
        info = GridInfo()
        check(lib().hh_grid_query(self.h, ctypes.byref(info)))
        return int(info.device_bytes)

    def export(self, what, level=0, axis=0):
        """Host copy of a setup array: 'aH','cH','dH','aM','cM','dM' (per axis),
        'phi' (per level), 'Minv' (coarsest inverse), 'galerkin' (the 25 x N
        stencil of a Galerkin level >= 1), 'ilu' (the 25 x N ILU(0) factors of
        a smoothing level)."""
        names = ["aH", "cH", "dH", "aM", "cM", "dM", "phi", "Minv", "galerkin", "ilu"]
        w = names.index(what)
        if w <= 5:
            out = np.zeros(self.level_dims[level][axis], dtype=np.complex128)
        elif w == 6:
            out = np.zeros(int(np.prod(self.level_dims[level])), dtype=np.float64)
        elif w == 7:
            out = np.zeros((self.Nc, self.Nc), dtype=np.complex128)
        else:
            out = np.zeros((25, int(np.prod(self.level_dims[level]))), dtype=np.complex128)
        check(lib().hh_grid_export(self.h, w, level, axis, out.ctypes.data, out.nbytes))
        return out

    def apply(self, x, op="H", prec="c128", out=None):
        torch = _torch()
        dt = torch.complex128 if prec == "c128" else torch.complex64
        _need(x, dt, self.N, "x")
        y = torch.empty_like(x) if out is None else out
        _need(y, dt, self.N, "y")
        check(lib().hh_apply_operator(self.h, OP_H if op == "H" else OP_M, C128 if prec == "c128" else C64,
                                      ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), _stream(x)))
        return y

    def vcycle(self, f, prec="c128", out=None):
        """u = V(f); f complex128; u complex128 (prec 'c128') or complex64 ('c64')."""
        torch = _torch()
        _need(f, torch.complex128, self.N, "f")
        dt = torch.complex128 if prec == "c128" else torch.complex64
        u = torch.empty(self.N, dtype=dt, device=f.device) if out is None else out
        _need(u, dt, self.N, "u")
        check(lib().hh_vcycle(self.h, C128 if prec == "c128" else C64, ctypes.c_void_p(f.data_ptr()),
                              ctypes.c_void_p(u.data_ptr()), _stream(f)))
        return u

    def vcycle_noalloc(self, f, prec="c128", out=None):
        """hh_vcycle_noalloc: the same cycle with the coarse levels in the
        library's static scratch array (nothing allocated by the call)."""
        torch = _torch()
        _need(f, torch.complex128, self.N, "f")
        dt = torch.complex128 if prec == "c128" else torch.complex64
        u = torch.empty(self.N, dtype=dt, device=f.device) if out is None else out
        _need(u, dt, self.N, "u")
        check(lib().hh_vcycle_noalloc(self.h, C128 if prec == "c128" else C64, ctypes.c_void_p(f.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr()), _stream(f)))
        return u

    def profile_vcycle(self, f, prec="c64", reps=50, out=None):
        """hh_profile_vcycle: average microseconds of one V-cycle and of one
        launch of the finest level's down- and up-leg kernels."""
        torch = _torch()
        _need(f, torch.complex128, self.N, "f")
        dt = torch.complex128 if prec == "c128" else torch.complex64
        u = torch.empty(self.N, dtype=dt, device=f.device) if out is None else out
        _need(u, dt, self.N, "u")
        r = VcycleProfile()
        check(lib().hh_profile_vcycle(self.h, C128 if prec == "c128" else C64, ctypes.c_void_p(f.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr()), int(reps), ctypes.byref(r), _stream(f)))
        return r.as_dict()

    def solve(self, b, x=None, x0_given=False, **kw):
        torch = _torch()
        _need(b, torch.complex128, self.N, "b")
        if x is None:
            x = torch.zeros_like(b)
        _need(x, torch.complex128, self.N, "x")
        o, keep = make_opts(**kw)
        o.x0_given = 1 if x0_given else 0
        info = SolveInfo()
        st = lib().hh_solve(self.h, ctypes.byref(o), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                            ctypes.byref(info), _stream(b))
        check(st, allow=(OK, -4, -5, -6))
        res = info.as_dict()
        if keep.get("hist") is not None:
            res["history"] = keep["hist"][: info.matvecs].copy()
        return x, res


def make_opts(method="bicgstab", tol=1e-8, max_matvec=20000, max_restarts=3, vcycle_prec="c128", s=4, P=None,
              history=False, history_len=20000):
    o = SolveOpts()
    o.method = BICGSTAB if method == "bicgstab" else IDR
    o.s = int(s)
    o.tol = float(tol)
    o.max_matvec = int(max_matvec)
    o.max_restarts = int(max_restarts)
    o.vcycle_prec = C128 if vcycle_prec == "c128" else C64
    o.x0_given = 0
    keep = {}
    if o.method == IDR:
        if P is None:
            raise ValueError("IDR(s) needs the shadow space P (device tensor N x s, column-major)")
        keep["P"] = P
        o.idr_P = P.data_ptr()
    if history:
        h = np.full(history_len, np.nan)
        keep["hist"] = h
        o.history = h.ctypes.data
        o.history_len = history_len
    return o, keep


def solve_batch(grids, bs, xs=None, **kw):
    """Solves len(grids) problems together (hh_solve_batch); same options for all."""
    torch = _torch()
    n = len(grids)
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    opts = (SolveOpts * n)()
    keeps = []
    for q in range(n):
        o, keep = make_opts(**kw)
        opts[q] = o
        keeps.append(keep)
    infos = (SolveInfo * n)()
    G = (ctypes.c_void_p * n)(*[g.h.value for g in grids])
    B = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
    X = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    st = lib().hh_solve_batch(G, n, opts, B, X, infos, _stream(bs[0]))
    check(st, allow=(OK, -4, -5, -6))
    return xs, [infos[q].as_dict() for q in range(n)]


def select_preconditioner(desc, f, phi=None, which="csg", start=math.pi / 4, factor=0.8, min_value=1e-3,
                          max_cycles=20, reduction=1e-7, max_steps=30):
    """hh_select_preconditioner: the smallest CSG angle (which "csg") or CSL
    imaginary shift (which "csl") of the sequence start * factor^j at which
    multigrid alone still converges; returns (result dict, trace rows)."""
    d, keep = make_desc(desc, phi if phi is not None else desc.get("phi"))
    o = SelectOpts()
    o.which = 0 if which == "csg" else 1
    o.start, o.factor, o.min_value = float(start), float(factor), float(min_value)
    o.max_cycles, o.reduction, o.max_steps = int(max_cycles), float(reduction), int(max_steps)
    r = SelectResult()
    tr = np.zeros(3 * max_steps)
    st = lib().hh_select_preconditioner(ctypes.byref(d), ctypes.byref(o), ctypes.c_void_p(f.data_ptr()),
                                        ctypes.byref(r), tr.ctypes.data_as(ctypes.c_void_p), _stream(f))
    check(st, allow=(OK, -4))
    res = {k: getattr(r, k) for k, _ in r._fields_}
    return res, tr.reshape(-1, 3)[: r.tried].copy()


def shadow_to_device(P, device="cuda"):
    """Column-major N x s complex128 shadow space as a flat device tensor."""
    torch = _torch()
    Pf = np.asfortranarray(P)
    return torch.from_numpy(Pf.reshape(-1, order="F").copy()).to(device)


def request_footprint(desc, **kw):
    """Device bytes the server reserves for one request (hh_request_footprint)."""
    d, _ = make_desc(desc)
    o = SolveOpts()
    o.method = BICGSTAB if kw.get("method", "bicgstab") == "bicgstab" else IDR
    o.s = int(kw.get("s", 4))
    o.tol = float(kw.get("tol", 1e-8))
    o.max_matvec = int(kw.get("max_matvec", 20000))
    o.max_restarts = int(kw.get("max_restarts", 3))
    o.vcycle_prec = C128 if kw.get("vcycle_prec", "c128") == "c128" else C64
    out = ctypes.c_uint64()
    check(lib().hh_request_footprint(ctypes.byref(d), ctypes.byref(o), ctypes.byref(out)))
    return int(out.value)


class Server:
    """Continuous-batching request server (hh_server_*).  Requests carry host
    arrays; results come back as host arrays."""

    def __init__(self, budget=0, max_slots=64, device=0):
        o = ServerOpts()
        o.hbm_budget_bytes = int(budget)
        o.max_slots = int(max_slots)
        o.device = int(device)
        self.h = ctypes.c_void_p()
        check(lib().hh_server_create(ctypes.byref(o), ctypes.byref(self.h)))
        self._keep = {}

    def submit(self, desc, b, phi=None, P=None, method="bicgstab", tol=1e-8, max_matvec=20000, max_restarts=3,
               vcycle_prec="c64", s=4):
        """Queues one solve; b (and P, N x s, for IDR) are complex128 host arrays
        in the grid's layout.  Returns the ticket."""
        r = Request()
        grid, phi_keep = make_desc(desc, phi=phi)
        r.grid = grid
        keep = {"phi": phi_keep}
        o = SolveOpts()
        o.method = BICGSTAB if method == "bicgstab" else IDR
        o.s = int(s)
        o.tol = float(tol)
        o.max_matvec = int(max_matvec)
        o.max_restarts = int(max_restarts)
        o.vcycle_prec = C128 if vcycle_prec == "c128" else C64
        r.opts = o
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.complex128).reshape(-1))
        x = np.zeros_like(bb)
        r.b_host = bb.ctypes.data
        r.x_host = x.ctypes.data
        if o.method == IDR:
            if P is None:
                raise ValueError("IDR(s) needs the shadow space P")
            Pf = np.asfortranarray(np.asarray(P, dtype=np.complex128))
            Pflat = Pf.reshape(-1, order="F").copy()
            keep["P"] = Pflat
            r.idr_P_host = Pflat.ctypes.data
        keep["b"] = bb
        t = ctypes.c_uint64()
        # the library copies b, P and phi before hh_submit returns
        check(lib().hh_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        del keep
        self._keep[t.value] = x
        return int(t.value)

    def poll(self, ticket):
        """None while pending, else (x, result dict)."""
        res = Result()
        st = check(lib().hh_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(res)), allow=(OK, PENDING))
        if st == PENDING:
            return None
        x = self._keep.pop(ticket)
        out = res.info.as_dict()
        out.update(t_submit=res.t_submit, t_admit=res.t_admit, t_done=res.t_done)
        return x, out

    def stats(self):
        st = ServerStats()
        check(lib().hh_server_query(self.h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.h:
            lib().hh_server_destroy(self.h)
            self.h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
