"""The request server through the C ABI: continuous batching of mixed
requests under a device-byte budget.

Each problem's arithmetic depends only on its own data (its tiles, its
reduction trees), so a result computed in the mix must equal the one computed
alone value for value, with the same matvec count.
"""
import math
import time

import numpy as np
import pytest

from paper_0912_0180_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0912_0180_amd import hh
    hh.lib()
    return hh


def small_request(seed, dim, n, method="bicgstab", prec="c64", s=2, zero=False):
    g = np.random.default_rng(seed)
    if dim == 3:
        layer = max(2, n // 8)
        h = 1.0 / (n - 2 * layer)
        lo, hi = -layer * h, 1.0 + layer * h
        d = W.base_desc(3, (n, n, n), (lo,) * 3, (hi,) * 3, (0.0,) * 3, (1.0,) * 3)
    else:
        d = W.base_desc(2, (n, n), (-0.25, -0.25), (1.25, 1.25), (0.0, 0.0), (1.0, 1.0))
        h = 1.5 / n
    ppw = g.uniform(8.0, 12.0)
    k0 = 2 * math.pi / (ppw * h)
    phi = W.bump_k(d, k0, g.uniform(0.15, 0.85, size=(8, dim)))
    b = W.gaussian_sources(d, g.uniform(0.1, 0.9, size=(int(g.integers(1, 5)), dim)))
    if zero:
        b = np.zeros_like(b)
    N = int(np.prod(d["n"][:dim]))
    req = {"desc": d, "phi": phi, "b": b, "method": method, "vcycle_prec": prec, "s": s}
    if method == "idr":
        req["P"] = W.shadow_space(N, s, 5000 + seed)
    return req


MIX = [
    dict(seed=1, dim=2, n=64),
    dict(seed=2, dim=2, n=128),
    dict(seed=3, dim=2, n=96),
    dict(seed=4, dim=2, n=80, prec="c128"),
    dict(seed=5, dim=2, n=64, method="idr", s=2),
    dict(seed=6, dim=3, n=32),
    dict(seed=7, dim=2, n=160),
    dict(seed=8, dim=2, n=64, zero=True),
    dict(seed=9, dim=2, n=112),
    dict(seed=10, dim=3, n=24, method="idr", s=4),
]


def solve_alone(hh, req):
    import torch
    grid = hh.Grid(req["desc"], phi=req["phi"])
    b = torch.from_numpy(np.ascontiguousarray(req["b"].reshape(-1))).to("cuda")
    kw = dict(method=req["method"], vcycle_prec=req["vcycle_prec"], s=req["s"])
    if req["method"] == "idr":
        kw["P"] = hh.shadow_to_device(req["P"])
    x, info = grid.solve(b, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


def submit(hh, sv, req):
    return sv.submit(req["desc"], req["b"], phi=req["phi"], P=req.get("P"), method=req["method"],
                     vcycle_prec=req["vcycle_prec"], s=req["s"])


def wait_all(sv, tickets, limit=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = sv.poll(t)
            if r is not None:
                out[t] = r
        if time.time() - t0 > limit:
            raise AssertionError("server did not finish within %.0f s: %s" % (limit, sv.stats()))
        time.sleep(0.002)
    return out


def test_mix_equals_alone_under_budget(hh_mod):
    hh = hh_mod
    reqs = [small_request(**m) for m in MIX]
    feet = [hh.request_footprint(r["desc"], method=r["method"], vcycle_prec=r["vcycle_prec"], s=r["s"]) for r in reqs]
    budget = int(2.2 * max(feet))            # at most a few requests fit at once
    print("footprints", feet, "budget", budget, flush=True)
    alone = [solve_alone(hh, r) for r in reqs]
    sv = hh.Server(budget=budget, max_slots=3)
    try:
        tickets = [submit(hh, sv, r) for r in reqs]
        res = wait_all(sv, tickets)
        st = sv.stats()
    finally:
        sv.close()
    assert st["submitted"] == len(reqs) and st["completed"] == len(reqs) and st["rejected"] == 0
    assert 0 < st["peak_bytes"] <= budget
    assert st["peak_actual"] <= st["peak_bytes"]
    for q, (t, r) in enumerate(zip(tickets, reqs)):
        x, info = res[t]
        xa, ia = alone[q]
        assert info["status"] == ia["status"] == 0, (q, info, ia)
        assert info["matvecs"] == ia["matvecs"], (q, info["matvecs"], ia["matvecs"])
        assert np.array_equal(x, xa), (q, np.max(np.abs(x - xa)))
        assert info["rel_res_true"] == ia["rel_res_true"]
        if MIX[q].get("zero"):
            assert info["matvecs"] == 0 and not np.any(x)
        else:
            assert info["rel_res_true"] < 1e-8
    # continuous batching: some request was admitted only after another
    # finished, and some ran while another was running
    spans = [(res[t][1]["t_admit"], res[t][1]["t_done"]) for t in tickets]
    assert any(a2 >= d1 for (a1, d1) in spans for (a2, d2) in spans if (a1, d1) != (a2, d2))
    assert any(a1 < d2 and a2 < d1 for i, (a1, d1) in enumerate(spans) for j, (a2, d2) in enumerate(spans) if i < j)


def test_footprint_covers_allocations(hh_mod):
    """peak_actual counts what the solves really hold (hierarchy, work space,
    vectors, plan); one request alone must stay within its footprint."""
    hh = hh_mod
    for m in (dict(seed=11, dim=2, n=256), dict(seed=12, dim=3, n=48, method="idr", s=4)):
        r = small_request(**m)
        foot = hh.request_footprint(r["desc"], method=r["method"], vcycle_prec=r["vcycle_prec"], s=r["s"])
        sv = hh.Server(budget=foot, max_slots=1)
        try:
            t = submit(hh, sv, r)
            res = wait_all(sv, [t])
            st = sv.stats()
        finally:
            sv.close()
        assert res[t][1]["status"] == 0
        assert 0 < st["peak_actual"] <= foot, (st["peak_actual"], foot)
        assert st["peak_actual"] > 0.8 * foot, (st["peak_actual"], foot)


def test_rejections(hh_mod):
    hh = hh_mod
    r = small_request(seed=13, dim=2, n=128)
    foot = hh.request_footprint(r["desc"], method="bicgstab", vcycle_prec="c64")
    sv = hh.Server(budget=foot - 1, max_slots=2)
    try:
        with pytest.raises(hh.HHError) as e:
            submit(hh, sv, r)
        assert e.value.status == -2
        bad = dict(r)
        bad["desc"] = dict(r["desc"], n=(130, 128))       # not divisible by 2^(levels-1)
        bad["desc"]["levels"] = 4
        with pytest.raises(hh.HHError) as e:
            submit(hh, sv, bad)
        assert e.value.status == -1
        with pytest.raises(hh.HHError) as e:
            sv.poll(12345)
        assert e.value.status == -8
        assert sv.stats()["rejected"] == 2
    finally:
        sv.close()


def test_destroy_with_requests_in_flight(hh_mod):
    hh = hh_mod
    sv = hh.Server(max_slots=2)
    for m in MIX[:4]:
        submit(hh, sv, small_request(**m))
    sv.close()          # running and queued requests are dropped; no leak, no hang


def test_server_drift_fallback_matches_alone(hh_mod, monkeypatch):
    """A request whose mixed solve drifts (forced by a 3-matvec stall limit)
    continues in the FP64 group and returns what hh_solve returns for it
    alone; a request in FP64 from the start is unaffected."""
    hh = hh_mod
    monkeypatch.setenv("HH_DRIFT_STALL", "3")
    monkeypatch.setenv("HH_MIXED_STAGE", "0")   # the guard alone, without stage restarts
    req = small_request(seed=32, dim=2, n=128)
    xa, ia = solve_alone(hh, req)
    assert ia["fp64_fallback"] == 1
    small = small_request(seed=31, dim=2, n=96, prec="c128")
    xs, is_ = solve_alone(hh, small)
    sv = hh.Server(max_slots=4)
    try:
        t1 = submit(hh, sv, req)
        t2 = submit(hh, sv, small)
        res = wait_all(sv, [t1, t2])
    finally:
        sv.close()
    x1, i1 = res[t1]
    assert i1["status"] == 0 and i1["fp64_fallback"] == 1 and i1["matvecs"] == ia["matvecs"]
    assert np.array_equal(x1, xa)
    x2, i2 = res[t2]
    assert i2["fp64_fallback"] == 0 and np.array_equal(x2, xs)


def test_full_size_serving_sample(hh_mod, oracle_mod):
    """The serving sample that bench.py measures: its first 16 requests, 2D
    up to 2048^2 and 3D up to 160^3 in mixed precision, through one server
    with 16 slots and the default budget.  Every request must complete with
    status 0 and a true residual below 1e-8, evaluated with the oracle's
    operator."""
    g = W.rng(5)
    reqs = [W.serving_request(g) for _ in range(16)]
    print("serving sample: 16 requests", flush=True)
    sv = hh_mod.Server(budget=0, max_slots=16)
    try:
        tickets = [sv.submit(r["desc"], r["b"], phi=r["phi"], method="bicgstab", vcycle_prec="c64") for r in reqs]
        out = wait_all(sv, tickets, limit=100.0)
    finally:
        sv.close()
    for q, (r, t) in enumerate(zip(reqs, tickets)):
        x, info = out[t]
        assert info["status"] == 0, (q, info)
        o = oracle_mod.Grid(r["desc"], r["phi"])
        res = np.linalg.norm(r["b"] - o.apply(x, "H")) / np.linalg.norm(r["b"])
        assert res < 1e-8, (q, res)
        del o
