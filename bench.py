"""Benchmark: CSG-multigrid-preconditioned Krylov solves of the ECS Helmholtz
problem on one MI355X.

Headline workload (one step = one whole solve, x0 = 0 -> ||b - Hx||/||b|| < 1e-8):
2D 1024 x 1024 cells over [-0.25, 1.25]^2 (interior [0,1]^2, ECS layers of
width 0.25 at angle pi/6), k0 at 10 points per wavelength,
k(x) = k0 (1 + 0.3 * sum of 8 seeded Gaussian bumps of width 0.05), unit point
source at the centre, CSG angle pi/8, 8 levels, one V(1,1) cycle per
preconditioner application, Bi-CGSTAB.  `value` is solves/s of the
mixed-precision solve (complex-FP32 V-cycle, FP64 Krylov).

Reported beside it: the FP64 solve, V-cycle and operator bandwidths, the
roofline of the dominant bandwidth-bound kernel of the solve (the finest
up-leg of the V-cycle, timed on the same recipe at 4096^2 so its data comes
from HBM), the C1 128^2 and 192^2 solves (microseconds per V-cycle and per
iteration), the 3D 128^3 solves (IDR(4) and Bi-CGSTAB), the 64-problem batched
solve, the serving stream, the paper's model problems, and the CPU oracle on a
bounded sample of the headline solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--no-cpu-baseline]
                    [--roofline-only] [--pmc-probe]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# HBM traffic of the roofline kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs (see the file); valid only while the kernel sources are unchanged
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_vup_finest_2d_4096_pmc.md")
# side of the HBM-resident grid the roofline kernel is measured on: the
# headline recipe at 4x the side, so one launch of the finest up-leg touches
# ~500 MB, twice the 256 MB Infinity Cache
ROOFLINE_N = 4096
# finest levels of at least this many unknowns run the streaming legs
STREAM_MIN = 8 << 20
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0912_0180_amd", "csrc", f) for f in ("hh_kernels.hpp", "hh_common.h")]


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary, or None if it is missing or the kernel changed since."""
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "kernel_sources_sha256")):
            k, v = line.strip().strip("`").split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def vcycle_bytes(g, fp32):
    """Algorithmic bytes of one fused V(1,1) cycle: every field read or
    written once per fused pass at its storage precision (level-0 input is the
    FP64 Krylov vector, read by the down-leg and again by the up-leg)."""
    dims = g.level_dims
    d = g.dim
    cb = 8 if fp32 else 16
    pb = 4 if fp32 else 8
    total = 0
    for l in range(g.levels - 1):
        N = int(np.prod(dims[l][:d]))
        Nc = N // (2 ** d)
        fin = 16 if l == 0 else cb
        down = N * (fin + pb) + Nc * cb
        up = N * (fin + pb) + Nc * cb + N * cb
        total += down + up
    total += g.Nc * g.Nc * cb + 2 * g.Nc * cb
    return total


def apply_bytes(g):
    """y = H x in FP64 with variable k: x and y (16 B each) and phi (8 B)."""
    return 40 * g.N


def leg_bytes(g, fp32):
    """Algorithmic bytes of one launch of the finest level's fused legs.
    Down-leg: read f (the FP64 Krylov vector, 16 B) and phi, write the
    restricted f of level 1.  Up-leg: read f and phi again and level 1's e,
    write u (the preconditioned vector, c64 in mixed precision)."""
    cb = 8 if fp32 else 16
    pb = 4 if fp32 else 8
    nc = g.N // (2 ** g.dim)
    down = g.N * (16 + pb) + nc * cb
    up = g.N * (16 + pb) + nc * cb + g.N * cb
    return down, up


def time_calls(torch, fn, reps):
    """Average duration of fn() over `reps` back-to-back calls, bracketed by
    HIP events on torch's current stream (the stream the kernels go to)."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def time_calls_graph(torch, fn, reps):
    """Average duration of fn() over `reps` calls captured in one HIP graph and
    replayed, so per-call host work (argument checks, the ctypes call) does
    not gap the stream; returns (seconds, "graph"), or the eager timing and
    "eager" if capture fails."""
    try:
        fn()
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for _ in range(reps):
                fn()
        gr.replay()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(3):
            gr.replay()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / 1e3 / (3 * reps), "graph"
    except Exception as ex:  # noqa: BLE001 - timing method only
        print("graph capture failed, timing eagerly:", ex, file=sys.stderr, flush=True)
        return time_calls(torch, fn, reps), "eager"


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else None


# --------------------------------------------------------------------------
# 2D 1024^2 (headline)
# --------------------------------------------------------------------------
def bench_c2(args, torch, hh, W, out):
    cfg = W.c2(n=args.n, levels=args.levels)
    t0 = time.perf_counter()
    g = hh.Grid(cfg["desc"], cfg["phi"])
    setup_s = time.perf_counter() - t0
    b = torch.from_numpy(cfg["b"]).to("cuda")
    x = torch.zeros_like(b)

    def solve(prec):
        return g.solve(b, x=x, tol=1e-8, vcycle_prec=prec, max_matvec=20000)

    for _ in range(args.warmup):
        solve("c64")
    torch.cuda.synchronize()
    t = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, info = solve("c64")
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    assert all(i["status"] == 0 and i["rel_res_true"] < 1e-8 for i in infos), infos
    info_m = infos[-1]
    ms_step = elapsed / args.steps * 1e3
    out.update({
        "metric": "time-to-1e-8 residual & V-cycle HBM GB/s (FP64 vs mixed); solves/s + p99 lat",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 V-cycle + c128 Krylov",
        "data": "synthetic (seeded Gaussian-bump wave number, point source)",
        "config": {"workload": "2D ECS Helmholtz %dx%d, 10 ppw, 8-bump k(x), point source, CSG pi/8, "
                               "%d-level V(1,1), Bi-CGSTAB to 1e-8 (mixed precision)" % (args.n, args.n, g.levels),
                   "unknowns": g.N, "levels": g.levels},
        "time_to_tol_ms_mixed": ms_step,
        "matvecs_mixed": info_m["matvecs"],
        "rel_res_true_mixed": info_m["rel_res_true"],
        "fp64_fallback_mixed": info_m["fp64_fallback"],
        "setup_s": setup_s,
    })
    if args.quick:
        return cfg, g
    solve("c128")
    torch.cuda.synchronize()
    t = time.perf_counter()
    x64, i64 = solve("c128")
    torch.cuda.synchronize()
    out["time_to_tol_ms_fp64"] = (time.perf_counter() - t) * 1e3
    out["matvecs_fp64"] = i64["matvecs"]
    out["rel_res_true_fp64"] = i64["rel_res_true"]
    x64 = x64.clone()
    xm, _ = solve("c64")
    out["rel_err_mixed_vs_fp64"] = float(torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64))
    out["mixed_speedup_vs_fp64"] = out["time_to_tol_ms_fp64"] / ms_step
    f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
    u64 = torch.empty_like(f)
    u32 = torch.empty(g.N, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(f)
    tv64 = time_calls(torch, lambda: g.vcycle(f, "c128", out=u64), 100)
    tv32 = time_calls(torch, lambda: g.vcycle(f, "c64", out=u32), 100)
    th, how = time_calls_graph(torch, lambda: g.apply(f, "H", out=y), 200)
    out["vcycle_us_fp64"] = tv64 * 1e6
    out["vcycle_us_mixed"] = tv32 * 1e6
    out["vcycle_GBps_fp64"] = vcycle_bytes(g, False) / tv64 / 1e9
    out["vcycle_GBps_mixed"] = vcycle_bytes(g, True) / tv32 / 1e9
    ah = apply_bytes(g) / th / 1e9
    out["applyH_us"] = th * 1e6
    out["applyH_GBps"] = ah
    # the finest legs as the timed solve launches them, at this (cache-resident) size
    prof = g.profile_vcycle(f, "c64", reps=100, out=u32)
    db, ub = leg_bytes(g, True)
    out["finest_legs_mixed"] = {"down_us": prof["down_us"], "up_us": prof["up_us"],
                                "down_GBps": db / prof["down_us"] / 1e3, "up_GBps": ub / prof["up_us"] / 1e3,
                                "down_shape": prof["down_shape"], "up_shape": prof["up_shape"],
                                "working_set_MB": (ub + db) / 1e6,
                                "note": "1024^2: the vectors stay in the 256 MB Infinity Cache between launches"}
    return cfg, g


def bench_roofline(args, torch, hh, W, out):
    """The dominant bandwidth-bound kernel of the timed solve, the finest
    up-leg k_vup (prolongation + correction + post-smoothing, FP32 V-cycle,
    FP64 input), measured on the headline recipe at ROOFLINE_N^2 so every
    launch streams from HBM: HIP events on the launch stream around 100
    back-to-back launches (hh_profile_vcycle), algorithmic bytes from
    leg_bytes.  The finest down-leg and the whole V-cycle are reported beside
    it, in both precisions."""
    n = args.roofline_n
    cfg = W.c2(n=n, levels=int(round(np.log2(n))) - 2)
    g = hh.Grid(cfg["desc"], cfg["phi"])
    f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
    res = {}
    for prec in ("c64", "c128"):
        u = torch.empty(g.N, dtype=torch.complex64 if prec == "c64" else torch.complex128, device="cuda")
        prof = g.profile_vcycle(f, prec, reps=100, out=u)
        db, ub = leg_bytes(g, prec == "c64")
        vb = vcycle_bytes(g, prec == "c64")
        res[prec] = {"down_us": prof["down_us"], "up_us": prof["up_us"], "vcycle_us": prof["vcycle_us"],
                     "down_GBps": db / prof["down_us"] / 1e3, "up_GBps": ub / prof["up_us"] / 1e3,
                     "vcycle_GBps": vb / prof["vcycle_us"] / 1e3,
                     "down_shape": prof["down_shape"], "up_shape": prof["up_shape"],
                     "up_groups": prof["up_groups"], "down_groups": prof["down_groups"]}
        del u
    m = res["c64"]
    _, ub = leg_bytes(g, True)
    ach = ub / m["up_us"] / 1e3
    out["roofline"] = {
        "bound": "hbm",
        "kernel": "hh::k_vup<2, float, double2, float2, %d, %s> (finest-level fused up-leg of the FP32 V-cycle: "
                  "bilinear prolongation + correction + weighted-Jacobi post-smoothing; hh_solve launches it twice "
                  "per Bi-CGSTAB iteration, in the streaming form (non-temporal per-point accesses) on finest "
                  "levels of at least 8M unknowns and in the plain form below, shape %d at 1024^2)"
                  % (m["up_shape"], "true" if g.N >= STREAM_MIN else "false",
                     out.get("finest_legs_mixed", {}).get("up_shape", -1)),
        "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS,
        "traffic": measured_traffic(), "bytes_per_unknown": 30, "unknowns_per_launch": g.N,
        "algorithmic_bytes_per_launch": ub, "launch_us": m["up_us"],
        "working_set": "2D %d^2 (headline recipe at 4x the side): %.0f MB read and written per launch, "
                       "beyond the 256 MB Infinity Cache" % (n, ub / 1e6),
        "timing": "HIP events on the launch stream around 100 back-to-back launches (hh_profile_vcycle)"}
    out["hbm_resident_%d" % n] = res
    g.close()


# --------------------------------------------------------------------------
# 3D 128^3
# --------------------------------------------------------------------------
def bench_c3(args, torch, hh, W):
    res = {"workload": "3D ECS Helmholtz %d^3, %d-cell layers, 8 ppw, 8-bump k(x), point + 4 sources, "
                       "c64 V-cycle, c128 Krylov" % (args.n3, args.n3 // 8)}
    cfg = W.c3(n=args.n3, layer=args.n3 // 8, method="idr", s=4)
    t0 = time.perf_counter()
    g = hh.Grid(cfg["desc"], cfg["phi"])
    res["setup_s"] = time.perf_counter() - t0
    res["unknowns"] = g.N
    res["levels"] = g.levels
    b = torch.from_numpy(cfg["b"]).to("cuda")
    P = hh.shadow_to_device(cfg["P"])
    x = torch.zeros_like(b)
    runs = [("idr4_mixed", dict(method="idr", s=4, P=P, vcycle_prec="c64")),
            ("bicgstab_mixed", dict(method="bicgstab", vcycle_prec="c64")),
            ("bicgstab_fp64", dict(method="bicgstab", vcycle_prec="c128"))]
    for name, kw in runs:
        g.solve(b, x=x, tol=1e-8, max_matvec=20000, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = g.solve(b, x=x, tol=1e-8, max_matvec=20000, **kw)
        torch.cuda.synchronize()
        res[name] = {"time_to_tol_ms": (time.perf_counter() - t) * 1e3, "matvecs": info["matvecs"],
                     "rel_res_true": info["rel_res_true"], "status": info["status"]}
    f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
    u32 = torch.empty(g.N, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(f)
    tv = time_calls(torch, lambda: g.vcycle(f, "c64", out=u32), 50)
    th, _ = time_calls_graph(torch, lambda: g.apply(f, "H", out=y), 100)
    res["vcycle_us_mixed"] = tv * 1e6
    res["vcycle_GBps_mixed"] = vcycle_bytes(g, True) / tv / 1e9
    res["applyH_GBps"] = apply_bytes(g) / th / 1e9
    g.close()
    return res


# --------------------------------------------------------------------------
# 64 independent 2D problems in one batch
# --------------------------------------------------------------------------
def bench_c4(args, torch, hh, W):
    probs = W.c4(count=args.batch)
    t0 = time.perf_counter()
    grids = [hh.Grid(p["desc"], p["phi"]) for p in probs]
    setup_s = time.perf_counter() - t0
    bs = [torch.from_numpy(p["b"]).to("cuda") for p in probs]
    xs = [torch.zeros_like(b) for b in bs]
    hh.solve_batch(grids, bs, xs=xs, vcycle_prec="c64")       # warm (work spaces)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, infos = hh.solve_batch(grids, bs, xs=xs, vcycle_prec="c64")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    assert all(i["status"] == 0 and i["rel_res_true"] < 1e-8 for i in infos), [i["status"] for i in infos]
    # the same problems one after another
    t = time.perf_counter()
    for g, b, x in zip(grids, bs, xs):
        g.solve(b, x=x, vcycle_prec="c64")
    torch.cuda.synchronize()
    seq = time.perf_counter() - t
    # the same batch with the FP64 V-cycle (the plain method)
    hh.solve_batch(grids, bs, xs=xs, vcycle_prec="c128")
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, infos64 = hh.solve_batch(grids, bs, xs=xs, vcycle_prec="c128")
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t
    assert all(i["status"] == 0 and i["rel_res_true"] < 1e-8 for i in infos64)
    mv = [i["matvecs"] for i in infos]
    mv64 = [i["matvecs"] for i in infos64]
    fb = [q for q, i in enumerate(infos) if i["fp64_fallback"]]
    res = {"workload": "%d independent 2D problems, sides from {256..1024}, 5-12 ppw, bump k(x), 1-4 Gaussian "
                       "sources, auto levels, c64 V-cycle, c128 Bi-CGSTAB, one launch per pass" % len(probs),
           "unknowns_total": int(sum(g.N for g in grids)), "setup_s": setup_s,
           "batched_s": wall, "solves_per_s": len(probs) / wall,
           "batched_fp64_s": wall64, "fp64_solves_per_s": len(probs) / wall64,
           "mixed_speedup_vs_fp64_batched": wall64 / wall,
           "sequential_s": seq, "sequential_solves_per_s": len(probs) / seq, "batch_speedup": seq / wall,
           "matvecs_p50": pct(mv, 50), "matvecs_max": int(max(mv)),
           "matvecs_total_mixed": int(sum(mv)), "matvecs_total_fp64": int(sum(mv64)),
           "fp64_fallbacks": len(fb),
           "fallback_matvecs_mixed": int(sum(mv[q] for q in fb)),
           "fallback_matvecs_fp64_alone": int(sum(mv64[q] for q in fb))}
    for g in grids:
        g.close()
    return res


# --------------------------------------------------------------------------
# serving: the Poisson stream
# --------------------------------------------------------------------------
def serve_stream(hh, reqs, arrivals, slots):
    """Submits reqs at their arrival times (seconds from the start) to one
    server and polls until all are done; returns per-request (x, result)."""
    sv = hh.Server(budget=0, max_slots=slots)
    n = len(reqs)
    tickets = [None] * n
    submit_err = []

    def producer():
        t0 = time.perf_counter()
        try:
            for q, r in enumerate(reqs):
                wait = arrivals[q] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                tickets[q] = sv.submit(r["desc"], r["b"], phi=r["phi"], method="bicgstab", vcycle_prec="c64")
        except Exception as e:       # reported below
            submit_err.append(repr(e))

    th = threading.Thread(target=producer)
    th.start()
    done = {}
    reported = 0
    while len(done) < n and not submit_err:
        for q in range(n):
            if q in done or tickets[q] is None:
                continue
            r = sv.poll(tickets[q])
            if r is not None:
                done[q] = r
        if len(done) >= reported + 100:
            reported = len(done) - len(done) % 100
            print("serving: %d of %d requests done" % (len(done), n), file=sys.stderr, flush=True)
        time.sleep(0.001)
    th.join()
    stats = sv.stats()
    sv.close()
    if submit_err:
        raise RuntimeError("serving submit failed: %s" % submit_err[0])
    return [done[q] for q in range(n)], stats


def stream_summary(reqs, results, first, rate):
    """Latency and load figures over the measured requests results[first:]."""
    meas = results[first:]
    lat = [r[1]["t_done"] - r[1]["t_submit"] for r in meas]
    qwait = [r[1]["t_admit"] - r[1]["t_submit"] for r in meas]
    t_sub = [r[1]["t_submit"] for r in meas]
    t_done = [r[1]["t_done"] for r in meas]
    span_in = max(t_sub) - min(t_sub)
    span_out = max(t_done) - min(t_sub)
    n = len(meas)
    return {"requests_measured": n, "ok": int(sum(r[1]["status"] == 0 for r in meas)),
            "offered_req_per_s": rate, "arrival_req_per_s": (n - 1) / span_in if span_in > 0 else None,
            "achieved_solves_per_s": n / span_out,
            "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99), "latency_max_s": max(lat),
            "queue_wait_p50_s": pct(qwait, 50), "queue_wait_p99_s": pct(qwait, 99),
            "unknowns_measured": int(sum(int(np.prod(q["desc"]["n"][:q["desc"]["dim"]])) for q in reqs[first:])),
            "max_rel_res_true": float(max(r[1]["rel_res_true"] for r in meas)),
            "fp64_fallbacks": int(sum(r[1]["fp64_fallback"] for r in meas))}


def bench_c5(args, torch, hh, W):
    """The serving stream of the workload mix (75% 2D 256-2048^2, 25% 3D
    64-160^3, 8-12 ppw, bump k(x), 1-4 Gaussian sources, mixed-precision
    Bi-CGSTAB to 1e-8), seeded Poisson arrivals:
    (a) at the offered 200 req/s, `serve_warmup` requests then
        `serve_requests` measured ones (arrivals far above capacity: latency
        is mostly queueing);
    (b) below capacity, `serve_low_requests` at `serve_low_rate` req/s.
    Untimed: the measured requests of (a) get their true residual with the
    CPU oracle's operator, in arrival order within `serve_residual_budget_s`
    (all of them at the default size); those up to 512^2 unknowns are solved
    by the oracle (FP64) and compared, smallest first, within
    `serve_oracle_budget_s`."""
    from oracle import oracle as O
    g = W.rng(5)
    nw, nm = args.serve_warmup, args.serve_requests
    reqs = [W.serving_request(g) for _ in range(nw + nm)]
    arrivals = W.poisson_arrivals(args.serve_rate, nw + nm, 55)
    t0 = time.perf_counter()
    results, stats = serve_stream(hh, reqs, arrivals, args.serve_slots)
    wall = time.perf_counter() - t0
    res = {"workload": "Poisson stream of the serving mix: 75%% 2D 256-2048^2, 25%% 3D 64-160^3, 8-12 ppw, bump "
                       "k(x), 1-4 Gaussian sources, mixed-precision Bi-CGSTAB to 1e-8; %d warm-up + %d measured "
                       "requests offered at %.0f req/s" % (nw, nm, args.serve_rate),
           "wall_s": wall, "peak_admitted_bytes": int(stats["peak_bytes"]), "budget_bytes": int(stats["bytes_budget"]),
           "peak_actual_bytes": int(stats["peak_actual"])}
    res.update(stream_summary(reqs, results, nw, args.serve_rate))
    # (b) below capacity
    g2 = W.rng(6)
    low = [W.serving_request(g2) for _ in range(args.serve_low_requests)]
    arr2 = W.poisson_arrivals(args.serve_low_rate, len(low), 66)
    res2, _ = serve_stream(hh, low, arr2, args.serve_slots)
    res["below_capacity"] = stream_summary(low, res2, 0, args.serve_low_rate)
    # untimed checks against the CPU oracle
    trues, errs = [], []
    order = sorted(range(nw, nw + nm), key=lambda q: int(np.prod(reqs[q]["desc"]["n"][:reqs[q]["desc"]["dim"]])))
    eligible = [q for q in order if int(np.prod(reqs[q]["desc"]["n"][:reqs[q]["desc"]["dim"]])) <= 512 * 512]
    t_or = time.perf_counter()
    for q in range(nw, nw + nm):
        if time.perf_counter() - t_or > args.serve_residual_budget_s:
            break
        r = reqs[q]
        o = O.Grid(r["desc"], r["phi"])
        x = results[q][0]
        bb = r["b"].reshape(-1)
        trues.append(float(np.linalg.norm(bb - o.apply(x, "H")) / np.linalg.norm(bb)))
        del o
        if len(trues) % 250 == 0:
            print("serving: %d true residuals checked by the oracle" % len(trues), file=sys.stderr, flush=True)
    t_or = time.perf_counter()
    for q in eligible:
        if time.perf_counter() - t_or > args.serve_oracle_budget_s:
            break
        r = reqs[q]
        o = O.Grid(r["desc"], r["phi"])
        xo, io = o.solve(r["b"], tol=1e-8)
        errs.append(float(np.linalg.norm(results[q][0] - xo) / np.linalg.norm(xo)))
        del o
        print("serving: %d requests solved by the oracle" % len(errs), file=sys.stderr, flush=True)
    res["oracle_true_residual_max"] = max(trues)
    res["oracle_true_residual_checked"] = len(trues)
    res["oracle_solve_eligible"] = len(eligible)
    res["oracle_solve_checked"] = len(errs)
    res["rel_err_vs_oracle_max"] = max(errs) if errs else None
    return res


# The paper's own figures for its model problems with ECS layers and the CSG
# preconditioner (Tables MP2 and MP3, Sec. 6.2; Sommerfeld rows of Table MP2):
# MG-preconditioned matvecs to a relative defect of 1e-6 with one ILU(0)
# V(0,1) Galerkin cycle per matvec, Matlab + mex-C on an 8-core Xeon.  Context
# only: the method here stops at 1e-8 with a V(1,1) weighted-Jacobi cycle on
# rediscretised levels.
PAPER_MP = {
    "mp2_nu7_k2": {"csg_angle": "pi/20", "bicgstab": [68, "31.5 s"], "idr4": [73, "32.1 s"], "idr8": [69, "33.2 s"]},
    "mp2_nu1_k4": {"csg_angle": "pi/26", "bicgstab": [115, "36.0 s"], "idr4": [123, "38.3 s"], "idr8": [114, "37.9 s"]},
    "mp3_r90_k2": {"csg_angle": "pi/17", "bicgstab": [139, "4m49s"], "idr4": [139, "4m30s"], "idr8": [134, "4m48s"]},
    "mp2_nu7_k2_sommerfeld": {"csg_angle": "-pi/20", "bicgstab": [113, "15.8 s"], "idr4": [115, "14.6 s"],
                              "idr8": [115, "16.2 s"]},
}


# Table MP1 (Sec. 6.2): MP1, k = 160, 256 interior points, the paper's
# multigrid (ILU(0) V(0,1), Galerkin), tolerance 1e-6; matvecs and the
# paper's CPU times (Matlab with mex-C, 2009), and the multigrid on the
# preconditioner alone (average factor per cycle, cycles for seven orders)
PAPER_MP1 = {
    "ecs": {"csg_angle": "pi/28", "mg": [0.24, 10], "bicgstab": [58, "9 s"], "idr4": [62, "9.23 s"],
            "idr8": [56, "9.62 s"]},
    "sommerfeld": {"csg_angle": "-pi/28", "mg": [0.24, 10], "bicgstab": [74, "4 s"], "idr4": [70, "3.98 s"],
                   "idr8": [72, "4.40 s"]},
    "ecs_csl": {"csl_shift_printed": "-1-0.2i", "mg": [0.29, 12], "bicgstab": [59, "9.15 s"], "idr4": [62, "9.11 s"],
                "idr8": [60, "9.61 s"]},
    "sommerfeld_csl": {"csl_shift_printed": "-1+0.2i", "mg": [0.31, 12], "bicgstab": [79, "4.75 s"],
                       "idr4": [72, "4 s"], "idr8": [76, "5.35 s"]},
}


# Tables MP2 and MP3 (Sec. 6.2), CSG rows: the multigrid alone (factor,
# cycles) and matvecs of Bi-CGSTAB, IDR(4), IDR(8), as printed
PAPER_MP23 = {
    "mp2_nu7_k2_ecs": {"csg_angle": "pi/20", "mg": [0.19, 9], "bicgstab": 68, "idr4": 73, "idr8": 69},
    "mp2_nu7_k2_sommerfeld": {"csg_angle": "-pi/20", "mg": [0.25, 10], "bicgstab": 113, "idr4": 115, "idr8": 115},
    "mp2_nu1_k4_ecs": {"csg_angle": "pi/26", "mg": [0.43, 18], "bicgstab": 115, "idr4": 123, "idr8": 114},
    "mp2_nu1_k4_sommerfeld": {"csg_angle": "-pi/27", "mg": [0.51, 21], "bicgstab": 161, "idr4": 164, "idr8": 161},
    "mp3_r90_k2_ecs": {"csg_angle": "pi/17", "mg": [0.27, 11], "bicgstab": 139, "idr4": 139, "idr8": 134},
    "mp3_r90_k2_sommerfeld": {"csg_angle": "-pi/17", "mg": [0.41, 16], "bicgstab": 205, "idr4": 207, "idr8": 207},
    "mp3_r150_k4_ecs": {"csg_angle": "pi/17", "mg": [0.31, 13], "bicgstab": 390, "idr4": 387, "idr8": 392},
    "mp3_r150_k4_sommerfeld": {"csg_angle": "-pi/17", "mg": [0.37, 15], "bicgstab": 620, "idr4": 650, "idr8": 652},
}


def bench_paper_tables(args, torch, hh, W):
    """Tables MP1-MP3 in the paper's own multigrid configuration: one ILU(0)
    V(0,1) cycle on Galerkin coarse operators per preconditioner application
    (FP64), Krylov tolerance 1e-6 as in the paper.  MP1 with k = 160 (ECS
    layers on 256 + 2 x 64 cells, CSG pi/28 or the CSL with the printed shift
    -1 - 0.2i; the Sommerfeld condition on 256^2, CSG -pi/28 or CSL
    -1 + 0.2i); MP2 (384 + 128 cells, nu = 7, k = 2 and nu = 1, k = 4) and MP3
    (r = 90, k = 2, 1024 + 256 cells; r = 150, k = 4, 2048 + 512 cells) with
    the tables' CSG angles, layers on the north and east edges or the
    Sommerfeld condition there.  Per row: the multigrid alone as a solver of
    the preconditioner problem, the ILU(0) V-cycle's time, and Bi-CGSTAB,
    IDR(4), IDR(8) (MP3: Bi-CGSTAB, one timed solve)."""
    PI = np.pi
    rows = []
    for bc in ("ecs", "sommerfeld", "ecs_csl", "sommerfeld_csl"):
        def mk(bc=bc):
            c = W.mp1(layers=bc.startswith("ecs"))
            if bc.endswith("_csl"):
                # the CSL preconditioner with beta^2 = 1 -+ 0.2i (printed shift -1 -+ 0.2i)
                d = dict(c["desc"])
                d["csg_mode"] = 2
                d["csl_shift"] = [1.0, 0.2 if bc == "ecs_csl" else -0.2]
                c = dict(c, desc=d)
            return c
        rows.append(("mp1_k160_" + bc, mk, PAPER_MP1[bc], True))
    mp = [("mp2_nu7_k2_ecs", lambda: W.mp2(nu=7.0, k=2.0, theta_csg=PI / 20)),
          ("mp2_nu7_k2_sommerfeld", lambda: W.mp2(nu=7.0, k=2.0, n_lay=0, bc="sommerfeld", theta_csg=-PI / 20)),
          ("mp2_nu1_k4_ecs", lambda: W.mp2(nu=1.0, k=4.0, theta_csg=PI / 26)),
          ("mp2_nu1_k4_sommerfeld", lambda: W.mp2(nu=1.0, k=4.0, n_lay=0, bc="sommerfeld", theta_csg=-PI / 27)),
          ("mp3_r90_k2_ecs", lambda: W.mp3(r=90.0, k=2.0, theta_csg=PI / 17)),
          ("mp3_r90_k2_sommerfeld", lambda: W.mp3(r=90.0, k=2.0, n_lay=0, bc="sommerfeld", theta_csg=-PI / 17)),
          ("mp3_r150_k4_ecs", lambda: W.mp3(r=150.0, k=4.0, n_int=2048, n_lay=512, theta_csg=PI / 17)),
          ("mp3_r150_k4_sommerfeld", lambda: W.mp3(r=150.0, k=4.0, n_int=2048, n_lay=0, bc="sommerfeld", theta_csg=-PI / 17))]
    for name, mk in mp:
        def mk2(mk=mk):
            c = mk()
            d = dict(c["desc"])
            d.update(smoother=1, coarse_op=1, nu1=0, omega=1.0)
            return dict(c, desc=d)
        rows.append((name, mk2, PAPER_MP23[name], name.startswith("mp2")))
    res = {}
    for name, mk, paper, all_methods in rows:
        c = mk()
        g = hh.Grid(c["desc"], c["phi"])
        b = torch.from_numpy(c["b"]).to("cuda")
        x = torch.zeros_like(b)
        row = {"grid": "%dx%d" % (c["desc"]["n"][0], c["desc"]["n"][1]), "levels": g.levels,
               "smoother": "ILU(0) V(0,1), Galerkin", "paper": paper}
        u = torch.empty_like(b)
        row["vcycle_ms"] = time_calls(torch, lambda: g.vcycle(b, "c128", out=u), 10 if all_methods else 3) * 1e3
        # the multigrid alone: u <- u + V(f - M u) until the residual drops by 1e-7
        uu = torch.zeros_like(b)
        r = b.clone()
        r0 = float(torch.linalg.vector_norm(b))
        it = 0
        while float(torch.linalg.vector_norm(r)) > 1e-7 * r0 and it < 60:
            uu += g.vcycle(r, "c128")
            r = b - g.apply(uu, "M")
            it += 1
        row["mg_alone"] = {"cycles": it, "factor": (float(torch.linalg.vector_norm(r)) / r0) ** (1.0 / it)}
        runs = [("bicgstab", dict(method="bicgstab"))]
        if all_methods:
            for sd in (4, 8):
                runs.append(("idr%d" % sd, dict(method="idr", s=sd, P=hh.shadow_to_device(W.shadow_space(g.N, sd, 500 + sd)))))
        for rname, kw in runs:
            if all_methods:
                g.solve(b, x=x, tol=1e-6, vcycle_prec="c128", max_matvec=3000, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = g.solve(b, x=x, tol=1e-6, vcycle_prec="c128", max_matvec=3000, **kw)
            torch.cuda.synchronize()
            row[rname] = {"time_to_tol_ms": (time.perf_counter() - t) * 1e3, "matvecs": info["matvecs"],
                          "rel_res_true": info["rel_res_true"], "status": info["status"]}
        res[name] = row
        g.close()
        print("bench: paper table row %s done" % name, file=sys.stderr, flush=True)
    return res


def bench_c1(args, torch, hh, W):
    """C1: the 128^2 grid (layers included) of Sec. 6.1 with kh = 0.625, CSG
    pi/8 uniform and interior, and the paper-aligned 192^2, k = 80 row, each
    with rediscretised coarse operators, plus the Galerkin rows (C1 with
    V(1,1), the 192^2 row with the paper's V(0,1)); 4 levels, Bi-CGSTAB to 1e-8.  The working set (a few MiB) stays in L2, so
    the row reports microseconds per V-cycle and per iteration (two matvecs)
    rather than a bandwidth fraction."""
    def galerkin(c, nu1):
        d = dict(c["desc"])
        d["coarse_op"], d["nu1"] = 1, nu1
        return dict(c, desc=d)

    cases = [("c1_uniform", lambda: W.c1(mode=0)), ("c1_interior", lambda: W.c1(mode=1)),
             ("c1_paper", lambda: W.c1_paper()),
             # the paper's multigrid configuration (Sec. 6.1): Galerkin coarse
             # operators, and the V(0,1) cycle (weighted Jacobi, not ILU(0))
             ("c1_galerkin", lambda: galerkin(W.c1(mode=0), 1)),
             ("c1_paper_galerkin_v01", lambda: galerkin(W.c1_paper(), 0))]
    res = {}
    for name, mk in cases:
        c = mk()
        g = hh.Grid(c["desc"], c["phi"])
        b = torch.from_numpy(c["b"]).to("cuda")
        x = torch.zeros_like(b)
        f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
        row = {"grid": "%dx%d" % (c["desc"]["n"][0], c["desc"]["n"][1]), "levels": g.levels,
               "csg_mode": ("uniform", "interior")[c["desc"]["csg_mode"]],
               "coarse_op": ("rediscretised", "galerkin")[c["desc"].get("coarse_op", 0)],
               "cycle": "V(%d,1)" % c["desc"].get("nu1", 1)}
        for prec in ("c128", "c64"):
            row["vcycle_us_" + prec] = g.profile_vcycle(f, prec, reps=200)["vcycle_us"]
        for rname, vp in (("bicgstab_fp64", "c128"), ("bicgstab_mixed", "c64")):
            g.solve(b, x=x, tol=1e-8, vcycle_prec=vp)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = g.solve(b, x=x, tol=1e-8, vcycle_prec=vp)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3
            row[rname] = {"time_to_tol_ms": ms, "matvecs": info["matvecs"],
                          "us_per_iteration": ms * 1e3 / max(1, info["matvecs"] / 2),
                          "rel_res_true": info["rel_res_true"], "status": info["status"]}
        res[name] = row
        g.close()
    return res


def bench_c5_long(args, torch, hh, W):
    """The serving stream at length: `serve_long_warmup` + `serve_long_requests`
    requests of the serving mix offered at `serve_long_rate` req/s (below
    capacity, so latency is service, not an ever-growing queue).  Request q is
    generated from its own seed just before it is submitted, and only the
    solutions the oracle checks are kept: every measured request of up to
    512^2 unknowns and a seeded 5% of the rest.  Untimed afterwards, each
    checked request is regenerated from its seed; its true residual is taken
    with the CPU oracle's operator, and those of up to 512^2 unknowns are
    solved by the oracle within `serve_oracle_budget_s` (smallest first)."""
    import concurrent.futures as cf
    from oracle import oracle as O
    nw, nm, rate = args.serve_long_warmup, args.serve_long_requests, args.serve_long_rate
    n = nw + nm
    arrivals = W.poisson_arrivals(rate, n, 57)
    sample5 = W.rng(58).uniform(size=n) < 0.05

    def make(q):
        return W.serving_request(W.rng(7_000_000 + q))

    sv = hh.Server(budget=0, max_slots=args.serve_slots)
    tickets = {}
    sizes = [0] * n
    err = []

    def producer():
        t0 = time.perf_counter()
        try:
            with cf.ThreadPoolExecutor(4) as ex:
                ahead = {q: ex.submit(make, q) for q in range(min(n, 16))}
                for q in range(n):
                    r = ahead.pop(q).result()
                    if q + 16 < n:
                        ahead[q + 16] = ex.submit(make, q + 16)
                    sizes[q] = int(np.prod(r["desc"]["n"][:r["desc"]["dim"]]))
                    wait = arrivals[q] - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                    tickets[q] = sv.submit(r["desc"], r["b"], phi=r["phi"], method="bicgstab", vcycle_prec="c64")
                    del r
        except Exception as e:       # reported below
            err.append(repr(e))

    th = threading.Thread(target=producer)
    t_start = time.perf_counter()
    th.start()
    done, keep_x = {}, {}
    reported = 0
    while len(done) < n and not err:
        for q, tk in dict(tickets).items():
            if q in done:
                continue
            r = sv.poll(tk)
            if r is None:
                continue
            done[q] = r[1]
            if q >= nw and (sizes[q] <= 512 * 512 or sample5[q]):
                keep_x[q] = r[0]
        if len(done) >= reported + 100:
            reported = len(done) - len(done) % 100
            print("serving (long): %d of %d requests done" % (len(done), n), file=sys.stderr, flush=True)
        time.sleep(0.002)
    th.join()
    wall = time.perf_counter() - t_start
    stats = sv.stats()
    sv.close()
    if err:
        raise RuntimeError("serving submit failed: %s" % err[0])
    meas = [done[q] for q in range(nw, n)]
    lat = [r["t_done"] - r["t_submit"] for r in meas]
    qwait = [r["t_admit"] - r["t_submit"] for r in meas]
    t_sub = [r["t_submit"] for r in meas]
    span_in = max(t_sub) - min(t_sub)
    span_out = max(r["t_done"] for r in meas) - min(t_sub)
    res = {"workload": "Poisson stream of the serving mix (as the default serving row), %d warm-up + %d measured "
                       "requests offered at %.1f req/s" % (nw, nm, rate),
           "wall_s": wall, "peak_admitted_bytes": int(stats["peak_bytes"]),
           "requests_measured": nm, "ok": int(sum(r["status"] == 0 for r in meas)),
           "offered_req_per_s": rate, "arrival_req_per_s": (nm - 1) / span_in if span_in > 0 else None,
           "achieved_solves_per_s": nm / span_out,
           "latency_p50_s": pct(lat, 50), "latency_p90_s": pct(lat, 90), "latency_p99_s": pct(lat, 99),
           "latency_max_s": max(lat), "queue_wait_p50_s": pct(qwait, 50), "queue_wait_p99_s": pct(qwait, 99),
           "unknowns_measured": int(sum(sizes[nw:])), "max_rel_res_true": float(max(r["rel_res_true"] for r in meas)),
           "fp64_fallbacks": int(sum(r["fp64_fallback"] for r in meas))}
    # untimed oracle checks of the kept solutions
    trues, errs = [], []
    t_or = time.perf_counter()
    for q in sorted(keep_x):
        if time.perf_counter() - t_or > args.serve_residual_budget_s:
            break
        r = make(q)
        o = O.Grid(r["desc"], r["phi"])
        bb = r["b"].reshape(-1)
        trues.append(float(np.linalg.norm(bb - o.apply(keep_x[q], "H")) / np.linalg.norm(bb)))
        del o
        if len(trues) % 10 == 0:
            print("serving (long): %d true residuals checked by the oracle" % len(trues), file=sys.stderr, flush=True)
    small = sorted((q for q in keep_x if sizes[q] <= 512 * 512), key=lambda q: sizes[q])
    t_or = time.perf_counter()
    for q in small:
        if time.perf_counter() - t_or > args.serve_oracle_budget_s:
            break
        r = make(q)
        xo, _ = O.Grid(r["desc"], r["phi"]).solve(r["b"], tol=1e-8)
        errs.append(float(np.linalg.norm(keep_x[q] - xo) / np.linalg.norm(xo)))
        print("serving (long): %d requests solved by the oracle" % len(errs), file=sys.stderr, flush=True)
    res.update({"oracle_checked": len(trues), "oracle_checked_small": sum(1 for q in keep_x if sizes[q] <= 512 * 512),
                "oracle_true_residual_max": max(trues) if trues else None,
                "oracle_solve_eligible": len(small), "oracle_solve_checked": len(errs),
                "rel_err_vs_oracle_max": max(errs) if errs else None})
    return res


def bench_mp(args, torch, hh, W):
    """The paper's model problems at its sizes: MP2 (nu = 7, k = 2 and nu = 1,
    k = 4; 384 + 128 cells per axis, r = 50), MP3 (r = 90, k = 2; 1024 + 256
    cells) with ECS layers on the north and east edges, and MP2 with
    Sommerfeld edges (384^2, CSG angle -pi/8); Bi-CGSTAB, IDR(4) and IDR(8) to
    1e-8, CSG pi/8, FP64 and mixed V-cycles.  On MP2 (nu = 7) the CSG angle is
    also chosen automatically (multigrid alone within 20 cycles, Sec. 6.2)."""
    probs = [("mp2_nu7_k2", lambda: W.mp2(nu=7.0, k=2.0)), ("mp2_nu1_k4", lambda: W.mp2(nu=1.0, k=4.0)),
             ("mp3_r90_k2", lambda: W.mp3(r=90.0, k=2.0)),
             ("mp2_nu7_k2_sommerfeld", lambda: W.mp2(nu=7.0, k=2.0, n_lay=0, bc="sommerfeld", theta_csg=-np.pi / 8))]
    res = {}
    for name, mk in probs:
        c = mk()
        g = hh.Grid(c["desc"], c["phi"])
        b = torch.from_numpy(c["b"]).to("cuda")
        x = torch.zeros_like(b)
        row = {"grid": "%dx%d" % (c["desc"]["n"][0], c["desc"]["n"][1]), "paper": PAPER_MP[name]}
        runs = [("bicgstab_fp64", dict(method="bicgstab", vcycle_prec="c128")),
                ("bicgstab_mixed", dict(method="bicgstab", vcycle_prec="c64"))]
        for s in (4, 8):
            P = hh.shadow_to_device(W.shadow_space(g.N, s, 3000 + s))
            runs.append(("idr%d_fp64" % s, dict(method="idr", s=s, P=P, vcycle_prec="c128")))
        for rname, kw in runs:
            g.solve(b, x=x, tol=1e-8, max_matvec=20000, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = g.solve(b, x=x, tol=1e-8, max_matvec=20000, **kw)
            torch.cuda.synchronize()
            row[rname] = {"time_to_tol_ms": (time.perf_counter() - t) * 1e3, "matvecs": info["matvecs"],
                          "rel_res_true": info["rel_res_true"], "status": info["status"],
                          "fp64_fallback": info["fp64_fallback"]}
        if name == "mp2_nu7_k2":
            t = time.perf_counter()
            sel, trace = hh.select_preconditioner(c["desc"], b, phi=c["phi"], which="csg", start=np.pi / 4,
                                                  factor=0.8, max_cycles=20)
            sel_s = time.perf_counter() - t
            d2 = dict(c["desc"])
            d2["theta_csg"] = sel["value"]
            g2 = hh.Grid(d2, c["phi"])
            _, i2 = g2.solve(b, x=x, tol=1e-8, vcycle_prec="c128")
            row["selected_csg"] = {"angle": sel["value"], "cycles": sel["cycles"], "candidates": sel["tried"],
                                   "search_s": sel_s, "bicgstab_fp64_matvecs": i2["matvecs"],
                                   "status": i2["status"]}
            g2.close()
        res[name] = row
        g.close()
    return res


def cpu_baseline(args, cfg, out):
    from oracle import oracle as O
    o = O.Grid(cfg["desc"], cfg["phi"])
    m = args.cpu_sample_matvecs
    t = time.perf_counter()
    _, io = o.solve(cfg["b"], tol=1e-8, max_matvec=m, max_restarts=0)
    ts = time.perf_counter() - t
    full_mv = out.get("matvecs_fp64", out["matvecs_mixed"])
    est = ts / io["matvecs"] * full_mv
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out["cpu_baseline"] = {"value": 1.0 / est, "unit": "solves/s", "cores": O.num_threads(), "kind": "oracle",
                           "cpu_model": cpu,
                           "sample": "FP64 oracle Bi-CGSTAB on the headline problem, first %d matvecs in %.1f s, "
                                     "scaled to the %d matvecs of the full FP64 solve" % (io["matvecs"], ts, full_mv)}


def pmc_probe(torch, hh, W, n):
    """Launches for counter runs: the mixed V-cycle profile at n^2 (its 10
    back-to-back launches of the finest up-leg are the roofline kernel's) and
    10 elementwise copies of 512 MiB (the calibration kernel)."""
    cfg = W.c2(n=n, levels=int(round(np.log2(n))) - 2)
    g = hh.Grid(cfg["desc"], cfg["phi"])
    f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
    u = torch.empty(g.N, dtype=torch.complex64, device="cuda")
    prof = g.profile_vcycle(f, "c64", reps=10, out=u)
    # calibration: an elementwise kernel reading and writing 512 MiB, over two
    # buffer pairs in turn so every source was last touched 1 GiB of traffic
    # earlier (beyond L2 and the Infinity Cache)
    n = (512 << 20) // 4
    xs = [torch.ones(n, dtype=torch.int32, device="cuda") for _ in range(2)]
    ys = [torch.empty_like(xs[0]) for _ in range(2)]
    for i in range(10):
        torch.mul(xs[i % 2], 1, out=ys[i % 2])
    torch.cuda.synchronize()
    print("pmc probe: 10 x finest up-leg (shape %d) on %d unknowns, 10 x elementwise copy of %d bytes"
          % (prof["up_shape"], g.N, 4 * n), flush=True)


def legs_probe(torch, hh, W):
    """Launches for SQ counter runs on the V-cycle legs: hh_profile_vcycle in
    complex float (20 cycles, 20 launches of each finest leg) on the 3D 128^3
    grid (16-cell layers) and on the 2D 1024^2 headline grid."""
    for name, mk in (("3d128", lambda: W.c3(n=128, layer=16, method="bicgstab")), ("2d1024", lambda: W.c2())):
        c = mk()
        g = hh.Grid(c["desc"], c["phi"])
        f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
        u = torch.empty(g.N, dtype=torch.complex64, device="cuda")
        r = g.profile_vcycle(f, "c64", reps=20, out=u)
        print("legs probe %s: down shape %d %.2f us, up shape %d %.2f us, V-cycle %.1f us"
              % (name, r["down_shape"], r["down_us"], r["up_shape"], r["up_us"], r["vcycle_us"]), flush=True)
        g.close()


def ilu_probe(torch, hh, W):
    """Launches for a kernel trace of the paper's multigrid: 5 FP64 ILU(0)
    V(0,1) cycles on Galerkin operators for Table MP1's problem with ECS layers
    (384^2) and Table MP3's (r = 90, k = 2) with ECS layers (1280^2) and with
    the Sommerfeld condition (1024^2), each printing its mean cycle time."""
    PI = np.pi
    cases = (("mp1_k160_ecs", lambda: W.mp1(layers=True)),
             ("mp3_r90_k2_ecs", lambda: W.mp3(r=90.0, k=2.0, theta_csg=PI / 17)),
             ("mp3_r90_k2_sommerfeld", lambda: W.mp3(r=90.0, k=2.0, n_lay=0, bc="sommerfeld", theta_csg=-PI / 17)))
    for name, mk in cases:
        c = mk()
        d = dict(c["desc"])
        d.update(smoother=1, coarse_op=1, nu1=0, omega=1.0)
        g = hh.Grid(d, c["phi"])
        b = torch.from_numpy(c["b"]).to("cuda")
        u = torch.empty_like(b)
        ms = time_calls(torch, lambda: g.vcycle(b, "c128", out=u), 5) * 1e3
        print("ilu probe %s: %dx%d, %d levels, V-cycle %.2f ms" % (name, d["n"][0], d["n"][1], g.levels, ms), flush=True)
        g.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--n3", type=int, default=128)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-warmup", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-low-rate", type=float, default=3.0)
    ap.add_argument("--serve-low-requests", type=int, default=80)
    ap.add_argument("--serve-oracle-budget-s", type=float, default=90.0)
    ap.add_argument("--serve-residual-budget-s", type=float, default=300.0,
                    help="seconds for the oracle's true-residual checks of the measured requests (in arrival order)")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-long", action="store_true",
                    help="also serve the long stream (serve-long-warmup + serve-long-requests at serve-long-rate)")
    ap.add_argument("--serve-long-requests", type=int, default=2000)
    ap.add_argument("--serve-long-warmup", type=int, default=200)
    ap.add_argument("--serve-long-rate", type=float, default=10.0)
    ap.add_argument("--skip", default="", help="comma list of c1,c3,c4,c5,mp to skip")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-matvecs", type=int, default=300)
    ap.add_argument("--quick", action="store_true", help="headline solve only")
    ap.add_argument("--pmc-probe", action="store_true", help="only the launches the counter runs read")
    ap.add_argument("--legs-probe", action="store_true", help="only the V-cycle leg launches of the SQ counter runs")
    ap.add_argument("--ilu-probe", action="store_true", help="only ILU(0) V-cycles of Tables MP1 and MP3 (kernel trace)")
    ap.add_argument("--roofline-n", type=int, default=ROOFLINE_N, help="side of the HBM-resident roofline grid")
    ap.add_argument("--roofline-only", action="store_true", help="only the roofline measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (multi-GPU sharding is described, not "
              "implemented, and is not part of the measured path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0912_0180_amd import hh
    from paper_0912_0180_amd import workloads as W

    torch.cuda.set_device(0)
    if args.pmc_probe:
        pmc_probe(torch, hh, W, args.roofline_n)
        return
    if args.legs_probe:
        legs_probe(torch, hh, W)
        return
    if args.ilu_probe:
        ilu_probe(torch, hh, W)
        return
    out = {}
    if args.roofline_only:
        bench_roofline(args, torch, hh, W, out)
        print(json.dumps(out), flush=True)
        return
    skip = set(s for s in args.skip.split(",") if s)
    cfg, g = bench_c2(args, torch, hh, W, out)
    g.close()
    if not args.quick:
        print("bench: roofline", file=sys.stderr, flush=True)
        bench_roofline(args, torch, hh, W, out)
    if not args.quick:
        if "c1" not in skip:
            print("bench: c1", file=sys.stderr, flush=True)
            out["c1"] = bench_c1(args, torch, hh, W)
        if "c3" not in skip:
            print("bench: c3", file=sys.stderr, flush=True)
            out["c3"] = bench_c3(args, torch, hh, W)
        if "c4" not in skip:
            print("bench: c4", file=sys.stderr, flush=True)
            out["c4"] = bench_c4(args, torch, hh, W)
        if "c5" not in skip:
            print("bench: c5", file=sys.stderr, flush=True)
            out["serving"] = bench_c5(args, torch, hh, W)
        if "mp" not in skip:
            print("bench: mp2/mp3", file=sys.stderr, flush=True)
            out["model_problems"] = bench_mp(args, torch, hh, W)
            print("bench: paper tables MP1-MP3 (ILU(0))", file=sys.stderr, flush=True)
            out["paper_tables"] = bench_paper_tables(args, torch, hh, W)
    if args.serve_long:
        print("bench: c5 long", file=sys.stderr, flush=True)
        out["serving_long"] = bench_c5_long(args, torch, hh, W)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu_baseline(args, cfg, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
