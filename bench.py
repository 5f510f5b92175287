"""Benchmark: CSG-multigrid-preconditioned Bi-CGSTAB on the ECS Helmholtz
problem, on one MI355X.

Workload (one step = one whole solve, x0 = 0 -> ||b - Hx|| / ||b|| < 1e-8):
2D 1024 x 1024 cells over [-0.25, 1.25]^2 (interior [0,1]^2, ECS layers of
width 0.25 at angle pi/6), k0 at 10 points per wavelength,
k(x) = k0 (1 + 0.3 * sum of 8 seeded Gaussian bumps of width 0.05), unit point
source at the centre, CSG angle pi/8, 8 levels, one V(1,1) cycle per
preconditioner application.  The headline value is solves/s of the
mixed-precision solve (complex-FP32 V-cycle, FP64 Krylov); the FP64 solve,
the V-cycle and operator bandwidths, the roofline of the dominant kernel and
the CPU oracle on a bounded sample are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def vcycle_bytes(g, fp32):
    """Algorithmic bytes of one fused V(1,1) cycle: every field read or
    written once per fused pass at its storage precision."""
    dims = g.level_dims
    d = g.dim
    cb = 8 if fp32 else 16          # complex bytes inside the cycle
    pb = 4 if fp32 else 8           # phi bytes
    total = 0
    for l in range(g.levels - 1):
        N = int(np.prod(dims[l][:d]))
        Nc = N // (2 ** d)
        fin = 16 if l == 0 else cb  # level-0 input is the FP64 Krylov vector
        down = N * (fin + pb) + Nc * cb
        up = N * (fin + pb) + Nc * cb + N * cb
        total += down + up
    total += g.Nc * g.Nc * cb + 2 * g.Nc * cb
    return total


def time_calls(torch, fn, reps):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-matvecs", type=int, default=24)
    ap.add_argument("--quick", action="store_true", help="skip the secondary measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (multi-GPU sharding is a design note, "
              "not part of the measured path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0912_0180_amd import hh
    from paper_0912_0180_amd import workloads as W

    torch.cuda.set_device(0)
    cfg = W.c2(n=args.n, levels=args.levels)
    t0 = time.perf_counter()
    g = hh.Grid(cfg["desc"], cfg["phi"])
    setup_s = time.perf_counter() - t0
    b = torch.from_numpy(cfg["b"]).to("cuda")
    x = torch.zeros_like(b)

    def solve(prec):
        return g.solve(b, x=x, tol=1e-8, vcycle_prec=prec, max_matvec=20000)

    # warmup (also allocates the work space)
    for _ in range(args.warmup):
        _, info = solve("c64")
    torch.cuda.synchronize()
    t = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, info = solve("c64")
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms_step = elapsed / args.steps * 1e3
    info_m = infos[-1]
    assert all(i["status"] == 0 and i["rel_res_true"] < 1e-8 for i in infos), infos

    out = {
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
        "setup_s": setup_s,
    }
    if not args.quick:
        _, i64 = solve("c128")
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, i64 = solve("c128")
        torch.cuda.synchronize()
        out["time_to_tol_ms_fp64"] = (time.perf_counter() - t) * 1e3
        out["matvecs_fp64"] = i64["matvecs"]
        out["rel_res_true_fp64"] = i64["rel_res_true"]
        # V-cycle and operator bandwidth (algorithmic bytes / time)
        f = torch.randn(g.N, dtype=torch.complex128, device="cuda")
        u64 = torch.empty_like(f)
        u32 = torch.empty(g.N, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(f)
        tv64 = time_calls(torch, lambda: g.vcycle(f, "c128", out=u64), 100)
        tv32 = time_calls(torch, lambda: g.vcycle(f, "c64", out=u32), 100)
        th = time_calls(torch, lambda: g.apply(f, "H", out=y), 200)
        out["vcycle_us_fp64"] = tv64 * 1e6
        out["vcycle_us_mixed"] = tv32 * 1e6
        out["vcycle_GBps_fp64"] = vcycle_bytes(g, False) / tv64 / 1e9
        out["vcycle_GBps_mixed"] = vcycle_bytes(g, True) / tv32 / 1e9
        ah = 40.0 * g.N / th / 1e9
        out["applyH_GBps"] = ah
        out["roofline"] = {"bound": "hbm", "kernel": "k_applyH (y = H x, c128)", "achieved": ah,
                           "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ah / HBM_PEAK_GBPS,
                           "traffic": None, "bytes_per_unknown": 40}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        o = O.Grid(cfg["desc"], cfg["phi"])
        m = args.cpu_sample_matvecs
        t = time.perf_counter()
        _, io = o.solve(cfg["b"], tol=1e-8, max_matvec=m, max_restarts=0)
        ts = time.perf_counter() - t
        full_mv = out.get("matvecs_fp64", info_m["matvecs"])
        est = ts / io["matvecs"] * full_mv
        out["cpu_baseline"] = {"value": 1.0 / est, "unit": "solves/s", "cores": O.num_threads(), "kind": "oracle",
                               "sample": "FP64 oracle Bi-CGSTAB on the same problem, first %d matvecs in %.1f s, "
                                         "scaled to the %d matvecs of the full solve" % (io["matvecs"], ts, full_mv)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
