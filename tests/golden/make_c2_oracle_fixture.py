"""Writes c2_1024_oracle_solve.json: the CPU oracle's FP64 Bi-CGSTAB solve of
the 2D 1024^2 headline problem (workloads.c2()) to 1e-8 -- matvec and
iteration counts, the whole residual history, the solution's norm and 64
seeded entries.  Calls only oracle/ and the input recipes; run from the
repository root:  python tests/golden/make_c2_oracle_fixture.py"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O                      # noqa: E402
from paper_0912_0180_amd import workloads as W      # noqa: E402


def main():
    c = W.c2()
    o = O.Grid(c["desc"], c["phi"])
    t = time.time()
    x, info = o.solve(c["b"], tol=1e-8, history=True)
    idx = np.sort(W.rng(1024).choice(o.N, size=64, replace=False))
    out = {"workload": "c2 (2D 1024^2, 8 levels, CSG pi/8, V(1,1)), FP64 Bi-CGSTAB to 1e-8, x0 = 0",
           "status": int(info["status"]), "matvecs": int(info["matvecs"]), "iterations": int(info["iterations"]),
           "rel_res_true": float(info["rel_res_true"]), "x_norm": float(np.linalg.norm(x)),
           "sample_index": [int(i) for i in idx],
           "sample_re": [float(x[i].real) for i in idx], "sample_im": [float(x[i].imag) for i in idx],
           "history": [float(v) for v in info["history"][: info["matvecs"]]],
           "oracle_seconds": time.time() - t, "oracle_threads": O.num_threads()}
    path = os.path.join(ROOT, "tests", "golden", "c2_1024_oracle_solve.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, out["matvecs"], "matvecs in %.0f s" % out["oracle_seconds"])


if __name__ == "__main__":
    main()
