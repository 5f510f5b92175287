"""Builds the gfx950 shared library libhh.so in-tree with hipcc.

    python -m paper_0912_0180_amd.build

Flags: -ffp-contract=off (fixed FP64 operation order: no fused multiply-add
contraction, so results are reproducible and comparable value by value), and
packed FP32 instructions switched off for the device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhh.so")
SOURCES = ["hh_setup.cpp", "hh_lib.hip", "hh_solve.hip", "hh_select.hip", "hh_server.cpp"]
HEADERS = ["hh_common.h", "hh_kernels.hpp", "hh_lib.h", "hh_setup.h", "hh_idr_kernels.hpp"]
ARCH = os.environ.get("HH_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose=True, jobs=8):
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(ROOT, "_build", os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip", "--offload-arch=" + ARCH] if src.endswith(".hip") else ["--offload-arch=" + ARCH]
        cmd = ["hipcc"] + lang + FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE, text=True))
    failed = False
    for p in procs:
        out, err = p.communicate()
        msg = "\n".join(l for l in (out + err).splitlines()
                        if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
        if msg.strip():
            print(msg, file=sys.stderr)
        if p.returncode != 0:
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
