"""Build checks that need no GPU: every device kernel compiles for gfx950
without private (scratch) memory, i.e. no register spills and no dynamically
indexed per-thread arrays."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0912_0180_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_no_kernel_uses_scratch(tmp_path):
    from paper_0912_0180_amd import build as B
    cmd = (["hipcc", "-x", "hip", "--offload-arch=gfx950"] + B.FLAGS +
           ["-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, "hh_lib.hip"),
            "-o", str(tmp_path / "hh_lib.o"), "-Rpass-analysis=kernel-resource-usage"])
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", out.stderr)
    scratch = [int(v) for v in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out.stderr)]
    assert len(names) == len(scratch) and len(names) > 20
    bad = [(n, s) for n, s in zip(names, scratch) if s != 0]
    assert not bad, bad
