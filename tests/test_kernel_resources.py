"""Register and scratch use of the device kernels (CPU: hipcc's resource-usage remarks for gfx950).

Every kernel of the solve path is compiled with no scratch (private memory) per lane: a spill
would put per-lane stack traffic on top of the HBM streams the kernels are sized for.  The one
exception is the clover builder (once per clover field), whose per-site Gauss-Jordan inversion
of the 2 N_R x 2 N_R blocks keeps its matrices in private memory by design.
"""

import concurrent.futures
import os
import re
import subprocess
import tempfile

import pytest

from paper_2405_19294_amd import build as hb

ALLOWED_SCRATCH = ("clover_build_kernel",)


def _resources(src, out_dir):
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = ["hipcc", *hb.HIPFLAGS, "-I", os.path.join(hb.HERE, "..", "include"), "-c", src, "-o", obj,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"(VGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1).split()[0]] = int(m.group(2))
    return kernels


def test_no_kernel_of_the_solve_path_uses_scratch():
    srcs = [s for s in hb.sources()]
    with tempfile.TemporaryDirectory() as d, concurrent.futures.ThreadPoolExecutor(4) as ex:
        results = list(ex.map(lambda s: _resources(s, d), srcs))
    kernels = {k: v for res in results for k, v in res.items()}
    assert any("hop_su3_kernel" in k for k in kernels) and any("hop_mrhs_kernel" in k for k in kernels)
    spilling = {k: v.get("ScratchSize") for k, v in kernels.items()
                if v.get("ScratchSize", 0) and not any(a in k for a in ALLOWED_SCRATCH)}
    assert not spilling, spilling
