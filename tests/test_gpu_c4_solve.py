"""The multi-source mixed-precision solve in the shape of the SU(3) two-index
symmetric workload (N_R = 6, 6-24 point-smeared sources, FP32 arithmetic on FP32,
bfloat16 or binary16 inner fields, FP64 reliable updates; the Sec. 3.3 CG with
several right-hand sides sharing each operator launch).

With 6 or more sources every hop of these solves runs the multi-source kernel
(links staged once per workgroup in LDS), including its fused CG-update instance.
Checked per source: the FP64 true residual recomputed by the oracle, the error
against the oracle's FP64 solution within cond(A) tol, and the batched solution
equal bit for bit to the same source solved alone (the per-source arithmetic and
the partial-sum layout do not depend on the batch).
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, rel, to_dev

pytestmark = pytest.mark.gpu

KAPPA = 0.135
# (6, 6, 2, 2): 72 sites per parity, a partly filled 16-site group and 64-site block
LATTICES = [(6, 6, 2, 2), (4, 4, 4, 6)]


def _sources(dims, nr, n):
    full = fx.point_smeared_sources(dims, nr, n, seed=7)
    return np.stack([orc.split_eo(dims, f)[0] for f in full])


def _check_solve(dims, ur, g, src, inner, single=(0, -1)):
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="ddag_d_eo", inner_dtype=inner,
                           reliable_every=50, reliable_delta=hrw.RELIABLE_DELTA[inner], theta=THETA_AP)
    n = src.shape[0]
    x, res, rc = hrw.cg_solve(g, to_dev(src), [KAPPA] * n, prm)
    assert rc == 0, res
    x = x.cpu().numpy()
    for k in range(n):
        assert res[k]["true_rel_resid"] <= 1e-10
        ax = orc.deo(dims, ur, KAPPA, orc.deo(dims, ur, KAPPA, x[k], THETA_AP), THETA_AP, dagger=True)
        assert rel(ax, src[k]) <= 1.01e-10, k
        xo, info = orc.cg(dims, ur, KAPPA, src[k], THETA_AP, orc.SYSTEM_EO, tol=1e-12)
        lo, hi = orc.lanczos_extremes(info["alpha"], info["beta"])
        assert rel(x[k], xo) <= (hi / lo) * 1e-10, k
    for k in single:
        x1, res1, rc1 = hrw.cg_solve(g, to_dev(src[k]), KAPPA, prm)
        assert rc1 == 0
        assert np.array_equal(x[k], x1.cpu().numpy().reshape(x[k].shape)), k
        assert res1[0]["iters"] == res[k]["iters"]
        assert res1[0]["reliable_updates"] == res[k]["reliable_updates"]


@pytest.mark.parametrize("sites", [16, 32])
@pytest.mark.parametrize("dims", LATTICES, ids=str)
@pytest.mark.parametrize("n_src", [6, 24])
def test_c4_shaped_fp32_multi_source_cg(dims, n_src, sites, monkeypatch):
    """With 16 or 32 sites per multi-source workgroup (two partial-sum groups in the latter)."""
    monkeypatch.setenv("HRW_MRHS_SITES", str(sites))
    assert hrw.rep_dim(3, "sym") == 6
    uf = fx.gauge_field(dims, 3, "thermal", seed=6, eps=0.3)
    ur = orc.rep_map(3, "sym", uf)
    g = hrw.Gauge(dims, 3, "sym", to_dev(uf), dtypes=("f64", "f32"))
    try:
        _check_solve(dims, ur, g, _sources(dims, 6, n_src), "f32")
    finally:
        g.close()


@pytest.mark.parametrize("inner", ["bf16", "f16"])
def test_c4_shaped_16bit_multi_source_cg(inner):
    dims = LATTICES[0]
    uf = fx.gauge_field(dims, 3, "thermal", seed=6, eps=0.3)
    ur = orc.rep_map(3, "sym", uf)
    g = hrw.Gauge(dims, 3, "sym", to_dev(uf), dtypes=("f64", inner))
    try:
        _check_solve(dims, ur, g, _sources(dims, 6, 24), inner)
    finally:
        g.close()


TUNE_SCRIPT = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import fixtures as fx, oracle as orc
from paper_2405_19294_amd import hrw
from gpu_helpers import THETA_AP, to_dev
dims = (4, 4, 4, 6)
uf = fx.gauge_field(dims, 3, "thermal", seed=6, eps=0.3)
g = hrw.Gauge(dims, 3, "sym", to_dev(uf), dtypes=("f32",))
pe = orc.split_eo(dims, fx.gaussian_spinor(dims, 6, seed=8, n_rhs=8))[0]
out = hrw.deo_apply(g, 0.13, to_dev(pe), THETA_AP, "f32").cpu().numpy()
np.save({out!r}, out)
"""


def test_tuned_launch_shapes_persist_across_processes(tmp_path):
    """The first process tunes the multi-source launch shape (threads, sites, walk chunk and its
    x1-planes) and writes it to the cache file (JSON, keyed by architecture, N_R, row split,
    storage, sources and volume class); a later
    process takes a shape from the file instead of tuning (a hand-edited entry survives it
    unchanged); the results are bitwise the same either way."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, HRW_TUNE_CACHE=str(cache))
    env.pop("HRW_MRHS_SITES", None)
    env.pop("HRW_TUNE", None)

    def run(tag):
        script = TUNE_SCRIPT.format(root=root, tests=os.path.join(root, "tests"), out=str(tmp_path / f"{tag}.npy"))
        r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return np.load(tmp_path / f"{tag}.npy")

    first = run("a")
    entries = json.loads(cache.read_text())
    keys = [k for k in entries if "/nr6/rs6/f32/n8/" in k]
    assert keys, entries
    e = entries[keys[0]]
    assert e["sites"] in (16, 32) and e["threads"] % 64 == 0 and e["cmax"] in (4, 16, 32, 64)
    assert e["planes"] in (1, 2, 4, 8)
    # a different (valid) shape in the file: the next process uses it without tuning
    entries[keys[0]] = {"threads": 128, "cmax": 4, "sites": 32 if e["sites"] == 16 else 16, "planes": 1, "us": 1.0}
    cache.write_text(json.dumps(entries, indent=1))
    second = run("b")
    assert json.loads(cache.read_text())[keys[0]]["threads"] == 128
    assert np.array_equal(first, second)
