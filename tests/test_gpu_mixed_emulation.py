"""Mixed-precision CG on the GPU against the oracle's emulation of the same method.

The oracle emulates reliable-update CG (the mixed-precision form of the Sec. 3.3
CG; reliable updates after Clark et al., CPC 181 (2010)) with float arithmetic on
fields stored in the inner format, FP64 folds of the solution and FP64 true
residuals, and the same trigger rule (every `reliable_every` iterations of the
system's own, a drop of |r| by `reliable_delta` since the last update, and
recursive convergence).  The GPU sums in another order, so the two recurrences
agree to rounding, not bit for bit; what must agree is the course of the solve:

  * the iteration count within 5% + 2 of the emulation's;
  * the number of reliable updates (FP64 true-residual evaluations) within 2;
  * both meet the FP64 true residual recomputed by the oracle, and their
    solutions agree within 2 cond(A) tol.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, rel, setup, to_dev

pytestmark = pytest.mark.gpu

CASES = [((8, 8, 8, 8), 3, "fund"), ((8, 8, 8, 8), 2, "adj"), ((4, 4, 4, 8), 4, "asym"), ((4, 4, 4, 8), 3, "sym")]
SCHEDULES = {"trigger": (50, None), "every20": (20, 0.0)}


def _resid(dims, ur, kappa, x, b):
    y = orc.deo(dims, ur, kappa, orc.deo(dims, ur, kappa, x, THETA_AP), THETA_AP, dagger=True)
    return rel(y, b) if np.linalg.norm(b) else 0.0


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("inner", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("dims,nc,rep", CASES, ids=lambda c: str(c))
def test_mixed_cg_follows_the_oracle_emulation(dims, nc, rep, inner, sched):
    kappa = 0.135
    every, delta = SCHEDULES[sched]
    if delta is None:
        delta = hrw.RELIABLE_DELTA[inner]
    uf, ur, g = setup(dims, nc, rep, "thermal", seed=71, dtypes=("f64", inner))
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, g.nr, seed=72))[0]
    xe, info = orc.cg_mixed(dims, ur, kappa, b, THETA_AP, orc.SYSTEM_EO, tol=1e-10, max_iter=5000, inner=inner,
                            every=every, delta=delta)
    assert info["status"] == 0 and info["true_rel_resid"] <= 1e-10
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="ddag_d_eo", inner_dtype=inner,
                           reliable_every=every, reliable_delta=delta, theta=THETA_AP)
    x, res, rc = hrw.cg_solve(g, to_dev(b), kappa, prm)
    x = x.cpu().numpy()
    assert rc == 0, res
    it_gpu, it_emu = res[0]["iters"], info["iters"]
    assert abs(it_gpu - it_emu) <= 0.05 * it_emu + 2, (it_gpu, it_emu)
    assert abs(res[0]["reliable_updates"] - info["updates"]) <= 2, (res[0]["reliable_updates"], info["updates"])
    assert _resid(dims, ur, kappa, x, b) <= 1.01e-10
    xo, cinfo = orc.cg(dims, ur, kappa, b, THETA_AP, orc.SYSTEM_EO, tol=1e-12)
    lo, hi = orc.lanczos_extremes(cinfo["alpha"], cinfo["beta"])
    assert rel(x, xe) <= 2 * (hi / lo) * 1e-10


def test_fp16_scaled_source_follows_the_emulation():
    """A source far below binary16's normal range (|b| ~ 1e-12): the per-system scale
    keeps both the emulation and the GPU on the unscaled course."""
    dims, nc, rep, kappa = (4, 4, 4, 8), 2, "adj", 0.135
    uf, ur, g = setup(dims, nc, rep, "thermal", seed=73, dtypes=("f64", "f16"))
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, g.nr, seed=74))[0] * 2.0 ** -40
    xe, info = orc.cg_mixed(dims, ur, kappa, b, THETA_AP, orc.SYSTEM_EO, tol=1e-10, max_iter=5000, inner="f16",
                            every=50, delta=1e-2)
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="ddag_d_eo", inner_dtype="f16",
                           reliable_every=50, reliable_delta=1e-2, theta=THETA_AP)
    x, res, rc = hrw.cg_solve(g, to_dev(b), kappa, prm)
    assert rc == 0 and info["status"] == 0
    assert abs(res[0]["iters"] - info["iters"]) <= 0.05 * info["iters"] + 2
    assert abs(res[0]["reliable_updates"] - info["updates"]) <= 2
    assert _resid(dims, ur, kappa, x.cpu().numpy(), b) <= 1.01e-10
