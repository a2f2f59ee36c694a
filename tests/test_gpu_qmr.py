"""GPU parity of QMR-g5 (the HIP library through its C ABI) against the CPU oracle.

Tolerances as for BiCGstab: the FP64 true residual recomputed by the oracle from the GPU's x is
<= tol (1 % slack) and matches the reported one; |x_gpu - x_oracle| / |x_oracle| <= 2 cond(D_hat)
tol with cond(D_hat) from the Lanczos extremes of an oracle CG run on the normal equations;
iteration counts within 5 % (+2) of the oracle's; several right-hand sides bitwise equal to single
ones.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, THETA_TW, rel, setup, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ((8, 8, 8, 8), 3, "fund", 0.135),
    ((4, 4, 4, 8), 2, "adj", 0.125),
    ((4, 4, 4, 4), 4, "asym", 0.125),
    ((4, 4, 4, 4), 3, "sym", 0.12),
    ((2, 4, 2, 6), 3, "fund", 0.13),
]


def ids(c):
    return f"{'x'.join(map(str, c[0]))}-su{c[1]}-{c[2]}"


def cond_dhat(dims, ur, kappa, be, theta):
    eta = orc.deo(dims, ur, kappa, be, theta, dagger=True)
    _, info = orc.cg(dims, ur, kappa, eta, theta, orc.SYSTEM_EO, tol=1e-8)
    lo, hi = orc.lanczos_extremes(info["alpha"], info["beta"])
    return float(np.sqrt(hi / lo))


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_qmr_g5_dhat_matches_oracle(case):
    dims, nc, rep, kappa = case
    uf, ur, g = setup(dims, nc, rep, "thermal", seed=91, dtypes=("f64",))
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, g.nr, seed=92))[0]
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", theta=THETA_AP)
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(be), kappa, prm)
    assert rc == 0, res
    x = x.cpu().numpy()
    r = rel(orc.deo(dims, ur, kappa, x, THETA_AP), be)
    assert r <= 1.01e-10 and abs(r - res[0]["true_rel_resid"]) <= 1e-3 * r + 1e-16
    xo, info = orc.qmr_g5(dims, ur, kappa, be, THETA_AP, orc.BICG_EO, tol=1e-10)
    assert info["status"] == 0
    assert abs(res[0]["iters"] - info["iters"]) <= 0.05 * info["iters"] + 2, (res[0]["iters"], info["iters"])
    assert rel(x, xo) <= 2 * cond_dhat(dims, ur, kappa, be, THETA_AP) * 1e-10


def test_qmr_g5_full_system_and_batches():
    dims, kappa = (4, 4, 4, 8), 0.13
    uf, ur, g = setup(dims, 3, "fund", "thermal", seed=93, dtypes=("f64",))
    b = fx.gaussian_spinor(dims, 3, seed=94)
    prm = hrw.solve_params(tol=1e-10, system="d_eo", theta=THETA_TW)
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(b), kappa, prm)
    assert rc == 0, res
    x = x.cpu().numpy()
    dres = rel(orc.dw(dims, ur, kappa, x, THETA_TW), b)
    assert dres <= 1e-9 and abs(dres - res[0]["d_rel_resid"]) <= 1e-3 * dres + 1e-16
    xc, _ = orc.solve_d_eo(dims, ur, kappa, b, THETA_TW, tol=1e-12)
    assert rel(x, xc) <= 1e-7
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=95, n_rhs=3))[0]
    ks = [0.12, 0.125, 0.13]
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", theta=THETA_AP)
    xm, resm, rc = hrw.qmr_g5_solve(g, to_dev(be), ks, prm)
    assert rc == 0
    xm = xm.cpu().numpy()
    for k in range(3):
        x1, res1, rc1 = hrw.qmr_g5_solve(g, to_dev(be[k]), ks[k], prm)
        assert rc1 == 0 and np.array_equal(xm[k], x1.cpu().numpy()) and res1[0]["iters"] == resm[k]["iters"]


def test_qmr_g5_edge_cases():
    dims = (4, 4, 4, 4)
    uf, ur, g = setup(dims, 2, "fund", "haar", seed=96, dtypes=("f64", "f32"))
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", theta=THETA_AP)
    zero = np.zeros((fx.volume(dims) // 2, 4, 2), complex)
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(zero), 0.12, prm)
    assert rc == 0 and res[0]["iters"] == 0 and not x.abs().max().item()
    nan = zero.copy()
    nan[5, 2, 1] = np.nan
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(nan), 0.12, prm)
    assert rc == hrw.EBREAKDOWN and res[0]["status"] == hrw.EBREAKDOWN
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 2, seed=97))[0]
    # kappa = 0: one step; x = ctau (v / rr) carries about a dozen roundings of b (v = r / |r|, the
    # J-products behind alpha and delta, the rotation), so agreement to 1e-14 ~ 90 u
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(b), 0.0, prm)
    assert rc == 0 and res[0]["iters"] == 1 and rel(x.cpu().numpy(), b) <= 1e-14
    few = hrw.solve_params(tol=1e-10, max_iter=4, system="dhat_eo", theta=THETA_AP)
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(b), 0.12, few)
    assert rc == hrw.NOT_CONVERGED and res[0]["iters"] == 4
    r = rel(orc.deo(dims, ur, 0.12, x.cpu().numpy(), THETA_AP), b)
    assert abs(r - res[0]["true_rel_resid"]) <= 1e-6 * r
    xo, info = orc.qmr_g5(dims, ur, 0.12, b, THETA_AP, orc.BICG_EO, tol=0.0, max_iter=4)
    assert rel(x.cpu().numpy(), xo) < 1e-12
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(np.stack([b, nan])), [0.12, 0.12], prm)
    assert rc == hrw.EBREAKDOWN and res[0]["status"] == 0 and res[1]["status"] == hrw.EBREAKDOWN
    with pytest.raises(hrw.HrwError) as e:
        hrw.qmr_g5_solve(g, to_dev(b), 0.12, hrw.solve_params(system="dhat_eo", inner_dtype="f32"))
    assert e.value.code == hrw.EUNSUPPORTED
