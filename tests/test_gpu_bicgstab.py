"""GPU parity of BiCGstab (the HIP library through its C ABI) against the CPU oracle.

Tolerances (the solution is unique, so every correct solver meets them):
  * the FP64 true residual |b - D_hat x| / |b| (or |b - D x| / |b|) recomputed by
    the oracle from the GPU's x is <= tol (1 % slack for the recomputation's
    own rounding), and matches the residual the library reports;
  * |x_gpu - x_oracle| / |x_oracle| <= 2 cond(D_hat) tol, with cond(D_hat) =
    sqrt(cond(D_hat^+ D_hat)) from the Lanczos extremes of an oracle CG run;
  * plain FP64 iteration counts within 5 % (+2) of the oracle's (the two
    reduce in different orders, so the paths part at rounding level);
  * several right-hand sides in one call give bitwise the single-system results.
BF16 inner storage (FP32 arithmetic, FP64 reliable updates every tenfold drop)
is held to the same FP64 tolerances: the reliable updates make the final
residual an FP64 one whatever the inner precision.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, THETA_TW, rel, setup, to_dev

pytestmark = pytest.mark.gpu

# (dims, nc, rep, kappa): N_R = 2, 3, 4, 6; a ragged half field (48 sites) and several tiles
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


def dhat_resid(dims, ur, kappa, x, b, theta):
    return rel(orc.deo(dims, ur, kappa, x, theta), b)


@pytest.mark.parametrize("case", CASES, ids=ids)
@pytest.mark.parametrize("inner", ["f64", "f32", "bf16"])
def test_bicgstab_dhat_matches_oracle(case, inner):
    dims, nc, rep, kappa = case
    uf, ur, g = setup(dims, nc, rep, "thermal", seed=81, dtypes=tuple(dict.fromkeys(("f64", inner))))
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, g.nr, seed=82))[0]
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", inner_dtype=inner, theta=THETA_AP,
                           reliable_delta=hrw.RELIABLE_DELTA[inner])
    x, res, rc = hrw.bicgstab_solve(g, to_dev(be), kappa, prm)
    x = x.cpu().numpy()
    assert rc == 0, res
    r = dhat_resid(dims, ur, kappa, x, be, THETA_AP)
    assert r <= 1.01e-10
    assert abs(r - res[0]["true_rel_resid"]) <= 1e-3 * r + 1e-16
    xo, info = orc.bicgstab(dims, ur, kappa, be, THETA_AP, orc.BICG_EO, tol=1e-10)
    assert info["status"] == 0
    assert rel(x, xo) <= 2 * cond_dhat(dims, ur, kappa, be, THETA_AP) * 1e-10
    if inner == "f64":
        assert abs(res[0]["iters"] - info["iters"]) <= 0.05 * info["iters"] + 2, (res[0]["iters"], info["iters"])
        assert res[0]["reliable_updates"] == 0
    else:
        assert res[0]["reliable_updates"] >= 1


@pytest.mark.parametrize("inner", ["f64", "f32", "bf16"])
def test_bicgstab_full_system_through_schur(inner):
    """D x = b (system d_eo): |b - D x| / |b| recomputed by the oracle equals the reported
    d_rel_resid, and x matches the oracle's BiCGstab route and its CG route."""
    dims, kappa = (4, 4, 4, 8), 0.13
    uf, ur, g = setup(dims, 3, "fund", "thermal", seed=83, dtypes=("f64", "f32", "bf16"))
    b = fx.gaussian_spinor(dims, 3, seed=84)
    prm = hrw.solve_params(tol=1e-10, system="d_eo", inner_dtype=inner, theta=THETA_TW,
                           reliable_delta=hrw.RELIABLE_DELTA[inner])
    x, res, rc = hrw.bicgstab_solve(g, to_dev(b), kappa, prm)
    x = x.cpu().numpy()
    assert rc == 0, res
    dres = rel(orc.dw(dims, ur, kappa, x, THETA_TW), b)
    assert abs(dres - res[0]["d_rel_resid"]) <= 1e-3 * dres + 1e-16
    assert dres <= 1e-9
    xb, ib = orc.solve_d_eo_bicgstab(dims, ur, kappa, b, THETA_TW, tol=1e-12)
    xc, ic = orc.solve_d_eo(dims, ur, kappa, b, THETA_TW, tol=1e-12)
    assert ib["status"] == 0 and ic["status"] == 0
    assert rel(x, xb) <= 1e-7 and rel(x, xc) <= 1e-7


def test_bicgstab_multi_rhs_bitwise_equals_single():
    dims = (4, 4, 4, 4)
    uf, ur, g = setup(dims, 3, "fund", "thermal", seed=85, dtypes=("f64", "f32", "bf16"))
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=86, n_rhs=4))[0]
    ks = [0.12, 0.125, 0.13, 0.135]
    for inner in ("f64", "f32", "bf16"):
        prm = hrw.solve_params(tol=1e-10, system="dhat_eo", inner_dtype=inner, theta=THETA_AP,
                               reliable_delta=hrw.RELIABLE_DELTA[inner])
        xm, resm, rc = hrw.bicgstab_solve(g, to_dev(b), ks, prm)
        assert rc == 0
        xm = xm.cpu().numpy()
        for k in range(4):
            x1, res1, rc1 = hrw.bicgstab_solve(g, to_dev(b[k]), ks[k], prm)
            assert rc1 == 0
            assert np.array_equal(xm[k], x1.cpu().numpy()), (inner, k)
            assert res1[0]["iters"] == resm[k]["iters"]


def test_bicgstab_deterministic():
    dims = (4, 4, 4, 4)
    uf, ur, g = setup(dims, 2, "adj", "thermal", seed=87, dtypes=("f64",))
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=88))[0]
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", theta=THETA_AP)
    x1 = hrw.bicgstab_solve(g, to_dev(b), 0.125, prm)[0].cpu().numpy()
    x2 = hrw.bicgstab_solve(g, to_dev(b), 0.125, prm)[0].cpu().numpy()
    assert np.array_equal(x1, x2)


def test_bicgstab_edge_cases():
    dims = (4, 4, 4, 4)
    uf, ur, g = setup(dims, 2, "fund", "haar", seed=89, dtypes=("f64", "f32"))
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", theta=THETA_AP)
    zero = np.zeros((fx.volume(dims) // 2, 4, 2), complex)
    x, res, rc = hrw.bicgstab_solve(g, to_dev(zero), 0.12, prm)
    assert rc == 0 and res[0]["iters"] == 0 and not x.abs().max().item()
    nan = zero.copy()
    nan[3, 1, 0] = np.nan
    x, res, rc = hrw.bicgstab_solve(g, to_dev(nan), 0.12, prm)
    assert rc == hrw.EBREAKDOWN and res[0]["status"] == hrw.EBREAKDOWN
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 2, seed=90))[0]
    # kappa = 0: D_hat = 1, one iteration
    x, res, rc = hrw.bicgstab_solve(g, to_dev(b), 0.0, prm)
    assert rc == 0 and res[0]["iters"] == 1 and rel(x.cpu().numpy(), b) <= 1e-15
    few = hrw.solve_params(tol=1e-10, max_iter=3, system="dhat_eo", theta=THETA_AP)
    x, res, rc = hrw.bicgstab_solve(g, to_dev(b), 0.12, few)
    assert rc == hrw.NOT_CONVERGED and res[0]["iters"] == 3 and res[0]["true_rel_resid"] > 1e-10
    assert abs(dhat_resid(dims, ur, 0.12, x.cpu().numpy(), b, THETA_AP) - res[0]["true_rel_resid"]) <= \
        1e-6 * res[0]["true_rel_resid"]
    # a good and a non-finite system in one call: the good one still converges
    x, res, rc = hrw.bicgstab_solve(g, to_dev(np.stack([b, nan])), [0.12, 0.12], prm)
    assert rc == hrw.EBREAKDOWN and res[0]["status"] == 0 and res[1]["status"] == hrw.EBREAKDOWN
    assert dhat_resid(dims, ur, 0.12, x[0].cpu().numpy(), b, THETA_AP) <= 1.01e-10
    # systems 0-2 are CG's; FP16 inner storage is not offered
    with pytest.raises(hrw.HrwError) as e:
        hrw.bicgstab_solve(g, to_dev(b), 0.12, hrw.solve_params(system="ddag_d_eo"))
    assert e.value.code == hrw.EINVAL
    with pytest.raises(hrw.HrwError) as e:
        hrw.cg_solve(g, to_dev(b), 0.12, hrw.solve_params(system="dhat_eo"))
    assert e.value.code == hrw.EINVAL
    with pytest.raises(hrw.HrwError) as e:
        hrw.bicgstab_solve(g, to_dev(b), 0.12, hrw.solve_params(system="dhat_eo", inner_dtype="f16"))
    assert e.value.code == hrw.EUNSUPPORTED
