"""Parity at the full sizes of the benchmark workloads, in the launch configurations bench.py times.

The inputs are the benchmarks' own seeded fields (fixtures); the references come from the CPU oracle,
either on the whole field (it finishes in seconds at these sizes) or through properties the oracle
recomputes (the residual of a solve):
  * SU(3) fund 32^4 (default workload): D_hat and D_hat^+ in FP64 to 1e-13, the full-lattice D_W in
    FP32 within the a-priori bound, and the |b - D x| / |b| of the FP64 CG solve, of the BiCGstab
    solves (FP64 and FP32 inner) and of the QMR-g5 solve recomputed by the oracle; with the clover
    term (c_sw = 1), D_hat_sw in FP64 and the FP32-inner BiCGstab solve of D_sw x = b; with the
    two-row SU(3) hop, D_hat in FP64 and the FP64 CG and BF16-inner BiCGstab solves;
  * SU(2) adj and SU(4) asym 24^3x48, with stored U_R and with the representation map fused into the
    hop: D_hat in FP64, and the FP32-inner mixed solve's residual of the even/odd normal equations
    recomputed by the oracle;
  * SU(3) sym 32^4 with 24 sources: the multi-source FP32 kernel (the launch the multi-source CG uses)
    bitwise equal to single-source applies, the batched FP64 D_hat against the oracle, and the mixed
    multi-source CG of the benchmark (24 sources, FP32 inner) with the residual of two sources
    recomputed by the oracle.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, U32, bound_check, fp64_close, rel, stored_input, to_dev

pytestmark = pytest.mark.gpu

C2 = (32, 32, 32, 32)
C3 = (48, 24, 24, 24)
KAPPA = 0.135


def _even(dims, full):
    return orc.split_eo(dims, full)[0]


@pytest.fixture(scope="module")
def c2_field():
    uf = fx.gauge_field(C2, 3, "thermal", seed=2, eps=0.3)
    ur = orc.rep_map(3, "fund", uf)
    g = hrw.Gauge(C2, 3, "fund", to_dev(uf), dtypes=("f64", "f32"))
    yield ur, g
    g.close()


def test_c2_operators_full_size(c2_field):
    ur, g = c2_field
    psi = fx.gaussian_spinor(C2, 3, seed=3)
    pe = _even(C2, psi)
    for dagger in (False, True):
        out = hrw.deo_apply(g, KAPPA, to_dev(pe), THETA_AP, "f64", dagger=dagger).cpu().numpy()
        fp64_close(out, orc.deo(C2, ur, KAPPA, pe, THETA_AP, dagger=dagger))
    ur_r = orc.round_to("f32", ur)
    q_r, psi_r = stored_input("f32", psi)
    out32 = hrw.dw_apply(g, KAPPA, to_dev(psi), THETA_AP, "f32").cpu().numpy()
    bound_check(C2, ur_r, q_r, KAPPA, out32, orc.dw(C2, ur_r, KAPPA, psi_r, THETA_AP), 3, 0.0, THETA_AP)


def test_c2_solve_residual_by_oracle(c2_field):
    """The default workload's solve (CGNR on the even/odd system, FP64, tol 1e-10)."""
    ur, g = c2_field
    b = fx.gaussian_spinor(C2, 3, seed=3)
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="d_cgnr_eo", inner_dtype="f64", theta=THETA_AP)
    x, res, rc = hrw.cg_solve(g, to_dev(b), KAPPA, prm)
    assert rc == 0 and res[0]["true_rel_resid"] <= 1e-10
    d_res = rel(orc.dw(C2, ur, KAPPA, x.cpu().numpy(), THETA_AP), b)
    assert abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res
    assert d_res < 1e-8


def test_c2_two_row_links_full_size():
    """The default workload's field with the SU(3) two-row hop (the bench's two-row rows): D_hat and
    D_hat^+ in FP64 to 1e-13, and the FP64 CG and BF16-inner BiCGstab solves of D x = b with
    |b - D x| / |b| recomputed by the oracle."""
    uf = fx.gauge_field(C2, 3, "thermal", seed=2, eps=0.3)
    ur = orc.rep_map(3, "fund", uf)
    g = hrw.Gauge(C2, 3, "fund", to_dev(uf), dtypes=("f64", "bf16"), two_rows=True)
    psi = fx.gaussian_spinor(C2, 3, seed=3)
    pe = _even(C2, psi)
    for dagger in (False, True):
        out = hrw.deo_apply(g, KAPPA, to_dev(pe), THETA_AP, "f64", dagger=dagger).cpu().numpy()
        fp64_close(out, orc.deo(C2, ur, KAPPA, pe, THETA_AP, dagger=dagger))
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="d_cgnr_eo", inner_dtype="f64", theta=THETA_AP)
    x, res, rc = hrw.cg_solve(g, to_dev(psi), KAPPA, prm)
    assert rc == 0 and res[0]["true_rel_resid"] <= 1e-10
    d_res = rel(orc.dw(C2, ur, KAPPA, x.cpu().numpy(), THETA_AP), psi)
    assert abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res and d_res < 1e-8
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="d_eo", inner_dtype="bf16", theta=THETA_AP,
                           reliable_delta=hrw.RELIABLE_DELTA["bf16"])
    x, res, rc = hrw.bicgstab_solve(g, to_dev(psi), KAPPA, prm)
    assert rc == 0, res
    d_res = rel(orc.dw(C2, ur, KAPPA, x.cpu().numpy(), THETA_AP), psi)
    assert abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res and d_res < 1e-9
    g.close()


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_c2_bicgstab_residual_by_oracle(c2_field, inner):
    """The default workload's system solved by BiCGstab on D_hat (FP64, and FP32 inner fields with
    FP64 reliable updates): |b - D x| / |b| recomputed by the oracle."""
    ur, g = c2_field
    b = fx.gaussian_spinor(C2, 3, seed=3)
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="d_eo", inner_dtype=inner, theta=THETA_AP,
                           reliable_delta=hrw.RELIABLE_DELTA[inner])
    x, res, rc = hrw.bicgstab_solve(g, to_dev(b), KAPPA, prm)
    assert rc == 0 and res[0]["true_rel_resid"] <= 1e-10
    d_res = rel(orc.dw(C2, ur, KAPPA, x.cpu().numpy(), THETA_AP), b)
    assert abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res
    assert d_res < 1e-9


def test_c2_qmr_g5_residual_by_oracle(c2_field):
    """The default workload's system solved by QMR-g5 (FP64): |b - D x| / |b| recomputed by the oracle."""
    ur, g = c2_field
    b = fx.gaussian_spinor(C2, 3, seed=3)
    prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="d_eo", theta=THETA_AP)
    x, res, rc = hrw.qmr_g5_solve(g, to_dev(b), KAPPA, prm)
    assert rc == 0 and res[0]["true_rel_resid"] <= 1e-10
    d_res = rel(orc.dw(C2, ur, KAPPA, x.cpu().numpy(), THETA_AP), b)
    assert abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res
    assert d_res < 1e-9


def test_c2_clover_full_size(c2_field):
    """The clover workload (c_sw = 1): D_hat_sw in FP64 against the oracle, and the FP32-inner BiCGstab
    solve of D_sw x = b with |b - D_sw x| / |b| recomputed by the oracle."""
    ur, g = c2_field
    c = hrw.Clover(g, KAPPA, 1.0, dtypes=("f64", "f32"))
    try:
        pe = _even(C2, fx.gaussian_spinor(C2, 3, seed=5))
        fp64_close(hrw.dsw_eo_apply(c, to_dev(pe), THETA_AP, "f64").cpu().numpy(),
                   orc.dsw_eo(C2, ur, KAPPA, 1.0, pe, THETA_AP))
        b = fx.gaussian_spinor(C2, 3, seed=3)
        prm = hrw.solve_params(tol=1e-10, max_iter=5000, system="d_eo", inner_dtype="f32", theta=THETA_AP,
                               reliable_delta=hrw.RELIABLE_DELTA["f32"])
        x, res, rc = hrw.clover_bicgstab_solve(c, to_dev(b), prm)
        assert rc == 0 and res[0]["true_rel_resid"] <= 1e-10
        d_res = rel(orc.dsw(C2, ur, KAPPA, 1.0, x.cpu().numpy(), THETA_AP), b)
        assert abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res
        assert d_res < 1e-9
    finally:
        c.close()


@pytest.mark.parametrize("fused", [False, True], ids=["stored_links", "fused_rep_map"])
@pytest.mark.parametrize("nc,rep", [(2, "adj"), (4, "asym")])
def test_c3_operator_and_mixed_solve_full_size(nc, rep, fused):
    uf = fx.gauge_field(C3, nc, "thermal", seed=3, eps=0.3)
    ur = orc.rep_map(nc, rep, uf)
    g = hrw.Gauge(C3, nc, rep, to_dev(uf), dtypes=("f64", "f32"), fused=fused)
    del uf
    try:
        eta = _even(C3, fx.gaussian_spinor(C3, g.nr, seed=4))
        fp64_close(hrw.deo_apply(g, KAPPA, to_dev(eta), THETA_AP, "f64").cpu().numpy(),
                   orc.deo(C3, ur, KAPPA, eta, THETA_AP))
        prm = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype="f32",
                               reliable_every=50, reliable_delta=hrw.RELIABLE_DELTA["f32"], theta=THETA_AP)
        x, res, rc = hrw.cg_solve(g, to_dev(eta), KAPPA, prm)
        assert rc == 0 and res[0]["true_rel_resid"] <= 1e-10
        xe = x.cpu().numpy()
        ax = orc.deo(C3, ur, KAPPA, orc.deo(C3, ur, KAPPA, xe, THETA_AP), THETA_AP, dagger=True)
        r = rel(ax, eta)
        assert r <= 1.01e-10
        assert abs(r - res[0]["true_rel_resid"]) <= 1e-3 * r
    finally:
        g.close()


@pytest.fixture(scope="module")
def c4_field():
    """SU(3) two-index symmetric 32^4 near-thermal links and the 24 point-smeared even sources
    of the multi-source workload."""
    dims, nmax = C2, 24
    uf = fx.gauge_field(dims, 3, "thermal", seed=6, eps=0.3)
    ur = orc.rep_map(3, "sym", uf)
    g = hrw.Gauge(dims, 3, "sym", to_dev(uf), dtypes=("f64", "f32"))
    del uf
    src = np.stack([_even(dims, fx.point_smeared_sources(dims, g.nr, nmax, seed=7, which=[k]))[0]
                    for k in range(nmax)])
    yield ur, g, src
    g.close()


def test_c4_multi_source_full_size(c4_field):
    ur, g, src = c4_field
    dims = C2
    dev_src = to_dev(src)
    many32 = hrw.deo_apply(g, KAPPA, dev_src, THETA_AP, "f32").cpu().numpy()
    for k in (0, 11, 23):
        one = hrw.deo_apply(g, KAPPA, dev_src[k], THETA_AP, "f32").cpu().numpy()
        assert np.array_equal(many32[k], one)
    many64 = hrw.deo_apply(g, KAPPA, dev_src, THETA_AP, "f64").cpu().numpy()
    for k in (0, 23):
        fp64_close(many64[k], orc.deo(dims, ur, KAPPA, src[k], THETA_AP))


def test_c4_mixed_multi_source_solve_residual_by_oracle(c4_field):
    """The multi-source workload's solve as the benchmark runs it (24 sources in one call, FP32
    inner fields, FP64 reliable updates every 50 iterations or on a drop of |r| by the FP32
    trigger, tol 1e-10): every source converges, and for the first and last source the FP64
    residual |eta - D_hat^+ D_hat x| / |eta| recomputed by the oracle meets the tolerance and
    matches the reported one."""
    ur, g, src = c4_field
    dims = C2
    prm = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype="f32",
                           reliable_every=50, reliable_delta=hrw.RELIABLE_DELTA["f32"], theta=THETA_AP)
    x, res, rc = hrw.cg_solve(g, to_dev(src), [KAPPA] * len(src), prm)
    assert rc == 0, res
    assert all(r["true_rel_resid"] <= 1e-10 for r in res)
    x = x.cpu().numpy()
    for k in (0, len(src) - 1):
        ax = orc.deo(dims, ur, KAPPA, orc.deo(dims, ur, KAPPA, x[k], THETA_AP), THETA_AP, dagger=True)
        r = rel(ax, src[k])
        assert r <= 1.01e-10, (k, r)
        assert abs(r - res[k]["true_rel_resid"]) <= 1e-3 * r, (k, r, res[k]["true_rel_resid"])
