"""GPU parity of the SU(3) fundamental hop that reads two rows of each link and rebuilds the third
(gauge fields created with HRW_STORE_SU3_TWO_ROWS) against the CPU oracle.

Tolerances:
  * FP64: the same as the stored-link path (l2 relative <= 1e-13, componentwise <= 1e-12 max|ref|);
    the rebuilt row conj(u_0 x u_1) equals the stored one to the unitarity of the FP64 links.
  * FP32 arithmetic on FP32 / BF16 / FP16 storage: the oracle applies FP64 D with the rounded stored
    links U_r (all three rows) to the stored input (its storage-basis components rounded; every
    bound is checked per real component of that basis, gpu_helpers).  Besides the hop's own bound
    gamma_m (|psi| + kappa |H||psi|) per real component (m = 2 N_R + 14, u = 2^-24,
    gpu_helpers.lowprec_bound), the rebuilt row differs from the
    rounded stored one: every entry is a difference of two products of rounded entries of modulus
    <= 1, so |row_2' - round(row_2)| <= 4 sqrt(2) u_s + sqrt(2) u_s + 2 gamma_2 <= 8 u_s + 8 u per
    entry (u_s the storage unit roundoff), which enters as kappa (8 u_s + 8 u) |H|_1 |psi| with |H|_1
    the hop with every link entry set to 1; plus one rounding of the stored output.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import (THETA_AP, THETA_TW, U32, U_BF16, U_F16, check_stored, fp64_close, lowprec_bound, rel,
                         stored_input, to_dev)
from spin_basis import storage_gammas

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 2, 4), "haar"),
    ((2, 2, 2, 6), "haar"),      # ragged half field (24 sites)
    ((4, 2, 4, 4), "thermal"),
    ((8, 8, 8, 8), "thermal"),   # several tiles
    ((6, 4, 4, 8), "haar"),
]
UNIT = {"f32": U32, "bf16": U_BF16, "f16": U_F16}


def ids(c):
    return f"{'x'.join(map(str, c[0]))}-{c[1]}"


def two_row_setup(dims, kind, dtypes=("f64", "f32", "bf16", "f16"), seed=21):
    uf = fx.gauge_field(dims, 3, kind, seed=seed)
    ur = orc.rep_map(3, "fund", uf)
    g = hrw.Gauge(dims, 3, "fund", to_dev(uf), dtypes=dtypes, two_rows=True)
    return uf, ur, g


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_two_rows_f64_operators(case):
    dims, kind = case
    uf, ur, g = two_row_setup(dims, kind, dtypes=("f64",))
    kappa = 0.131
    psi = fx.gaussian_spinor(dims, 3, seed=22)
    for dagger in (False, True):
        out = hrw.dw_apply(g, kappa, to_dev(psi), THETA_TW, "f64", dagger=dagger).cpu().numpy()
        fp64_close(out, orc.dw(dims, ur, kappa, psi, THETA_TW, dagger=dagger))
    pe, po = orc.split_eo(dims, psi)
    for dagger in (False, True):
        out = hrw.deo_apply(g, kappa, to_dev(pe), THETA_TW, "f64", dagger=dagger).cpu().numpy()
        fp64_close(out, orc.deo(dims, ur, kappa, pe, THETA_TW, dagger=dagger))
    fp64_close(hrw.hop_eo(g, 1, to_dev(pe), THETA_TW, "f64").cpu().numpy(), orc.hop_eo(dims, ur, pe, 1, THETA_TW))
    fp64_close(hrw.hop_eo(g, 0, to_dev(po), THETA_TW, "f64").cpu().numpy(), orc.hop_eo(dims, ur, po, 0, THETA_TW))


@pytest.mark.parametrize("case", CASES[:4], ids=ids)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_two_rows_low_precision_within_bound(case, dtype):
    dims, kind = case
    uf, ur, g = two_row_setup(dims, kind, dtypes=(dtype,), seed=23)
    kappa = 0.137
    psi = fx.gaussian_spinor(dims, 3, seed=24)
    ur_r = orc.round_to(dtype, ur)
    q_r, psi_r = stored_input(dtype, psi)
    out = hrw.dw_apply(g, kappa, to_dev(psi), THETA_TW, dtype).cpu().numpy()
    ref = orc.dw(dims, ur_r, kappa, psi_r, THETA_TW)
    ones = np.ones_like(np.abs(ur_r))
    row2 = (8 * UNIT[dtype] + 8 * U32) * kappa * orc.hop_abs(dims, ones, np.abs(q_r), gammas=storage_gammas())
    check_stored(out, ref, lowprec_bound(dims, ur_r, q_r, kappa, 3) + row2 * (1 + 1j),
                 0.0 if dtype == "f32" else UNIT[dtype])
    assert rel(out, orc.dw(dims, ur, kappa, psi, THETA_TW)) < {"f32": 1e-6, "bf16": 2e-2, "f16": 3e-3}[dtype]


def test_two_rows_match_stored_path_and_multi_source_keeps_stored_links():
    """FP64 two-row and stored-link applies agree to rounding; with enough sources for the
    multi-source kernel a two-row field reads the stored rows (bitwise the result of a field
    without the flag)."""
    dims = (4, 4, 4, 4)
    uf = fx.gauge_field(dims, 3, "thermal", seed=25)
    gt = hrw.Gauge(dims, 3, "fund", to_dev(uf), dtypes=("f64", "f32"), two_rows=True)
    gs = hrw.Gauge(dims, 3, "fund", to_dev(uf), dtypes=("f64", "f32"))
    pe = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=26, n_rhs=24))[0]
    a = hrw.deo_apply(gt, 0.13, to_dev(pe[0]), THETA_AP, "f64").cpu().numpy()
    b = hrw.deo_apply(gs, 0.13, to_dev(pe[0]), THETA_AP, "f64").cpu().numpy()
    assert rel(a, b) < 1e-14
    for dt in ("f64", "f32"):
        many_t = hrw.deo_apply(gt, 0.13, to_dev(pe), THETA_AP, dt).cpu().numpy()
        many_s = hrw.deo_apply(gs, 0.13, to_dev(pe), THETA_AP, dt).cpu().numpy()
        assert np.array_equal(many_t, many_s), dt


def test_two_rows_solves():
    """CG (FP64 and FP32-inner mixed) and BiCGstab (FP64 and BF16 inner) on a two-row field: the
    true residual recomputed by the oracle meets the tolerance and the solution matches the
    oracle's within cond x tol."""
    dims, kappa = (4, 4, 4, 8), 0.13
    uf, ur, g = two_row_setup(dims, "thermal", dtypes=("f64", "f32", "bf16"), seed=27)
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=28))[0]
    xo, info = orc.cg(dims, ur, kappa, b, THETA_AP, orc.SYSTEM_EO, tol=1e-10)
    lo, hi = orc.lanczos_extremes(info["alpha"], info["beta"])
    for inner in ("f64", "f32"):
        prm = hrw.solve_params(tol=1e-10, system="ddag_d_eo", inner_dtype=inner, theta=THETA_AP,
                               reliable_delta=hrw.RELIABLE_DELTA[inner])
        x, res, rc = hrw.cg_solve(g, to_dev(b), kappa, prm)
        x = x.cpu().numpy()
        assert rc == 0, res
        ax = orc.deo(dims, ur, kappa, orc.deo(dims, ur, kappa, x, THETA_AP), THETA_AP, dagger=True)
        assert rel(ax, b) <= 1.01e-10
        assert rel(x, xo) <= 2 * (hi / lo) * 1e-10
    for inner in ("f64", "bf16"):
        prm = hrw.solve_params(tol=1e-10, system="dhat_eo", inner_dtype=inner, theta=THETA_AP,
                               reliable_delta=hrw.RELIABLE_DELTA[inner])
        y, res, rc = hrw.bicgstab_solve(g, to_dev(b), kappa, prm)
        assert rc == 0, res
        r = rel(orc.deo(dims, ur, kappa, y.cpu().numpy(), THETA_AP), b)
        assert r <= 1.01e-10 and abs(r - res[0]["true_rel_resid"]) <= 1e-3 * r + 1e-16


def test_two_rows_refuse_links_that_are_not_special_unitary():
    """Gauge creation with two-row storage measures max |u_2 - conj(u_0 x u_1)| and refuses a
    field with a U(3) link (unitary, det = exp(3 i a) != 1) or a non-unitary field beyond the
    tolerance of the stored formats; the same links without the flag are accepted."""
    dims = (4, 4, 2, 4)
    uf = fx.gauge_field(dims, 3, "haar", seed=27)
    hrw.Gauge(dims, 3, "fund", to_dev(uf), dtypes=("f64",), two_rows=True).close()
    u3 = uf.copy()
    u3[5, 2] *= np.exp(0.15j)                 # one link leaves SU(3) for U(3)
    stretched = uf * (1 + 1e-9)               # every link 1e-9 off unitarity
    for bad, dtypes in ((u3, ("f64",)), (u3, ("f32",)), (stretched, ("f64", "f32"))):
        with pytest.raises(hrw.HrwError) as e:
            hrw.Gauge(dims, 3, "fund", to_dev(bad), dtypes=dtypes, two_rows=True)
        assert e.value.code == hrw.EINVAL and "special unitary" in str(e.value)
        hrw.Gauge(dims, 3, "fund", to_dev(bad), dtypes=dtypes).close()
    # 1e-9 is within four FP32 units: accepted when only FP32 links are stored
    hrw.Gauge(dims, 3, "fund", to_dev(stretched), dtypes=("f32",), two_rows=True).close()
