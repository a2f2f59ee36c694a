"""GPU parity of the clover-improved operator (HIP library through its C ABI) against the CPU oracle.

Tolerances:
  * FP64: l2 relative <= 1e-13 and componentwise <= 1e-12 max|ref| (as every FP64 operator).
  Every FP32 bound is checked in the library's storage spin basis (spin_basis: q = T psi, g_0
  diagonal), where the block products run as u = (q_s + q_{s+2}) / 2, d = (q_{s+2} - q_s) / 2,
  then (A_+ u - A_- d, A_+ u + A_- d) with the chiral blocks A_+-.
  * FP32 D_sw: the kernel applies the FP32-rounded clover blocks A_r (built in FP64, rounded once)
    and the FP32-rounded links to the stored input q_r; the reference is A_r psi_r - kappa H(U_r)
    psi_r in FP64 on psi_r = T^-1 q_r and the difference must sit inside
    gamma_k (|T A_r T^-1||q_r| + kappa |H'||q_r|) + u |ref| with k = 4 N_R + 20 (a hop of
    2 N_R + 16 operations per component plus a block product of 2 N_R and the two conversions),
    u = 2^-24.
  * FP32 D_hat_sw = A_ee psi - kappa^2 H_eo A_oo^-1 H_oe psi, evaluated in four FP32 stages (plain
    hop t1 = H_oe psi, stored; t2 = A_oo^-1 t1, stored; s = A_ee psi, stored; s - kappa^2 H_eo t2):
    per real component against the FP64 value on the stored input and rounded links, with the
    FP64 blocks of the oracle, within the stages' a-priori bounds propagated through the later
    stages (dhat_sw_bound below).
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, THETA_TW, U32, check_stored, fp64_close, pair_slack, rel, stored_input, to_dev
from spin_basis import storage_gammas, to_storage

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 2, 4), 2, "fund"),
    ((4, 2, 4, 4), 3, "fund"),
    ((2, 2, 2, 6), 3, "fund"),     # ragged half field
    ((4, 4, 2, 4), 2, "adj"),
    ((2, 4, 4, 4), 3, "sym"),
    ((4, 2, 2, 4), 4, "asym"),
    ((8, 8, 8, 8), 3, "fund"),     # several tiles
]
KAPPA, CSW = 0.13, 1.25


def ids(c):
    return f"{'x'.join(map(str, c[0]))}-su{c[1]}-{c[2]}"


def setup(dims, nc, rep, dtypes=("f64", "f32"), seed=41):
    uf = fx.gauge_field(dims, nc, "haar", seed=seed)
    ur = orc.rep_map(nc, rep, uf)
    g = hrw.Gauge(dims, nc, rep, to_dev(uf), dtypes=dtypes)
    c = hrw.Clover(g, KAPPA, CSW, dtypes=tuple(d for d in dtypes if d in ("f64", "f32")))
    return ur, g, c


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_clover_f64_operators(case):
    dims, nc, rep = case
    ur, g, c = setup(dims, nc, rep, dtypes=("f64",))
    psi = fx.gaussian_spinor(dims, g.nr, seed=42)
    for dagger in (False, True):
        out = hrw.dsw_apply(c, to_dev(psi), THETA_TW, "f64", dagger=dagger).cpu().numpy()
        fp64_close(out, orc.dsw(dims, ur, KAPPA, CSW, psi, THETA_TW, dagger=dagger))
    pe = orc.split_eo(dims, psi)[0]
    for dagger in (False, True):
        out = hrw.dsw_eo_apply(c, to_dev(pe), THETA_TW, "f64", dagger=dagger).cpu().numpy()
        fp64_close(out, orc.dsw_eo(dims, ur, KAPPA, CSW, pe, THETA_TW, dagger=dagger))


@pytest.mark.parametrize("case", CASES[:6], ids=ids)
def test_clover_f32_within_bound(case):
    dims, nc, rep = case
    ur, g, c = setup(dims, nc, rep, dtypes=("f64", "f32"), seed=43)
    nr = g.nr
    psi = fx.gaussian_spinor(dims, nr, seed=44)
    ur_r = orc.round_to("f32", ur)
    q_r, psi_r = stored_input("f32", psi)
    a_r = orc.round_to("f32", orc.clover(dims, ur, KAPPA, CSW))
    out = hrw.dsw_apply(c, to_dev(psi), THETA_TW, "f32").cpu().numpy()
    flat = psi_r.reshape(len(psi_r), 4 * nr)
    ref = to_storage(np.einsum("sij,sj->si", a_r, flat).reshape(psi.shape)
                     - KAPPA * orc.hop(dims, ur_r, psi_r, THETA_TW))
    absa = _abs_block_stored(np.abs(a_r), np.abs(q_r))
    bound = orc.gamma_k(4 * nr + 20, U32) * (absa + KAPPA * orc.hop_abs(dims, np.abs(ur_r), np.abs(q_r),
                                                                       gammas=storage_gammas()))
    bound += pair_slack(bound) + U32 * np.abs(ref) + 1e-300
    assert np.max(np.abs(to_storage(out) - ref) / bound) <= 1.0
    pe = orc.split_eo(dims, psi)[0]
    out = hrw.dsw_eo_apply(c, to_dev(pe), THETA_TW, "f32").cpu().numpy()
    pq_r, pe_r = stored_input("f32", pe)
    ref, bound = dhat_sw_bound(dims, ur_r, orc.clover(dims, ur, KAPPA, CSW), pq_r, pe_r, nr)
    check_stored(out, ref, bound, 0.0)
    assert rel(out, orc.dsw_eo(dims, ur, KAPPA, CSW, pe, THETA_TW)) <= 1e-5


def _absmul(m, x):
    """Per real component of m x (m [n][k][k], x [n][k], complex): the sum of the absolute
    values of its real monomials, coded as one complex array (real part for the real
    components, imaginary part for the imaginary ones)."""
    mr, mi, xr, xi = np.abs(m.real), np.abs(m.imag), np.abs(x.real), np.abs(x.imag)
    mul = lambda a, b: np.einsum("sij,sj->si", a, b)
    return mul(mr, xr) + mul(mi, xi) + 1j * (mul(mi, xr) + mul(mr, xi))


def _pair_mean(x, part):
    """(|x_s| + |x_{s+2}|) / 2 per spin pair of a storage-basis array [n][4][nr], the bound
    of both chiral halves u and d the block products take (part: abs of the real or the
    imaginary parts, or the modulus)."""
    a, b = part(x[:, 0:2, :]), part(x[:, 2:4, :])
    return 0.5 * (a + b)


def _blocks_stored(m, h, mul):
    """Both output halves of the storage-basis block product from the halves' bound h
    [n][2][nr]: A_+ u -+ A_- d is bounded by |A_+| h + |A_-| h in either half."""
    n, _, nr = h.shape
    k = 2 * nr
    hf = h.reshape(n, k)
    p = (mul(m[:, :k, :k], hf) + mul(m[:, k:, k:], hf)).reshape(n, 2, nr)
    return np.concatenate([p, p], axis=1)


def _abs_block_stored(m_abs, q_abs):
    """|T A T^-1||q| by complex moduli (m_abs, q_abs: moduli, q in the storage basis)."""
    h = _pair_mean(q_abs, lambda z: z)
    return _blocks_stored(m_abs, h, lambda a, b: np.einsum("sij,sj->si", a, b))


def _absmul_stored(m, x):
    """_absmul of the storage-basis block product T m T^-1 x (x [n][4][nr] in the storage
    basis, m block diagonal in the chiral basis), as the library evaluates it."""
    h = _pair_mean(x, lambda z: np.abs(z.real)) + 1j * _pair_mean(x, lambda z: np.abs(z.imag))
    return _blocks_stored(m, h, _absmul)


def _hop_half_abs(dims, ur, half, out_parity):
    """oracle.hop_abs_real of an even/odd block in the storage basis: the input half embedded
    in the full lattice."""
    z = np.zeros_like(half)
    full = orc.merge_eo(dims, half, z) if out_parity == 1 else orc.merge_eo(dims, z, half)
    return orc.split_eo(dims, orc.hop_abs_real(dims, ur, full, THETA_TW, gammas=storage_gammas()))[out_parity]


def dhat_sw_bound(dims, ur_r, a64, pq_r, pe_r, nr):
    """FP64 reference of D_hat_sw on the stored input (pq_r in the storage basis, pe_r = the
    same in the chiral basis) and rounded links, and the per-real-component bound, in the
    storage basis, of the FP32 evaluation in the kernel's four stages (Higham, Accuracy and
    Stability of Numerical Algorithms, Sec. 3.1, 3.6), each stage's own rounding bound gamma_m
    times the absolute monomial sums of its computed inputs, plus the earlier stages' bounds
    carried through it:
      t1 = H_oe psi: the hop (projection 1, phase 3, link row 2 N_R, 7 additions) and the FP32
           store: m = 2 N_R + 12;
      t2 = A_oo^-1 t1, s = A_ee psi: the conversion to the chiral halves (1), the block entries
           rounded to FP32 (1), a 2 N_R complex product chain (4 N_R), the conversion back (1)
           and the store (1): m = 4 N_R + 4;
      out = s - kappa^2 H_eo t2: the hop and the epilogue (kappa^2 rounded, product,
           difference): m = 2 N_R + 14.
    Returns the reference in the chiral basis and the bound in the storage basis."""
    h, k = pe_r.shape[0], 4 * nr
    par = orc.parity_of_sites(dims)
    ae, ainv = a64[par == 0], np.linalg.inv(a64[par == 1])
    kk = KAPPA * KAPPA
    g = lambda m: orc.gamma_k(m, U32)
    cabs = lambda z: np.abs(z.real) + 1j * np.abs(z.imag)
    flat = lambda z: z.reshape(h, k)
    t1 = orc.hop_eo(dims, ur_r, pe_r, 1, THETA_TW)
    e1 = g(2 * nr + 12) * _hop_half_abs(dims, ur_r, pq_r, 1)
    t2 = np.einsum("sij,sj->si", ainv, flat(t1)).reshape(t1.shape)
    e2 = _absmul_stored(ainv, e1) + g(4 * nr + 4) * _absmul_stored(ainv, cabs(to_storage(t1)) + e1)
    sv = np.einsum("sij,sj->si", ae, flat(pe_r)).reshape(pe_r.shape)
    e3 = g(4 * nr + 4) * _absmul_stored(ae, pq_r)
    ref = sv - kk * orc.hop_eo(dims, ur_r, t2, 0, THETA_TW)
    e4 = (e3 + kk * _hop_half_abs(dims, ur_r, e2, 0)
          + g(2 * nr + 14) * (cabs(to_storage(sv)) + e3
                               + kk * _hop_half_abs(dims, ur_r, cabs(to_storage(t2)) + e2, 0)))
    return ref, e4


def test_clover_multi_rhs_and_limits():
    """Several right-hand sides in one call equal single calls bitwise; c_sw = 0 reproduces D_W
    bitwise; a clover term without FP32 blocks refuses FP32 applies."""
    dims = (4, 4, 4, 4)
    ur, g, c = setup(dims, 3, "fund")
    psi = fx.gaussian_spinor(dims, 3, seed=45, n_rhs=3)
    many = hrw.dsw_apply(c, to_dev(psi), THETA_AP, "f64").cpu().numpy()
    for k in range(3):
        assert np.array_equal(many[k], hrw.dsw_apply(c, to_dev(psi[k]), THETA_AP, "f64").cpu().numpy())
    pe = orc.split_eo(dims, psi)[0]
    many = hrw.dsw_eo_apply(c, to_dev(pe), THETA_AP, "f32").cpu().numpy()
    for k in range(3):
        assert np.array_equal(many[k], hrw.dsw_eo_apply(c, to_dev(pe[k]), THETA_AP, "f32").cpu().numpy())
    c0 = hrw.Clover(g, KAPPA, 0.0, dtypes=("f64",))
    a = hrw.dsw_apply(c0, to_dev(psi[0]), THETA_AP, "f64").cpu().numpy()
    fp64_close(a, orc.dw(dims, ur, KAPPA, psi[0], THETA_AP))
    with pytest.raises(hrw.HrwError) as e:
        hrw.dsw_apply(c0, to_dev(psi[0]), THETA_AP, "f32")
    assert e.value.code == hrw.EUNSUPPORTED


@pytest.mark.parametrize("inner", ["f64", "f32"])
@pytest.mark.parametrize("nc,rep,dims", [(3, "fund", (4, 4, 4, 8)), (2, "adj", (4, 4, 4, 4)),
                                         (4, "asym", (4, 4, 2, 4))])
def test_clover_bicgstab(inner, nc, rep, dims):
    """BiCGstab on D_hat_sw (and D_sw x = b through the Schur complement), FP64 and FP32 inner: the
    FP64 true residual recomputed by the oracle meets the tolerance and matches the reported one;
    the solution (unique) agrees with the oracle's BiCGstab (run to 1e-12) within 1e-7, i.e.
    cond(D_hat_sw) x 1e-10 for a condition number below 10^3 on these smooth fields."""
    uf = fx.gauge_field(dims, nc, "thermal", seed=46)
    ur = orc.rep_map(nc, rep, uf)
    g = hrw.Gauge(dims, nc, rep, to_dev(uf), dtypes=("f64", "f32"))
    c = hrw.Clover(g, KAPPA, CSW, dtypes=("f64", "f32"))
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, g.nr, seed=47))[0]
    prm = hrw.solve_params(tol=1e-10, system="dhat_eo", inner_dtype=inner, theta=THETA_AP,
                           reliable_delta=hrw.RELIABLE_DELTA[inner])
    x, res, rc = hrw.clover_bicgstab_solve(c, to_dev(be), prm)
    assert rc == 0, res
    x = x.cpu().numpy()
    r = rel(orc.dsw_eo(dims, ur, KAPPA, CSW, x, THETA_AP), be)
    assert r <= 1.01e-10 and abs(r - res[0]["true_rel_resid"]) <= 1e-3 * r + 1e-16
    xo, info = orc.bicgstab_sw(dims, ur, KAPPA, CSW, be, THETA_AP, orc.BICG_EO, tol=1e-12)
    assert info["status"] == 0 and rel(x, xo) <= 1e-7
    b = fx.gaussian_spinor(dims, g.nr, seed=48)
    prm = hrw.solve_params(tol=1e-10, system="d_eo", inner_dtype=inner, theta=THETA_AP,
                           reliable_delta=hrw.RELIABLE_DELTA[inner])
    x, res, rc = hrw.clover_bicgstab_solve(c, to_dev(b), prm)
    assert rc == 0, res
    x = x.cpu().numpy()
    d_res = rel(orc.dsw(dims, ur, KAPPA, CSW, x, THETA_AP), b)
    assert d_res <= 1e-9 and abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res + 1e-16
    xs, info = orc.solve_dsw_eo_bicgstab(dims, ur, KAPPA, CSW, b, THETA_AP, tol=1e-12)
    assert rel(x, xs) <= 1e-7


def test_clover_two_row_links():
    """The clover operator on an SU(3) fundamental field whose hops read two rows of each link:
    D_sw and D_hat_sw in FP64 against the oracle to 1e-13, and the FP32-inner BiCGstab solve of
    D_sw x = b with |b - D_sw x| / |b| recomputed by the oracle."""
    dims = (4, 4, 4, 8)
    uf = fx.gauge_field(dims, 3, "thermal", seed=49)
    ur = orc.rep_map(3, "fund", uf)
    g = hrw.Gauge(dims, 3, "fund", to_dev(uf), dtypes=("f64", "f32"), two_rows=True)
    c = hrw.Clover(g, KAPPA, CSW, dtypes=("f64", "f32"))
    psi = fx.gaussian_spinor(dims, 3, seed=50)
    fp64_close(hrw.dsw_apply(c, to_dev(psi), THETA_AP, "f64").cpu().numpy(),
               orc.dsw(dims, ur, KAPPA, CSW, psi, THETA_AP))
    pe = orc.split_eo(dims, psi)[0]
    fp64_close(hrw.dsw_eo_apply(c, to_dev(pe), THETA_AP, "f64").cpu().numpy(),
               orc.dsw_eo(dims, ur, KAPPA, CSW, pe, THETA_AP))
    prm = hrw.solve_params(tol=1e-10, system="d_eo", inner_dtype="f32", theta=THETA_AP,
                           reliable_delta=hrw.RELIABLE_DELTA["f32"])
    x, res, rc = hrw.clover_bicgstab_solve(c, to_dev(psi), prm)
    assert rc == 0, res
    d_res = rel(orc.dsw(dims, ur, KAPPA, CSW, x.cpu().numpy(), THETA_AP), psi)
    assert d_res <= 1e-9 and abs(d_res - res[0]["d_rel_resid"]) <= 1e-3 * d_res + 1e-16

