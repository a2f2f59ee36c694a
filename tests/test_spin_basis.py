"""Pins of the storage spin basis the GPU tests check their bounds in (spin_basis) and of the
oracle's absolute-value hops evaluated with its gamma matrices (the `gammas` argument of
oracle.hop_abs and oracle.hop_abs_real).

The storage basis is q = T psi with q_s = psi_s - psi_{s+2}, q_{s+2} = psi_s + psi_{s+2}.  What
pins it: the Clifford algebra of the transformed matrices and their closed form (g_0 diagonal,
g_1..g_3 unchanged, g_5 the exchange of the spin pairs); the round trip; and the transformed
hop T H T^-1 q, computed through the oracle's chiral hop, bounded by the absolute-value hops of
the new basis, with their free-field closed form.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from spin_basis import storage_gammas, storage_matrix, storage_matrix_inverse, to_chiral, to_storage

THETA_TW = (np.pi, 0.7, -0.4, 1.3)


def test_transformed_gammas_closed_form_and_clifford_algebra():
    g = storage_gammas()
    assert np.array_equal(g[0], np.diag([1, 1, -1, -1]).astype(complex))
    for mu in (1, 2, 3):
        assert np.array_equal(g[mu], orc.gamma(mu))
    for mu in range(4):
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * (mu == nu) * np.eye(4), atol=0)
    t, ti = storage_matrix(), storage_matrix_inverse()
    g5 = t @ orc.gamma(4) @ ti
    assert np.array_equal(g5, np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]]))
    assert np.array_equal(g5, g[0] @ g[1] @ g[2] @ g[3])
    # T is sqrt(2) times a unitary map
    assert np.array_equal(t.conj().T @ t, 2 * np.eye(4))


def test_conversions_are_t_and_its_inverse():
    psi = fx.gaussian_spinor((2, 2, 2, 4), 3, seed=3)
    t = storage_matrix()
    assert np.allclose(to_storage(psi), np.einsum("st,...tc->...sc", t, psi), rtol=0, atol=1e-15)
    # dyadic values: every FP64 sum and halving is exact, so the round trip is the identity
    d = np.round(psi * 1024) / 1024
    assert np.array_equal(to_chiral(to_storage(d)), d)
    assert np.array_equal(to_storage(to_chiral(d)), d)


def _hop_stored(dims, ur, q, dagger=False):
    """T H T^-1 q through the oracle's chiral hop."""
    return to_storage(orc.hop(dims, ur, to_chiral(q), THETA_TW, dagger))


@pytest.mark.parametrize("dagger", [False, True])
def test_abs_hops_in_the_storage_basis_bound_the_transformed_hop(dagger):
    dims = (2, 2, 2, 4)
    uf = fx.gauge_field(dims, 3, "haar", seed=5)
    ur = orc.rep_map(3, "fund", uf)
    q = fx.gaussian_spinor(dims, 3, seed=6)
    gs = storage_gammas()
    h = _hop_stored(dims, ur, q, dagger)
    b = orc.hop_abs_real(dims, ur, q, THETA_TW, dagger, gammas=gs)
    assert np.all(np.abs(h.real) <= b.real * (1 + 1e-12)) and np.all(np.abs(h.imag) <= b.imag * (1 + 1e-12))
    assert np.all(np.abs(h) <= orc.hop_abs(dims, np.abs(ur), np.abs(q), gammas=gs, dagger=dagger) * (1 + 1e-12))
    # brute force: the real embedding of T H T^-1 column by column
    n = q.size
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        cols.append(_hop_stored(dims, ur, e.reshape(q.shape), dagger).reshape(-1))
    hm = np.stack(cols, axis=1)
    pr, pi_ = np.abs(q.real).reshape(-1), np.abs(q.imag).reshape(-1)
    bf = b.reshape(-1)
    assert np.all(np.abs(hm.real) @ pr + np.abs(hm.imag) @ pi_ <= bf.real * (1 + 1e-12))
    assert np.all(np.abs(hm.imag) @ pr + np.abs(hm.real) @ pi_ <= bf.imag * (1 + 1e-12))


@pytest.mark.parametrize("dagger", [False, True])
def test_abs_hop_storage_basis_free_field_closed_form(dagger):
    """Unit links, zero phases, a real non-negative field: along mu = 0 the forward hop of H
    keeps 2 q_{2,3}(x + 0) in spins 2, 3 and the backward hop 2 q_{0,1}(x - 0) in spins 0, 1
    (H^+ the other way round); mu = 1..3 keep the chiral pattern."""
    dims = (2, 2, 2, 4)
    unit = fx.unit_gauge(dims, 3)
    pos = np.abs(fx.gaussian_spinor(dims, 3, seed=7).real)
    b = orc.hop_abs_real(dims, unit, pos, dagger=dagger, gammas=storage_gammas())
    p4 = pos.reshape(tuple(dims) + (4, 3))
    partner = {1: [3, 2, 1, 0], 2: [3, 2, 1, 0], 3: [2, 3, 0, 1]}
    er = np.zeros_like(p4)
    ei = np.zeros_like(p4)
    for mu in (1, 2, 3):
        for sh in (-1, 1):
            q = np.roll(p4, sh, axis=mu)
            er += q + (q[..., partner[mu], :] if mu == 2 else 0)
            ei += q[..., partner[mu], :] if mu in (1, 3) else 0
    fwd, bwd = np.roll(p4, -1, axis=0), np.roll(p4, 1, axis=0)
    lo, hi = (slice(2, 4), slice(0, 2)) if not dagger else (slice(0, 2), slice(2, 4))
    er[..., lo, :] += 2 * fwd[..., lo, :]
    er[..., hi, :] += 2 * bwd[..., hi, :]
    assert np.allclose(b.real, er.reshape(pos.shape), rtol=1e-14)
    assert np.allclose(b.imag, ei.reshape(pos.shape), rtol=1e-14, atol=0)
    # column sums of |1 -+ g|: 2 for every spin along mu = 1..3 (both hops), along mu = 0 2 for
    # the kept half and 0 for the other: 12 + 2 times the field's sum
    ha = orc.hop_abs(dims, np.abs(unit), pos, gammas=storage_gammas(), dagger=dagger)
    assert np.allclose(ha.sum(), 14 * pos.sum(), rtol=1e-12)


def test_chiral_default_unchanged():
    """Without gammas the absolute-value hops are the chiral ones, and in the chiral basis H and
    H^+ give the same hop_abs."""
    dims = (2, 2, 2, 4)
    ur = orc.rep_map(2, "adj", fx.gauge_field(dims, 2, "haar", seed=9))
    p = np.abs(fx.gaussian_spinor(dims, 3, seed=10))
    a = orc.hop_abs(dims, np.abs(ur), p)
    assert np.array_equal(a, orc.hop_abs(dims, np.abs(ur), p, dagger=True))
    chiral = [orc.gamma(mu) for mu in range(4)]
    assert np.array_equal(a, orc.hop_abs(dims, np.abs(ur), p, gammas=chiral))
    q = fx.gaussian_spinor(dims, 3, seed=11)
    assert np.array_equal(orc.hop_abs_real(dims, ur, q, THETA_TW), orc.hop_abs_real(dims, ur, q, THETA_TW, gammas=chiral))
