"""The spin basis the library stores spinor fields in, for the tests' error bounds.

The library holds q = T psi, psi in the chiral basis of the oracle and T acting on the spin
pairs (s, s + 2) of every colour as q_s = psi_s - psi_{s+2}, q_{s+2} = psi_s + psi_{s+2}
(s = 0, 1).  T is sqrt(2) times a unitary map; the operator on q is T D T^-1, whose gamma
matrices are T g T^-1: g_1..g_3 unchanged and g_0 = diag(1, 1, -1, -1).  The conversions
below use the FP64 operations of the library's packing and unpacking, in the same order, so
that a test can reproduce the stored input and recover the stored output exactly.

The spin index is the second-to-last axis of every spinor array ([..., 4, N_R]).
"""

import numpy as np

import oracle as orc


def to_storage(psi):
    """q = T psi in FP64: q_s = psi_s - psi_{s+2}, q_{s+2} = psi_s + psi_{s+2}."""
    p = np.asarray(psi)
    up, dn = p[..., 0:2, :], p[..., 2:4, :]
    return np.concatenate([up - dn, up + dn], axis=-2)


def to_chiral(q):
    """psi = T^-1 q in FP64: psi_s = (q_s + q_{s+2}) / 2, psi_{s+2} = (q_{s+2} - q_s) / 2."""
    q = np.asarray(q)
    a, b = q[..., 0:2, :], q[..., 2:4, :]
    return np.concatenate([(b + a) * 0.5, (b - a) * 0.5], axis=-2)


def storage_matrix():
    """T as a 4 x 4 spin matrix."""
    i2 = np.eye(2)
    return np.block([[i2, -i2], [i2, i2]]).astype(complex)


def storage_matrix_inverse():
    """T^-1 = (1/2) [[1, 1], [-1, 1]] on the spin pairs, as a 4 x 4 spin matrix."""
    i2 = np.eye(2)
    return 0.5 * np.block([[i2, i2], [-i2, i2]]).astype(complex)


def storage_gammas():
    """T g_mu T^-1 for mu = 0..3 (the gamma matrices of the operator on stored fields)."""
    t, ti = storage_matrix(), storage_matrix_inverse()
    return [t @ orc.gamma(mu) @ ti for mu in range(4)]


def stored(dtype, psi):
    """What the library stores for the canonical FP64 field psi in format dtype: the
    storage-basis components, formed in FP64 and rounded to nearest even."""
    return orc.round_to(dtype, to_storage(psi))
