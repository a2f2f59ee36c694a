"""Shared setup for the GPU parity tests (inputs from fixtures, references from oracle).

The low-precision bounds are checked in the library's storage spin basis (spin_basis): the
library rounds the storage-basis components of its input, evaluates the operator there and
returns the chiral components of its stored output, which a test recovers exactly.
"""

import numpy as np
import torch

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw
from spin_basis import storage_gammas, stored, to_chiral, to_storage

THETA_AP = (np.pi, 0.0, 0.0, 0.0)
THETA_TW = (np.pi, 0.7, -0.4, 1.3)
U32, U_BF16, U_F16 = 2.0 ** -24, 2.0 ** -8, 2.0 ** -11


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def setup(dims, nc, rep, kind="haar", seed=1, dtypes=("f64", "f32", "bf16", "f16"), eps=0.3):
    uf = fx.gauge_field(dims, nc, kind, seed=seed, eps=eps)
    ur = orc.rep_map(nc, rep, uf)
    g = hrw.Gauge(dims, nc, rep, to_dev(uf), dtypes=dtypes)
    return uf, ur, g


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def fp64_close(out, ref):
    """FP64 operator parity: l2 relative <= 1e-13 and componentwise <= 1e-12 max|ref|."""
    assert rel(out, ref) <= 1e-13, rel(out, ref)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def hop_rounding_count(nr):
    """Roundings an FP32 evaluation of D_W = 1 - kappa H applies to one real monomial of
    a hop term, counted along the kernel's evaluation order: the spin projection (1
    addition), the boundary phase on a wrap (the phase rounded to FP32, a product and
    a sum: 3), the complex link row times the half-spinor as a chain of 2 N_R fused
    multiply-adds (2 N_R), the sum over the 8 directions (7 additions; the first goes
    into zero) and the epilogue psi - kappa acc (kappa rounded to FP32, a product and
    a difference: 3).  The self term passes through one rounding."""
    return 2 * nr + 14


def lowprec_bound(dims, ur_r, q_r, kappa, nr, theta=THETA_TW, dagger=False):
    """Per real component of the storage basis, the a-priori bound of an FP32 evaluation of
    D_W (or D_W^+) on the stored input q_r: gamma_m (|q| + kappa |H'||q|) with |H'||q| the sum
    of the absolute values of the real monomials of the hop in that basis
    (oracle.hop_abs_real with its gamma matrices) and m from hop_rounding_count (Higham,
    Accuracy and Stability of Numerical Algorithms, Sec. 3.1, 3.6).  Returned as one complex
    array: real part for the real components, imaginary part for the imaginary ones."""
    hr = orc.hop_abs_real(dims, ur_r, q_r, theta, dagger, gammas=storage_gammas())
    gm = orc.gamma_k(hop_rounding_count(nr), U32)
    p = np.asarray(q_r)
    return gm * (np.abs(p.real) + kappa * hr.real) + 1j * gm * (np.abs(p.imag) + kappa * hr.imag)


def pair_slack(bound, rel=1e-12):
    """rel times the bound summed over each spin pair (s, s + 2): room for the FP64 rounding
    of the oracle's reference and of the basis conversions (relative 1e-16, four orders
    below the FP32 bounds it is added to), which mix the two components of a pair."""
    b = np.asarray(bound)
    return rel * (b + np.concatenate([b[..., 2:4, :], b[..., 0:2, :]], axis=-2))


def check_real_bound(out, ref, bound, unit_out):
    """|Re(out - ref)| <= Re bound + unit_out (|Re ref| + Re bound), the same for the
    imaginary parts; unit_out bounds the final rounding to the output format (0 in FP32
    arithmetic with FP32 output: the bound already covers it)."""
    br = bound.real + unit_out * (np.abs(ref.real) + bound.real) + 1e-300
    bi = bound.imag + unit_out * (np.abs(ref.imag) + bound.imag) + 1e-300
    d = out - ref
    excess = max(np.max(np.abs(d.real) / br), np.max(np.abs(d.imag) / bi))
    assert excess <= 1.0, excess
    return excess


def check_stored(out, ref, bound, unit_out):
    """check_real_bound in the storage basis: out is the library's result in the chiral
    basis (its stored output recovered exactly by to_storage), ref the oracle's FP64 value
    in the chiral basis and bound a storage-basis bound (widened by pair_slack)."""
    return check_real_bound(to_storage(out), to_storage(ref), bound + pair_slack(bound), unit_out)


def stored_input(dtype, psi):
    """(q_r, psi_r): the library's stored form of psi and the same field in the chiral basis
    (exact), the input the oracle's reference is evaluated on."""
    q_r = stored(dtype, psi)
    return q_r, to_chiral(q_r)


def bound_check(dims, ur_r, q_r, kappa, out, ref, nr, unit_out, theta=THETA_TW, dagger=False):
    """A low-precision D_W apply against the oracle's FP64 D_W on the same stored input
    (ref = D_W to_chiral(q_r)), per real component of the storage basis within
    lowprec_bound, plus one rounding to the output format for 16-bit storage (FP32 output:
    unit_out is the FP32 unit, a harmless extra)."""
    return check_stored(out, ref, lowprec_bound(dims, ur_r, q_r, kappa, nr, theta, dagger), unit_out)
