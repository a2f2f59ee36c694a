"""Shared setup for the GPU parity tests (inputs from fixtures, references from oracle)."""

import numpy as np
import torch

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

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


def lowprec_bound(dims, ur_r, psi_r, kappa, nr, theta=THETA_TW, dagger=False):
    """Per real component, the a-priori bound of an FP32 evaluation of D_W (or D_W^+)
    on the rounded inputs: gamma_m (|psi| + kappa |H||psi|) with |H||psi| the sum of the
    absolute values of the real monomials (oracle.hop_abs_real) and m from
    hop_rounding_count (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1,
    3.6).  Returned as one complex array: real part for the real components, imaginary
    part for the imaginary ones."""
    hr = orc.hop_abs_real(dims, ur_r, psi_r, theta, dagger)
    gm = orc.gamma_k(hop_rounding_count(nr), U32)
    p = np.asarray(psi_r)
    return gm * (np.abs(p.real) + kappa * hr.real) + 1j * gm * (np.abs(p.imag) + kappa * hr.imag)


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


def bound_check(dims, ur_r, psi_r, kappa, out, ref, nr, unit_out, theta=THETA_TW, dagger=False):
    """A low-precision D_W apply against the oracle's FP64 D_W on the same rounded inputs,
    per real component within lowprec_bound, plus one rounding to the output format
    for 16-bit storage (FP32 output: unit_out is the FP32 unit, a harmless extra)."""
    return check_real_bound(out, ref, lowprec_bound(dims, ur_r, psi_r, kappa, nr, theta, dagger), unit_out)
