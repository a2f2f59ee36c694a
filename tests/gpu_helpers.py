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


def bound_check(dims, ur_r, psi_r, kappa, out, ref, nr, unit_out):
    """|out - ref| <= gamma_k (|psi| + kappa |H||psi|) + unit_out |ref| componentwise (a-priori bound of a
    low-precision D_W evaluation on the rounded inputs; k = 2 N_R + 16)."""
    bound = orc.gamma_k(2 * nr + 16, U32) * (np.abs(psi_r) + kappa * orc.hop_abs(dims, np.abs(ur_r), np.abs(psi_r)))
    bound = bound + unit_out * np.abs(ref) + 1e-300
    excess = np.abs(out - ref) / bound
    assert np.max(excess) <= 1.0, np.max(excess)
