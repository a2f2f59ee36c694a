"""The allocation-free D_hat entry point (hrw_deo_apply_noalloc), called through the C ABI,
against the workspace entry point hrw_deo_apply: the same kernels, so the results must be
equal bit for bit, and in FP64 within the operator tolerance of the oracle.  Two calls in a
row, the second on a smaller input (fewer sources, a smaller lattice, another representation),
show that the shared static scratch carries nothing from one call to the next."""

import ctypes

import numpy as np
import pytest
import torch

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_TW, fp64_close, setup, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(g, kappas, pe, dtype, dagger=False):
    lib = hrw.load()
    x = to_dev(pe)
    out = torch.full_like(x, float("nan"))
    n = len(kappas)
    rc = lib.hrw_deo_apply_noalloc(g.handle, (ctypes.c_double * n)(*kappas), (ctypes.c_double * 4)(*THETA_TW),
                                   hrw.DTYPES[dtype], n, int(dagger), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(0))
    assert rc == 0, lib.hrw_last_error().decode()
    torch.cuda.synchronize()
    return out.cpu().numpy()


CALLS = [  # (dims, nc, rep, n_rhs, dtype, dagger): each call smaller than the one before
    ((8, 8, 8, 8), 3, "fund", 3, "f64", False),
    ((4, 4, 2, 6), 2, "adj", 1, "f64", True),
]


@pytest.mark.parametrize("dtype2", ["f64", "f32"])
def test_noalloc_deo_equals_workspace_entry_on_consecutive_calls(dtype2):
    for k, (dims, nc, rep, n, dtype, dagger) in enumerate(CALLS):
        dtype = dtype if k == 0 else dtype2
        uf, ur, g = setup(dims, nc, rep, "thermal", seed=90 + k, dtypes=("f64", "f32"))
        pe = orc.split_eo(dims, fx.gaussian_spinor(dims, g.nr, seed=91 + k, n_rhs=n))[0]
        kappas = [0.12 + 0.004 * j for j in range(n)]
        got = _noalloc(g, kappas, pe, dtype, dagger)
        ref = hrw.deo_apply(g, kappas, to_dev(pe), THETA_TW, dtype, dagger).cpu().numpy()
        assert np.array_equal(got, ref), (k, dims)
        if dtype == "f64":
            for j in range(n):
                fp64_close(got[j], orc.deo(dims, ur, kappas[j], pe[j], THETA_TW, dagger))
        g.close()


def test_noalloc_refuses_more_than_its_scratch():
    dims = (16, 16, 16, 16)
    uf = fx.unit_gauge(dims, 3)
    g = hrw.Gauge(dims, 3, "fund", to_dev(uf), dtypes=("f64",))
    lib = hrw.load()
    n = 64  # 3 x 64 x 6.3 MB of FP64 half fields: beyond HRW_NOALLOC_SCRATCH_BYTES
    x = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    rc = lib.hrw_deo_apply_noalloc(g.handle, (ctypes.c_double * n)(*([0.1] * n)), (ctypes.c_double * 4)(*THETA_TW),
                                   0, n, 0, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr() + 64),
                                   ctypes.c_void_p(0))
    assert rc == hrw.ENOMEM and "static scratch" in lib.hrw_last_error().decode()
    g.close()
