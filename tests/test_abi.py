"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hrw_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2405_19294_amd import hrw
    return hrw.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["hrw_rep_map", "hrw_gauge_create", "hrw_dw_apply", "hrw_hop_eo", "hrw_deo_apply",
                 "hrw_cg_solve", "hrw_workspace_size", "hrw_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_signatures_cover_header():
    from paper_2405_19294_amd import hrw
    assert set(hrw.SIGNATURES) == set(declared_functions())


def test_rep_dim_and_sizes(lib):
    from paper_2405_19294_amd import hrw
    assert hrw.rep_dim(3, "sym") == 6 and hrw.rep_dim(4, "asym") == 6 and hrw.rep_dim(2, "adj") == 3
    assert hrw.rep_dim(4, "adj") == 15
    # storage: two copies (one per parity block) of 4V links, 256-byte aligned
    dims = (4, 4, 4, 4)
    n = hrw.gauge_storage_size(dims, 3, "fund", ("f64",))
    assert n >= 2 * 4 * 256 * 9 * 16
    n2 = hrw.gauge_storage_size(dims, 3, "fund", ("f64", "f32"))
    assert n2 > n
    p = hrw.solve_params()
    assert hrw.workspace_size(dims, 3, "fund", 2, p) > hrw.workspace_size(dims, 3, "fund", 1, p)
    assert hrw.workspace_size(dims, 3, "fund", 1) > 0


def test_validation_errors(lib):
    from paper_2405_19294_amd import hrw
    dims = (4, 4, 4, 4)
    with pytest.raises(hrw.HrwError) as e:
        hrw.gauge_storage_size((4, 4, 3, 4), 3, "fund")
    assert e.value.code == hrw.EINVAL and "even" in str(e.value)
    with pytest.raises(hrw.HrwError) as e:
        hrw.gauge_storage_size(dims, 5, "fund")
    assert e.value.code == hrw.EUNSUPPORTED
    with pytest.raises(hrw.HrwError) as e:  # SU(4) adjoint: N_R = 15 has no hopping kernel
        hrw.gauge_storage_size(dims, 4, "adj")
    assert e.value.code == hrw.EUNSUPPORTED
    out = ctypes.c_void_p()
    rc = lib.hrw_gauge_create((ctypes.c_int * 4)(*dims), 3, 0, None, 1, None, 0, None, ctypes.byref(out))
    assert rc == hrw.EINVAL
    assert lib.hrw_last_error()
    rc = lib.hrw_dw_apply(None, 0.1, None, 0, 1, 0, None, None, None, 0, None)
    assert rc == hrw.EINVAL
    p = hrw.solve_params()
    p.tol = -1
    sz = ctypes.c_size_t()
    assert lib.hrw_workspace_size((ctypes.c_int * 4)(*dims), 3, 0, 1, ctypes.byref(p), ctypes.byref(sz)) == hrw.EINVAL
    assert lib.hrw_rep_map(3, 0, 10, None, None, None) == hrw.EINVAL
    assert lib.hrw_timing_read(7, None, None, None) == hrw.EINVAL


def test_bicgstab_systems_sizes_and_validation(lib):
    from paper_2405_19294_amd import hrw
    dims = (4, 4, 4, 4)
    cg = hrw.workspace_size(dims, 3, "fund", 1, hrw.solve_params(system="ddag_d_eo"))
    dhat = hrw.workspace_size(dims, 3, "fund", 1, hrw.solve_params(system="dhat_eo"))
    d = hrw.workspace_size(dims, 3, "fund", 1, hrw.solve_params(system="d_eo"))
    mixed = hrw.workspace_size(dims, 3, "fund", 1, hrw.solve_params(system="dhat_eo", inner_dtype="f32"))
    # FP32 inner fields take half the bytes of the FP64 ones; mixed mode adds an FP64 solution
    assert 0 < cg and 0 < dhat < d and 0 < mixed < dhat
    p = hrw.solve_params(system="dhat_eo")
    res = (hrw.SolveResult * 1)()
    k = (ctypes.c_double * 1)(0.13)
    assert lib.hrw_bicgstab_solve(None, ctypes.byref(p), 1, k, None, None, res, None, 0, None) == hrw.EINVAL
    bad = hrw.solve_params(system="dhat_eo")
    bad.system = 5
    sz = ctypes.c_size_t()
    assert lib.hrw_workspace_size((ctypes.c_int * 4)(*dims), 3, 0, 1, ctypes.byref(bad), ctypes.byref(sz)) == hrw.EINVAL


def test_fused_rep_map_storage_flag(lib):
    from paper_2405_19294_amd import hrw
    dims = (4, 4, 4, 4)
    base = hrw.gauge_storage_size(dims, 3, "sym", ("f64", "f32"))
    fused = hrw.gauge_storage_size(dims, 3, "sym", ("f64", "f32"), fused=True)
    # the fundamental blocks (N = 3) add N^2 / N_R^2 = 1/4 of the symmetric (N_R = 6) ones
    assert abs((fused - base) / base - 0.25) < 0.01
    for nc, rep in [(2, "adj"), (2, "sym"), (4, "asym")]:
        assert hrw.gauge_storage_size(dims, nc, rep, ("f32",), fused=True) > hrw.gauge_storage_size(dims, nc, rep, ("f32",))
    for nc, rep in [(3, "fund"), (3, "adj"), (3, "asym"), (4, "fund")]:
        with pytest.raises(hrw.HrwError) as e:
            hrw.gauge_storage_size(dims, nc, rep, ("f64",), fused=True)
        assert e.value.code == hrw.EUNSUPPORTED
    with pytest.raises(hrw.HrwError) as e:
        lib_mask = (1 << 6) | 1
        out = ctypes.c_size_t()
        hrw._check(lib.hrw_gauge_storage_size((ctypes.c_int * 4)(*dims), 3, 2, lib_mask, ctypes.byref(out)))
    assert e.value.code == hrw.EINVAL


def test_su3_two_row_storage_flag(lib):
    """The two-row flag keeps all rows stored (plus one aligned 8-byte slot for the
    special-unitarity check) and is refused for anything but SU(3) fundamental fields."""
    from paper_2405_19294_amd import hrw
    dims = (4, 4, 4, 4)
    assert hrw.STORE_SU3_TWO_ROWS == 1 << 5
    assert hrw.gauge_storage_size(dims, 3, "fund", ("f64", "f32"), two_rows=True) == \
        hrw.gauge_storage_size(dims, 3, "fund", ("f64", "f32")) + 8
    for nc, rep in [(2, "fund"), (4, "fund"), (3, "sym"), (3, "adj")]:
        with pytest.raises(hrw.HrwError) as e:
            hrw.gauge_storage_size(dims, nc, rep, ("f64",), two_rows=True)
        assert e.value.code == hrw.EUNSUPPORTED
