"""Python binding of libhrw (ctypes): argument marshalling only.

Every operation runs in the HIP library; torch supplies device memory and the
current stream.  Fields are complex128 CUDA tensors in the canonical layout of
include/hrw.h ([rhs][site][spin 4][colour N_R], half-parity fields listing that
parity's sites lexicographically).  The binding raises if the library is
missing or a call fails; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrw.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, EBREAKDOWN = -1, -2, -3, -4, -5
REPS = {"fund": 0, "adj": 1, "sym": 2, "asym": 3}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
SYSTEMS = {"ddag_d_full": 0, "ddag_d_eo": 1, "d_cgnr_eo": 2,   # CG (normal equations)
           "dhat_eo": 3, "d_eo": 4}                             # BiCGstab (the operator itself)


class HrwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hrw error {code}: {msg}")
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("system", ctypes.c_int),
                ("inner_dtype", ctypes.c_int), ("reliable_every", ctypes.c_int),
                ("reliable_delta", ctypes.c_double), ("theta", ctypes.c_double * 4)]


class SolveResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("restarts", ctypes.c_int), ("true_rel_resid", ctypes.c_double),
                ("recursive_rel_resid", ctypes.c_double), ("d_rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
P, I, LL, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double, ctypes.c_size_t
IP, DP, SZP = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_size_t)

SIGNATURES = {
    "hrw_last_error": (ctypes.c_char_p, []),
    "hrw_version": (ctypes.c_char_p, []),
    "hrw_rep_dim": (I, [I, I, IP]),
    "hrw_rep_map": (I, [I, I, LL, P, P, P]),
    "hrw_gauge_storage_size": (I, [IP, I, I, ctypes.c_uint, SZP]),
    "hrw_gauge_create": (I, [IP, I, I, P, ctypes.c_uint, P, SZ, P, ctypes.POINTER(P)]),
    "hrw_gauge_destroy": (I, [P]),
    "hrw_gauge_info": (I, [P, IP, IP, IP, IP, ctypes.POINTER(ctypes.c_uint)]),
    "hrw_workspace_size": (I, [IP, I, I, I, ctypes.POINTER(SolveParams), SZP]),
    "hrw_dw_apply": (I, [P, D, DP, I, I, I, P, P, P, SZ, P]),
    "hrw_hop_eo": (I, [P, I, DP, I, I, I, P, P, P, SZ, P]),
    "hrw_deo_apply": (I, [P, DP, DP, I, I, I, P, P, P, SZ, P]),
    "hrw_deo_apply_noalloc": (I, [P, DP, DP, I, I, I, P, P, P]),
    "hrw_cg_solve": (I, [P, ctypes.POINTER(SolveParams), I, DP, P, P, ctypes.POINTER(SolveResult), P, SZ, P]),
    "hrw_bicgstab_solve": (I, [P, ctypes.POINTER(SolveParams), I, DP, P, P, ctypes.POINTER(SolveResult), P, SZ,
                               P]),
    "hrw_qmr_g5_solve": (I, [P, ctypes.POINTER(SolveParams), I, DP, P, P, ctypes.POINTER(SolveResult), P, SZ, P]),
    "hrw_clover_storage_size": (I, [P, ctypes.c_uint, SZP]),
    "hrw_clover_create": (I, [P, D, D, ctypes.c_uint, P, SZ, P, ctypes.POINTER(P)]),
    "hrw_clover_destroy": (I, [P]),
    "hrw_dsw_apply": (I, [P, DP, I, I, I, P, P, P, SZ, P]),
    "hrw_dsw_eo_apply": (I, [P, DP, I, I, I, P, P, P, SZ, P]),
    "hrw_clover_workspace_size": (I, [P, I, ctypes.POINTER(SolveParams), SZP]),
    "hrw_clover_bicgstab_solve": (I, [P, ctypes.POINTER(SolveParams), I, P, P, ctypes.POINTER(SolveResult), P, SZ,
                                      P]),
    "hrw_cg_session_create": (I, [P, ctypes.POINTER(SolveParams), I, P, SZ, P, ctypes.POINTER(P)]),
    "hrw_cg_session_load": (I, [P, I, I, DP, P]),
    "hrw_cg_session_step": (I, [P, I, IP]),
    "hrw_cg_session_slots": (I, [P, IP]),
    "hrw_cg_session_read": (I, [P, I, I, P, ctypes.POINTER(SolveResult)]),
    "hrw_cg_session_destroy": (I, [P]),
    "hrw_timing_enable": (I, [I]),
    "hrw_timing_read": (I, [I, ctypes.POINTER(ctypes.c_longlong), DP, DP]),
}


def load(path: str = LIB_PATH):
    """Load libhrw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_2405_19294_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, allow_positive: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_positive):
        raise HrwError(rc, load().hrw_last_error().decode())
    return rc


def _ints(vals):
    return (ctypes.c_int * len(vals))(*[int(v) for v in vals])


def _doubles(vals):
    return (ctypes.c_double * len(vals))(*[float(v) for v in vals])


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev_field(t: torch.Tensor, what: str) -> int:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous complex128 CUDA tensor")
    return t.data_ptr()


def _alloc_bytes(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def version() -> str:
    return load().hrw_version().decode()


def rep_dim(nc: int, rep: str) -> int:
    out = ctypes.c_int()
    _check(load().hrw_rep_dim(nc, REPS[rep], ctypes.byref(out)))
    return out.value


def rep_map(nc: int, rep: str, u_f: torch.Tensor, stream=None) -> torch.Tensor:
    """U_F [..., nc, nc] -> U_R [..., N_R, N_R] on the device."""
    nr = rep_dim(nc, rep)
    n_links = u_f.numel() // (nc * nc)
    out = torch.empty(u_f.shape[:-2] + (nr, nr), dtype=torch.complex128, device=u_f.device)
    _check(load().hrw_rep_map(nc, REPS[rep], n_links, _dev_field(u_f, "u_f"), out.data_ptr(), _stream(stream)))
    return out


STORE_FUND_HOP = 1 << 4  # keep the fundamental links too: single-source hops build U_R in registers
STORE_SU3_TWO_ROWS = 1 << 5  # SU(3) fundamental links are special unitary: hops read two rows per link


def _storage_mask(dtypes, fused: bool, two_rows: bool = False) -> int:
    return (sum(1 << DTYPES[d] for d in dtypes) | (STORE_FUND_HOP if fused else 0)
            | (STORE_SU3_TWO_ROWS if two_rows else 0))


def gauge_storage_size(dims, nc: int, rep: str, dtypes=("f64",), fused: bool = False, two_rows: bool = False) -> int:
    out = ctypes.c_size_t()
    _check(load().hrw_gauge_storage_size(_ints(dims), nc, REPS[rep], _storage_mask(dtypes, fused, two_rows),
                                         ctypes.byref(out)))
    return out.value


class Gauge:
    """Resident represented gauge field: a handle plus the torch storage it lives in."""

    def __init__(self, dims, nc: int, rep: str, u_f: torch.Tensor, dtypes=("f64", "f32"), stream=None,
                 fused: bool = False, two_rows: bool = False):
        self.dims = tuple(int(d) for d in dims)
        self.nc, self.rep = int(nc), rep
        self.nr = rep_dim(nc, rep)
        self.dtypes = tuple(dtypes)
        self.fused = bool(fused)
        self.two_rows = bool(two_rows)
        mask = _storage_mask(dtypes, fused, two_rows)
        nbytes = gauge_storage_size(dims, nc, rep, dtypes, fused, two_rows)
        self.storage = _alloc_bytes(nbytes, u_f.device)
        h = ctypes.c_void_p()
        _check(load().hrw_gauge_create(_ints(dims), nc, REPS[rep], _dev_field(u_f, "u_f"), mask,
                                       self.storage.data_ptr(), nbytes, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.device = u_f.device

    def close(self):
        if getattr(self, "handle", None):
            load().hrw_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def volume(self) -> int:
        d = self.dims
        return d[0] * d[1] * d[2] * d[3]


def gauge_create(dims, nc, rep, u_f, dtypes=("f64", "f32"), stream=None, fused=False, two_rows=False) -> Gauge:
    return Gauge(dims, nc, rep, u_f, dtypes, stream, fused, two_rows)


def workspace_size(dims, nc: int, rep: str, n_rhs: int = 1, params: SolveParams | None = None) -> int:
    out = ctypes.c_size_t()
    _check(load().hrw_workspace_size(_ints(dims), nc, REPS[rep], n_rhs,
                                     ctypes.byref(params) if params is not None else None, ctypes.byref(out)))
    return out.value


class Workspace:
    """Caller-owned device scratch for the operator applies and solves."""

    def __init__(self, nbytes: int, device):
        self.buf = _alloc_bytes(nbytes, device)
        self.nbytes = int(nbytes)

    @classmethod
    def for_apply(cls, g: Gauge, n_rhs: int = 1):
        return cls(workspace_size(g.dims, g.nc, g.rep, n_rhs), g.device)


def _n_rhs(t: torch.Tensor, per_field: int) -> int:
    n = t.numel() // per_field
    if n * per_field != t.numel() or n < 1:
        raise ValueError("field size does not match the lattice")
    return n


def dw_apply(g: Gauge, kappa: float, psi: torch.Tensor, theta=(0, 0, 0, 0), dtype="f64", dagger=False,
             out=None, ws: Workspace | None = None, stream=None) -> torch.Tensor:
    """D_W psi (or D_W^+ psi) for one or more stacked full-lattice fields."""
    n = _n_rhs(psi, g.volume * 4 * g.nr)
    out = torch.empty_like(psi) if out is None else out
    ws = ws or Workspace.for_apply(g, n)
    _check(load().hrw_dw_apply(g.handle, kappa, _doubles(theta), DTYPES[dtype], n, int(bool(dagger)),
                               _dev_field(psi, "psi"), _dev_field(out, "out"), ws.buf.data_ptr(), ws.nbytes,
                               _stream(stream)))
    return out


def hop_eo(g: Gauge, out_parity: int, psi_half: torch.Tensor, theta=(0, 0, 0, 0), dtype="f64", dagger=False,
           out=None, ws: Workspace | None = None, stream=None) -> torch.Tensor:
    """H_eo (out_parity 0) or H_oe (out_parity 1) on half-parity fields."""
    n = _n_rhs(psi_half, g.volume // 2 * 4 * g.nr)
    out = torch.empty_like(psi_half) if out is None else out
    ws = ws or Workspace.for_apply(g, n)
    _check(load().hrw_hop_eo(g.handle, int(out_parity), _doubles(theta), DTYPES[dtype], n, int(bool(dagger)),
                             _dev_field(psi_half, "psi"), _dev_field(out, "out"), ws.buf.data_ptr(), ws.nbytes,
                             _stream(stream)))
    return out


def deo_apply(g: Gauge, kappa, psi_e: torch.Tensor, theta=(0, 0, 0, 0), dtype="f64", dagger=False, out=None,
              ws: Workspace | None = None, stream=None) -> torch.Tensor:
    """D_hat = 1 - kappa^2 H_eo H_oe on even-site fields; kappa scalar or one per rhs."""
    n = _n_rhs(psi_e, g.volume // 2 * 4 * g.nr)
    ks = [kappa] * n if isinstance(kappa, (int, float)) else list(kappa)
    out = torch.empty_like(psi_e) if out is None else out
    ws = ws or Workspace.for_apply(g, n)
    _check(load().hrw_deo_apply(g.handle, _doubles(ks), _doubles(theta), DTYPES[dtype], n, int(bool(dagger)),
                                _dev_field(psi_e, "psi"), _dev_field(out, "out"), ws.buf.data_ptr(), ws.nbytes,
                                _stream(stream)))
    return out


def deo_apply_noalloc(g: Gauge, kappa, psi_e: torch.Tensor, out: torch.Tensor, theta=(0, 0, 0, 0), dtype="f64",
                      dagger=False, stream=None) -> torch.Tensor:
    """deo_apply with the library's static device scratch instead of a workspace: the call
    allocates nothing (out is the caller's).  Calls that overlap on one GPU race."""
    n = _n_rhs(psi_e, g.volume // 2 * 4 * g.nr)
    ks = [kappa] * n if isinstance(kappa, (int, float)) else list(kappa)
    _check(load().hrw_deo_apply_noalloc(g.handle, _doubles(ks), _doubles(theta), DTYPES[dtype], n,
                                        int(bool(dagger)), _dev_field(psi_e, "psi"), _dev_field(out, "out"),
                                        _stream(stream)))
    return out


# Reliable-update trigger used by the benchmarks and the server for each inner
# precision: a system is brought back to FP64 once its residual has fallen by
# this factor since its last update (besides the fixed interval).  Measured on
# SU(3) sym 32^4, 24 sources, FP32 inner: a fixed 50-iteration interval alone
# takes 67 iterations to 1e-10, the 1e-3 trigger the same 51 as plain FP64.
# The coarser 16-bit formats get correspondingly larger factors.
RELIABLE_DELTA = {"f64": 0.0, "f32": 1e-3, "f16": 1e-2, "bf16": 1e-1}


def qmr_g5_solve(g: Gauge, b: torch.Tensor, kappa, params: SolveParams, x=None, ws: Workspace | None = None,
                 stream=None):
    """QMR-g5 for n_rhs stacked systems ("dhat_eo" or "d_eo", FP64); returns (x, results, status)."""
    n = _n_rhs(b, _system_field(g, params.system))
    ks = [kappa] * n if isinstance(kappa, (int, float)) else list(kappa)
    x = torch.empty_like(b) if x is None else x
    ws = ws or cg_workspace(g, params, n)
    res = (SolveResult * n)()
    rc = load().hrw_qmr_g5_solve(g.handle, ctypes.byref(params), n, _doubles(ks), _dev_field(b, "b"),
                                 _dev_field(x, "x"), res, ws.buf.data_ptr(), ws.nbytes, _stream(stream))
    if rc < 0 and rc != EBREAKDOWN:
        _check(rc)
    return x, [r.as_dict() for r in res], rc


class Clover:
    """Resident clover term of a gauge field for one (kappa, c_sw): blocks of A and A^-1 per site."""

    def __init__(self, g: Gauge, kappa: float, csw: float, dtypes=("f64",), stream=None):
        self.g, self.kappa, self.csw = g, float(kappa), float(csw)
        mask = sum(1 << DTYPES[d] for d in dtypes)
        out = ctypes.c_size_t()
        _check(load().hrw_clover_storage_size(g.handle, mask, ctypes.byref(out)))
        self.storage = _alloc_bytes(out.value, g.device)
        h = ctypes.c_void_p()
        _check(load().hrw_clover_create(g.handle, self.kappa, self.csw, mask, self.storage.data_ptr(), out.value,
                                        _stream(stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().hrw_clover_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dsw_apply(c: Clover, psi: torch.Tensor, theta=(0, 0, 0, 0), dtype="f64", dagger=False, out=None,
              ws: Workspace | None = None, stream=None) -> torch.Tensor:
    """D_sw psi = A psi - kappa H psi on the full lattice."""
    g = c.g
    n = _n_rhs(psi, g.volume * 4 * g.nr)
    out = torch.empty_like(psi) if out is None else out
    ws = ws or Workspace.for_apply(g, n)
    _check(load().hrw_dsw_apply(c.handle, _doubles(theta), DTYPES[dtype], n, int(dagger), _dev_field(psi, "psi"),
                                _dev_field(out, "out"), ws.buf.data_ptr(), ws.nbytes, _stream(stream)))
    return out


def dsw_eo_apply(c: Clover, psi_e: torch.Tensor, theta=(0, 0, 0, 0), dtype="f64", dagger=False, out=None,
                 ws: Workspace | None = None, stream=None) -> torch.Tensor:
    """D_hat_sw psi_e = A_ee psi_e - kappa^2 H_eo A_oo^-1 H_oe psi_e on even half fields."""
    g = c.g
    n = _n_rhs(psi_e, g.volume // 2 * 4 * g.nr)
    out = torch.empty_like(psi_e) if out is None else out
    ws = ws or Workspace.for_apply(g, n)
    _check(load().hrw_dsw_eo_apply(c.handle, _doubles(theta), DTYPES[dtype], n, int(dagger), _dev_field(psi_e, "psi_e"),
                                   _dev_field(out, "out"), ws.buf.data_ptr(), ws.nbytes, _stream(stream)))
    return out


def solve_params(tol=1e-10, max_iter=10000, system="ddag_d_eo", inner_dtype="f64", reliable_every=50,
                 theta=(0, 0, 0, 0), reliable_delta=0.0) -> SolveParams:
    p = SolveParams()
    p.tol, p.max_iter, p.system = tol, max_iter, SYSTEMS[system]
    p.inner_dtype, p.reliable_every, p.reliable_delta = DTYPES[inner_dtype], reliable_every, float(reliable_delta)
    for k in range(4):
        p.theta[k] = float(theta[k])
    return p


def _system_field(g: Gauge, system: int) -> int:
    """Complex elements of one right-hand side: even half field for the systems on D_hat."""
    half = system in (SYSTEMS["ddag_d_eo"], SYSTEMS["dhat_eo"])
    return (g.volume // 2 if half else g.volume) * 4 * g.nr


def cg_workspace(g: Gauge, params: SolveParams, n_rhs: int = 1) -> Workspace:
    return Workspace(workspace_size(g.dims, g.nc, g.rep, n_rhs, params), g.device)


def cg_solve(g: Gauge, b: torch.Tensor, kappa, params: SolveParams, x=None, ws: Workspace | None = None,
             stream=None):
    """CG for n_rhs stacked systems; returns (x, [result dict per rhs], overall status)."""
    n = _n_rhs(b, _system_field(g, params.system))
    ks = [kappa] * n if isinstance(kappa, (int, float)) else list(kappa)
    x = torch.empty_like(b) if x is None else x
    ws = ws or cg_workspace(g, params, n)
    res = (SolveResult * n)()
    rc = load().hrw_cg_solve(g.handle, ctypes.byref(params), n, _doubles(ks), _dev_field(b, "b"),
                             _dev_field(x, "x"), res, ws.buf.data_ptr(), ws.nbytes, _stream(stream))
    if rc < 0 and rc != EBREAKDOWN:
        _check(rc)
    return x, [r.as_dict() for r in res], rc


def bicgstab_solve(g: Gauge, b: torch.Tensor, kappa, params: SolveParams, x=None, ws: Workspace | None = None,
                   stream=None):
    """BiCGstab for n_rhs stacked systems (params.system "dhat_eo": even half
    fields, "d_eo": full-lattice fields); returns (x, [result dict per rhs],
    overall status)."""
    n = _n_rhs(b, _system_field(g, params.system))
    ks = [kappa] * n if isinstance(kappa, (int, float)) else list(kappa)
    x = torch.empty_like(b) if x is None else x
    ws = ws or cg_workspace(g, params, n)
    res = (SolveResult * n)()
    rc = load().hrw_bicgstab_solve(g.handle, ctypes.byref(params), n, _doubles(ks), _dev_field(b, "b"),
                                   _dev_field(x, "x"), res, ws.buf.data_ptr(), ws.nbytes, _stream(stream))
    if rc < 0 and rc != EBREAKDOWN:
        _check(rc)
    return x, [r.as_dict() for r in res], rc


def clover_bicgstab_solve(c: Clover, b: torch.Tensor, params: SolveParams, x=None, stream=None):
    """BiCGstab with the clover term for n_rhs stacked systems at the clover's kappa
    ("dhat_eo": even half fields, "d_eo": full-lattice fields); returns (x, results, status)."""
    g = c.g
    n = _n_rhs(b, _system_field(g, params.system))
    x = torch.empty_like(b) if x is None else x
    out = ctypes.c_size_t()
    _check(load().hrw_clover_workspace_size(c.handle, n, ctypes.byref(params), ctypes.byref(out)))
    ws = Workspace(out.value, g.device)
    res = (SolveResult * n)()
    rc = load().hrw_clover_bicgstab_solve(c.handle, ctypes.byref(params), n, _dev_field(b, "b"), _dev_field(x, "x"),
                                          res, ws.buf.data_ptr(), ws.nbytes, _stream(stream))
    if rc < 0 and rc != EBREAKDOWN:
        _check(rc)
    return x, [r.as_dict() for r in res], rc


class Session:
    """A CG session of n_slots slots over one resident gauge field (continuous batching).

    Systems are loaded into free slots and read out when finished, between
    steps, while the other slots keep iterating; each slot's result is the
    same as a standalone solve of that system.
    """

    def __init__(self, g: Gauge, params: SolveParams, n_slots: int, stream=None):
        self.g, self.params, self.n_slots = g, params, int(n_slots)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws = cg_workspace(g, params, n_slots)
        h = ctypes.c_void_p()
        _check(load().hrw_cg_session_create(g.handle, ctypes.byref(params), self.n_slots, self.ws.buf.data_ptr(),
                                            self.ws.nbytes, self.stream.cuda_stream, ctypes.byref(h)))
        self.handle = h
        per = (g.volume // 2 if params.system == SYSTEMS["ddag_d_eo"] else g.volume) * 4 * g.nr
        self.field_elems = per

    def load(self, slot: int, b: torch.Tensor, kappa):
        n = _n_rhs(b, self.field_elems)
        ks = [kappa] * n if isinstance(kappa, (int, float)) else list(kappa)
        _check(load().hrw_cg_session_load(self.handle, slot, n, _doubles(ks), _dev_field(b, "b")))

    def step(self, max_iters: int) -> int:
        running = ctypes.c_int()
        _check(load().hrw_cg_session_step(self.handle, int(max_iters), ctypes.byref(running)))
        return running.value

    def slots(self):
        st = (ctypes.c_int * self.n_slots)()
        _check(load().hrw_cg_session_slots(self.handle, st))
        return list(st)

    def read(self, slot: int, n: int, x: torch.Tensor | None = None):
        shape = (n, self.field_elems // (4 * self.g.nr), 4, self.g.nr)
        x = torch.empty(shape, dtype=torch.complex128, device=self.g.device) if x is None else x
        res = (SolveResult * n)()
        rc = load().hrw_cg_session_read(self.handle, slot, n, _dev_field(x, "x"), res)
        if rc < 0 and rc != EBREAKDOWN:
            _check(rc)
        return x, [r.as_dict() for r in res], rc

    def close(self):
        if getattr(self, "handle", None):
            load().hrw_cg_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool = True, every: int = 1):
    """Start (clearing the counters) or stop the hopping-kernel timing; `every` = n times one
    launch in n of each epilogue class."""
    _check(load().hrw_timing_enable(max(1, int(every)) if on else 0))


def timing_read(kernel_class: int = 0):
    n = ctypes.c_longlong()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(load().hrw_timing_read(kernel_class, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return {"launches": n.value, "ms": ms.value, "bytes": by.value}
