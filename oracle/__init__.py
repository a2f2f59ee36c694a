"""CPU oracle for the Wilson-Dirac operator in higher representations.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this package to check and time the GPU library.  The
library itself never imports, links or runs anything here.

The arithmetic lives in ``oracle.c`` (plain FP64 C, OpenMP over sites); this
module marshals numpy arrays in the canonical layout:

  * gauge field ``[V][4][n][n]`` complex128, spinor ``[V][4][nr]`` complex128;
  * half-parity fields list that parity's sites in lexicographic order, with
    even sites having ``x0+x1+x2+x3`` even.

Each function names the passage of arXiv 2405.19294 it follows; conventions the
paper leaves open are fixed in ``oracle.c``'s header.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REP_IDS = {"fund": 0, "adj": 1, "sym": 2, "asym": 3}
FMT_IDS = {"f32": 0, "bf16": 1, "f16": 2}

_lib = None


def build(force: bool = True, path: str = _LIB, opt=("-O2",)) -> str:
    """Compile oracle.c into a shared library (gcc, OpenMP; -O2 for the tests)."""
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        cmd = ["gcc", *opt, "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


def load_native(directory: str) -> str:
    """Build the same source with -O3 -march=native for the machine this runs on, into
    ``directory``, and use it for every later call (the timing of the oracle as a CPU
    baseline; the tests keep the portable -O2 build)."""
    global _lib
    path = build(True, os.path.join(directory, "liboracle_native.so"), ("-O3", "-march=native"))
    _lib = None
    _load(path)
    return path


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L = ctypes.c_long
        D = ctypes.c_double
        sig = {
            "orc_gamma": (None, [I, P]),
            "orc_rep_dim": (I, [I, I]),
            "orc_rep_map": (I, [I, I, L, P, P]),
            "orc_rep_basis": (I, [I, I, P]),
            "orc_hop": (I, [P, I, P, P, I, P, P]),
            "orc_dw": (I, [P, I, P, D, P, I, P, P]),
            "orc_hop_eo": (I, [P, I, P, P, I, I, P, P]),
            "orc_deo": (I, [P, I, P, D, P, I, P, P]),
            "orc_cg": (I, [P, I, P, D, P, I, P, P, D, I, P, P, P]),
            "orc_cg_mixed": (I, [P, I, P, D, P, I, P, P, D, I, I, I, D, P, P, I, P]),
            "orc_set_mixed_mutation": (None, [I]),
            "orc_bicgstab": (I, [P, I, P, D, P, I, P, P, D, I, P]),
            "orc_bicgstab_sw": (I, [P, I, P, D, D, P, I, P, P, D, I, P]),
            "orc_qmr_g5": (I, [P, I, P, D, P, I, P, P, D, I, P]),
            "orc_clover": (I, [P, I, P, D, D, P]),
            "orc_clover_apply": (I, [P, I, P, D, D, I, I, P, P]),
            "orc_dsw": (I, [P, I, P, D, D, P, I, P, P]),
            "orc_dsw_eo": (I, [P, I, P, D, D, P, I, P, P]),
            "orc_round": (I, [I, L, P]),
            "orc_parity_count": (I, [P, I]),
            "orc_num_threads": (I, []),
            "orc_set_num_threads": (None, [I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dims(dims) -> np.ndarray:
    d = np.ascontiguousarray(dims, dtype=np.int32)
    if d.shape != (4,):
        raise ValueError("dims must have 4 entries")
    return d


def _theta(theta) -> np.ndarray:
    t = np.zeros(4) if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    if t.shape != (4,):
        raise ValueError("theta must have 4 entries")
    return t


def _check(rc: int, what: str):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


# ---------------------------------------------------------------- conventions

def gamma(m: int) -> np.ndarray:
    """Euclidean chiral gamma matrix m (0..3; 4 = gamma_5), 4x4 complex."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().orc_gamma(int(m), _ptr(out))
    return out


def rep_dim(nc: int, rep: str) -> int:
    """Dimension N_R of representation ``rep`` of SU(nc) (Sec. 3.1.2 scaling ~N_f)."""
    return int(_load().orc_rep_dim(int(nc), REP_IDS[rep]))


def rep_basis(nc: int, rep: str) -> np.ndarray:
    """Basis matrices of the representation space, [nr][nc][nc]."""
    nr = rep_dim(nc, rep)
    out = np.zeros((nr, nc, nc), dtype=np.complex128)
    _check(_load().orc_rep_basis(int(nc), REP_IDS[rep], _ptr(out)), "rep_basis")
    return out


def rep_map(nc: int, rep: str, u_f) -> np.ndarray:
    """Represented links U_R for fundamental links U_F (any leading shape).

    Fermions in a higher representation see the gauge field through U_R
    (Sec. 3.1, Sec. 3.1.2).
    """
    u = _c128(u_f)
    if u.shape[-2:] != (nc, nc):
        raise ValueError("u_f must end in (nc, nc)")
    nr = rep_dim(nc, rep)
    lead = u.shape[:-2]
    n = int(np.prod(lead)) if lead else 1
    out = np.zeros(lead + (nr, nr), dtype=np.complex128)
    _check(_load().orc_rep_map(int(nc), REP_IDS[rep], n, _ptr(u), _ptr(out)), "rep_map")
    return out


# ---------------------------------------------------------------- operator

def _nr_of(u_r) -> int:
    return int(u_r.shape[-1])


def hop(dims, u_r, psi, theta=None, dagger=False) -> np.ndarray:
    """Hopping term H psi (or H^+ psi) on the full lattice (Sec. 3.1)."""
    u, p = _c128(u_r), _c128(psi)
    out = np.zeros_like(p)
    _check(_load().orc_hop(_ptr(_dims(dims)), _nr_of(u), _ptr(u), _ptr(_theta(theta)),
                           int(bool(dagger)), _ptr(p), _ptr(out)), "hop")
    return out


def dw(dims, u_r, kappa, psi, theta=None, dagger=False) -> np.ndarray:
    """Wilson-Dirac operator D psi = psi - kappa H psi (or D^+ psi) (Sec. 3.1)."""
    u, p = _c128(u_r), _c128(psi)
    out = np.zeros_like(p)
    _check(_load().orc_dw(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa),
                          _ptr(_theta(theta)), int(bool(dagger)), _ptr(p), _ptr(out)), "dw")
    return out


def hop_eo(dims, u_r, in_half, out_parity, theta=None, dagger=False) -> np.ndarray:
    """Off-diagonal block of H from parity 1-out_parity to out_parity (Sec. 3.1, even/odd)."""
    u, p = _c128(u_r), _c128(in_half)
    out = np.zeros_like(p)
    _check(_load().orc_hop_eo(_ptr(_dims(dims)), _nr_of(u), _ptr(u), _ptr(_theta(theta)),
                              int(bool(dagger)), int(out_parity), _ptr(p), _ptr(out)), "hop_eo")
    return out


def deo(dims, u_r, kappa, in_e, theta=None, dagger=False) -> np.ndarray:
    """Even/odd Schur operator D_hat = 1 - kappa^2 H_eo H_oe on even sites (Sec. 3.1)."""
    u, p = _c128(u_r), _c128(in_e)
    out = np.zeros_like(p)
    _check(_load().orc_deo(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa),
                           _ptr(_theta(theta)), int(bool(dagger)), _ptr(p), _ptr(out)), "deo")
    return out


def gamma5(psi) -> np.ndarray:
    """gamma_5 applied to a spinor field [..., 4, nr]."""
    g5 = gamma(4)
    return np.einsum("ab,...bc->...ac", g5, _c128(psi))


# ---------------------------------------------------------------- parity helpers

def parity_of_sites(dims) -> np.ndarray:
    x = np.indices(tuple(int(v) for v in dims)).reshape(4, -1)
    return (x.sum(axis=0) & 1).astype(np.int8)


def split_eo(dims, psi):
    """Full field -> (even half, odd half), each listing its sites lexicographically."""
    par = parity_of_sites(dims)
    p = _c128(psi)
    return np.ascontiguousarray(p[..., par == 0, :, :]), np.ascontiguousarray(p[..., par == 1, :, :])


def merge_eo(dims, even, odd):
    par = parity_of_sites(dims)
    e = _c128(even)
    out = np.zeros(e.shape[:-3] + (len(par),) + e.shape[-2:], dtype=np.complex128)
    out[..., par == 0, :, :] = e
    out[..., par == 1, :, :] = _c128(odd)
    return out


# ---------------------------------------------------------------- CG

SYSTEM_FULL = 0   # A = D^+ D on the full lattice
SYSTEM_EO = 1     # A = D_hat^+ D_hat on the even sites


def cg(dims, u_r, kappa, eta, theta=None, system=SYSTEM_EO, tol=1e-10, max_iter=10000):
    """Conjugate gradient for A x = eta from x = 0 (Sec. 3.3).

    Returns (x, info) with info = {"status", "iters", "true_rel_resid",
    "restarts", "alpha", "beta"}; the true residual is recomputed in FP64.
    """
    u, b = _c128(u_r), _c128(eta)
    x = np.zeros_like(b)
    alpha = np.zeros(max_iter)
    beta = np.zeros(max_iter)
    info = np.zeros(3)
    rc = _load().orc_cg(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), _ptr(_theta(theta)),
                        int(system), _ptr(b), _ptr(x), float(tol), int(max_iter),
                        _ptr(alpha), _ptr(beta), _ptr(info))
    _check(rc if rc != -5 else 0, "cg")
    it = int(info[0])
    return x, {"status": int(rc), "iters": it, "true_rel_resid": float(info[1]),
               "restarts": int(info[2]), "alpha": alpha[:it].copy(), "beta": beta[:it].copy()}


MIXED_FMT = {"f64": -1, "f32": 0, "bf16": 1, "f16": 2}
UPDATE_CAUSE = {1: "every", 2: "delta", 3: "converged"}


def cg_mixed(dims, u_r, kappa, eta, theta=None, system=SYSTEM_EO, tol=1e-10, max_iter=10000, inner="f32",
             every=50, delta=0.0):
    """CG with reliable updates in mixed precision, emulated on the CPU (the
    mixed-precision form of the Sec. 3.3 CG; reliable updates after Clark et
    al., CPC 181 (2010)).  The inner iteration stores its fields in ``inner``
    ("f32", "bf16", "f16"; "f64" for plain FP64 arithmetic) with float
    arithmetic; every ``every`` iterations, when |r| fell by ``delta`` since
    the last update, or when the recursion meets ``tol``, the solution is
    folded into FP64 and the residual recomputed in FP64 (see orc_cg_mixed).

    Returns (x, info): info = {"status", "iters", "true_rel_resid",
    "restarts", "updates", "log", "drop"}; log rows are (iteration, cause,
    |r64|/|eta|) per update, drop[k] = |r|^2 after iteration k+1 over |r|^2
    at the last update.
    """
    u, b = _c128(u_r), _c128(eta)
    x = np.zeros_like(b)
    info = np.zeros(5)
    cap = max_iter + 64
    log = np.zeros((cap, 3))
    drop = np.zeros(max_iter)
    rc = _load().orc_cg_mixed(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), _ptr(_theta(theta)),
                              int(system), _ptr(b), _ptr(x), float(tol), int(max_iter), MIXED_FMT[inner],
                              int(every), float(delta), _ptr(info), _ptr(log), cap, _ptr(drop))
    _check(rc if rc != -5 else 0, "cg_mixed")
    it, nlog = int(info[0]), int(info[4])
    rows = [(int(a), UPDATE_CAUSE[int(c)], float(t)) for a, c, t in log[:nlog]]
    return x, {"status": int(rc), "iters": it, "true_rel_resid": float(info[1]), "restarts": int(info[2]),
               "updates": int(info[3]), "log": rows, "drop": drop[:it].copy()}


def set_mixed_mutation(k: int) -> None:
    """Plant mistake k (0 = none) in the mixed-precision CG emulation.  For the
    tests that show the emulation's pins reject each planted mistake."""
    _load().orc_set_mixed_mutation(int(k))


def lanczos_extremes(alpha, beta):
    """Extreme eigenvalues of A from CG coefficients (CG-Lanczos relation).

    T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1}, T_k,k+1 = sqrt(beta_k)/alpha_k
    (Golub & Van Loan, Matrix Computations, Sec. 11.3).
    """
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    k = len(a)
    if k == 0:
        return 0.0, 0.0
    diag = 1.0 / a
    diag[1:] += b[:-1] / a[:-1]
    off = np.sqrt(b[:-1]) / a[:-1]
    t = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    ev = np.linalg.eigvalsh(t)
    return float(ev[0]), float(ev[-1])


def solve_d_eo(dims, u_r, kappa, b, theta=None, tol=1e-10, max_iter=10000):
    """Solve D x = b by the even/odd Schur complement and CG on the normal equations.

    b'_e = b_e + kappa H_eo b_o; D_hat x_e = b'_e (as D_hat^+ D_hat x_e =
    D_hat^+ b'_e); x_o = b_o + kappa H_oe x_e (Sec. 3.1 even/odd, Sec. 3.3 CG).
    """
    be, bo = split_eo(dims, b)
    bpe = be + kappa * hop_eo(dims, u_r, bo, 0, theta)
    eta = deo(dims, u_r, kappa, bpe, theta, dagger=True)
    xe, info = cg(dims, u_r, kappa, eta, theta, SYSTEM_EO, tol, max_iter)
    xo = bo + kappa * hop_eo(dims, u_r, xe, 1, theta)
    return merge_eo(dims, xe, xo), info


# ---------------------------------------------------------------- BiCGstab

BICG_FULL = 0     # D x = b on the full lattice
BICG_EO = 1       # D_hat x_e = b_e on the even sites


def bicgstab(dims, u_r, kappa, b, theta=None, system=BICG_EO, tol=1e-10, max_iter=10000):
    """Stabilised bi-conjugate gradient for D x = b or D_hat x_e = b_e from x = 0
    (Sec. 3.3 inverters; van der Vorst 1992).

    Returns (x, info) with info = {"status", "iters", "true_rel_resid",
    "restarts"}; the true residual is recomputed in FP64.
    """
    u, bb = _c128(u_r), _c128(b)
    x = np.zeros_like(bb)
    info = np.zeros(3)
    rc = _load().orc_bicgstab(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), _ptr(_theta(theta)),
                              int(system), _ptr(bb), _ptr(x), float(tol), int(max_iter), _ptr(info))
    _check(rc if rc != -5 else 0, "bicgstab")
    return x, {"status": int(rc), "iters": int(info[0]), "true_rel_resid": float(info[1]),
               "restarts": int(info[2])}


def solve_d_eo_bicgstab(dims, u_r, kappa, b, theta=None, tol=1e-10, max_iter=10000):
    """Solve D x = b by the even/odd Schur complement and BiCGstab on D_hat.

    b'_e = b_e + kappa H_eo b_o; D_hat x_e = b'_e; x_o = b_o + kappa H_oe x_e
    (Sec. 3.1 even/odd, Sec. 3.3 inverters).
    """
    be, bo = split_eo(dims, b)
    bpe = be + kappa * hop_eo(dims, u_r, bo, 0, theta)
    xe, info = bicgstab(dims, u_r, kappa, bpe, theta, BICG_EO, tol, max_iter)
    xo = bo + kappa * hop_eo(dims, u_r, xe, 1, theta)
    return merge_eo(dims, xe, xo), info


def qmr_g5(dims, u_r, kappa, b, theta=None, system=BICG_EO, tol=1e-10, max_iter=10000):
    """QMR on the g5-symmetric Lanczos process for D x = b or D_hat x_e = b_e from x = 0
    (the QMR-g5 inverter of Sec. 3.3).  Returns (x, info) as bicgstab."""
    u, bb = _c128(u_r), _c128(b)
    x = np.zeros_like(bb)
    info = np.zeros(3)
    rc = _load().orc_qmr_g5(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), _ptr(_theta(theta)),
                            int(system), _ptr(bb), _ptr(x), float(tol), int(max_iter), _ptr(info))
    _check(rc if rc != -5 else 0, "qmr_g5")
    return x, {"status": int(rc), "iters": int(info[0]), "true_rel_resid": float(info[1]),
               "restarts": int(info[2])}


# ---------------------------------------------------------------- clover (Sheikholeslami-Wohlert)

def clover(dims, u_r, kappa, csw) -> np.ndarray:
    """A(x) = 1 - kappa c_sw sum_{mu<nu} g_mu g_nu (x) F_mu,nu(x), F the clover average of the
    represented plaquette leaves (Sec. 3.1 clover improvement); shape [V][4 nr][4 nr], index
    spin * nr + colour."""
    u = _c128(u_r)
    nr = _nr_of(u)
    v = int(np.prod(np.asarray(_dims(dims), dtype=np.int64)))
    out = np.zeros((v, 4 * nr, 4 * nr), dtype=np.complex128)
    _check(_load().orc_clover(_ptr(_dims(dims)), nr, _ptr(u), float(kappa), float(csw), _ptr(out)), "clover")
    return out


def clover_apply(dims, u_r, kappa, csw, parity, in_half, inverse=False) -> np.ndarray:
    """A or A^-1 applied on the sites of one parity."""
    u, a = _c128(u_r), _c128(in_half)
    out = np.zeros_like(a)
    _check(_load().orc_clover_apply(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), float(csw), int(parity),
                                    int(bool(inverse)), _ptr(a), _ptr(out)), "clover_apply")
    return out


def dsw(dims, u_r, kappa, csw, psi, theta=None, dagger=False) -> np.ndarray:
    """D_sw psi = A psi - kappa H psi (H^+ with dagger)."""
    u, a = _c128(u_r), _c128(psi)
    out = np.zeros_like(a)
    _check(_load().orc_dsw(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), float(csw), _ptr(_theta(theta)),
                           int(bool(dagger)), _ptr(a), _ptr(out)), "dsw")
    return out


def dsw_eo(dims, u_r, kappa, csw, in_e, theta=None, dagger=False) -> np.ndarray:
    """D_hat_sw = A_ee - kappa^2 H_eo A_oo^-1 H_oe on even sites (the Schur complement of D_sw)."""
    u, a = _c128(u_r), _c128(in_e)
    out = np.zeros_like(a)
    _check(_load().orc_dsw_eo(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), float(csw),
                              _ptr(_theta(theta)), int(bool(dagger)), _ptr(a), _ptr(out)), "dsw_eo")
    return out


def bicgstab_sw(dims, u_r, kappa, csw, b, theta=None, system=BICG_EO, tol=1e-10, max_iter=10000):
    """BiCGstab for D_sw x = b (BICG_FULL) or D_hat_sw x_e = b_e (BICG_EO) from x = 0."""
    u, bb = _c128(u_r), _c128(b)
    x = np.zeros_like(bb)
    info = np.zeros(3)
    rc = _load().orc_bicgstab_sw(_ptr(_dims(dims)), _nr_of(u), _ptr(u), float(kappa), float(csw),
                                 _ptr(_theta(theta)), int(system), _ptr(bb), _ptr(x), float(tol), int(max_iter),
                                 _ptr(info))
    _check(rc if rc != -5 else 0, "bicgstab_sw")
    return x, {"status": int(rc), "iters": int(info[0]), "true_rel_resid": float(info[1]),
               "restarts": int(info[2])}


def solve_dsw_eo_bicgstab(dims, u_r, kappa, csw, b, theta=None, tol=1e-10, max_iter=10000):
    """D_sw x = b through the Schur complement: b'_e = b_e + kappa H_eo A_oo^-1 b_o,
    D_hat_sw x_e = b'_e, x_o = A_oo^-1 (b_o + kappa H_oe x_e)."""
    be, bo = split_eo(dims, b)
    bpe = be + kappa * hop_eo(dims, u_r, clover_apply(dims, u_r, kappa, csw, 1, bo, inverse=True), 0, theta)
    xe, info = bicgstab_sw(dims, u_r, kappa, csw, bpe, theta, BICG_EO, tol, max_iter)
    xo = clover_apply(dims, u_r, kappa, csw, 1, bo + kappa * hop_eo(dims, u_r, xe, 1, theta), inverse=True)
    return merge_eo(dims, xe, xo), info


# ---------------------------------------------------------------- 16-bit storage

def round_to(fmt: str, a) -> np.ndarray:
    """Round every real component to binary32 / bfloat16 / binary16 (ties to even),
    returned as float64 (complex arrays round real and imaginary parts)."""
    arr = np.array(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64, copy=True)
    flat = arr.view(np.float64).reshape(-1)
    _check(_load().orc_round(FMT_IDS[fmt], flat.size, _ptr(flat)), "round")
    return arr


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's later OpenMP loops."""
    _load().orc_set_num_threads(int(n))


# ---------------------------------------------------------------- rounding-error bound

def hop_abs(dims, u_r_abs, psi_abs, gammas=None, dagger=False) -> np.ndarray:
    """|H| |psi| (or |H^+| |psi|): the hop with every link, projector and spinor
    entry replaced by its absolute value (boundary phases have modulus one and
    drop out).  `gammas` (four 4x4 matrices) evaluates the projectors in another
    spin basis (default: the chiral gamma matrices of gamma()); in the chiral
    basis |1 - g| = |1 + g| entrywise, so H and H^+ give the same array.

    Used for the a-priori componentwise bound of a low-precision D_W
    evaluation, |D psi - fl(D psi)| <= gamma_k (|psi| + kappa |H| |psi|),
    gamma_k = k u / (1 - k u) (Higham, Accuracy and Stability of Numerical
    Algorithms, Sec. 3.1).
    """
    d = tuple(int(v) for v in dims)
    nr = psi_abs.shape[-1]
    u = np.asarray(u_r_abs, dtype=np.float64).reshape(d + (4, nr, nr))
    p = np.asarray(psi_abs, dtype=np.float64).reshape(d + (4, nr))
    out = np.zeros_like(p)
    sign = -1.0 if dagger else 1.0
    for mu in range(4):
        g = gamma(mu) if gammas is None else np.asarray(gammas[mu])
        pf = np.roll(p, -1, axis=mu)            # psi(x + mu)
        pb = np.roll(p, 1, axis=mu)             # psi(x - mu)
        ub = np.roll(u[..., mu, :, :], 1, axis=mu)  # U_mu(x - mu)
        tf = np.einsum("...ab,...sb->...sa", u[..., mu, :, :], pf)
        tb = np.einsum("...ba,...sb->...sa", ub, pb)
        out += np.einsum("st,...tc->...sc", np.abs(np.eye(4) - sign * g), tf)
        out += np.einsum("st,...tc->...sc", np.abs(np.eye(4) + sign * g), tb)
    return out.reshape(np.asarray(psi_abs).shape)


def hop_abs_real(dims, u_r, psi, theta=None, dagger=False, gammas=None) -> np.ndarray:
    """Per real component of H psi (or H^+ psi), the sum of the absolute values of
    its real monomials: every complex product expanded into real products, each
    taken with its absolute value (the real-arithmetic |H||psi| of a rounding-error
    analysis, Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.6).
    `gammas` (four 4x4 matrices) evaluates the projectors in another spin basis
    (default: the chiral gamma matrices of gamma()).

    Returned as one complex array: the real part bounds the real components, the
    imaginary part the imaginary components.  A computed evaluation whose every
    monomial passes through at most m roundings then satisfies, per real
    component, |fl(H psi) - H psi| <= gamma_m (this array's component).
    """
    d = tuple(int(v) for v in dims)
    nr = np.asarray(psi).shape[-1]
    u = _c128(u_r).reshape(d + (4, nr, nr))
    p = _c128(psi).reshape(d + (4, nr))
    th = _theta(theta)
    ar, ai = np.abs(p.real), np.abs(p.imag)
    out_r = np.zeros(ar.shape)
    out_i = np.zeros(ar.shape)
    x = np.indices(d)
    sign = -1.0 if dagger else 1.0
    for mu in range(4):
        g = gamma(mu) if gammas is None else np.asarray(gammas[mu])
        for fwd in (True, False):
            if fwd:
                link = u[..., mu, :, :]
                pr, pi_ = np.roll(ar, -1, axis=mu), np.roll(ai, -1, axis=mu)
                wrap = x[mu] == d[mu] - 1
                proj = np.eye(4) - sign * g
                ph = np.exp(1j * th[mu])
            else:
                link = np.conj(np.swapaxes(np.roll(u[..., mu, :, :], 1, axis=mu), -1, -2))
                pr, pi_ = np.roll(ar, 1, axis=mu), np.roll(ai, 1, axis=mu)
                wrap = x[mu] == 0
                proj = np.eye(4) + sign * g
                ph = np.exp(-1j * th[mu])
            lr, li = np.abs(link.real), np.abs(link.imag)
            tr = np.einsum("...ab,...sb->...sa", lr, pr) + np.einsum("...ab,...sb->...sa", li, pi_)
            ti = np.einsum("...ab,...sb->...sa", li, pr) + np.einsum("...ab,...sb->...sa", lr, pi_)
            qr, qi = np.abs(proj.real), np.abs(proj.imag)
            sr = np.einsum("st,...tc->...sc", qr, tr) + np.einsum("st,...tc->...sc", qi, ti)
            si = np.einsum("st,...tc->...sc", qi, tr) + np.einsum("st,...tc->...sc", qr, ti)
            c, sn = abs(ph.real), abs(ph.imag)
            w = wrap[..., None, None]
            out_r += np.where(w, c * sr + sn * si, sr)
            out_i += np.where(w, sn * sr + c * si, si)
    return (out_r + 1j * out_i).reshape(np.asarray(psi).shape)


def gamma_k(k: int, unit_roundoff: float) -> float:
    return k * unit_roundoff / (1 - k * unit_roundoff)
