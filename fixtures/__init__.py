"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module holds input generation only: random SU(N) link fields, Gaussian
spinor fields and point-like sources in the canonical layout. It contains none
of the Wilson-Dirac method itself (no representation map, no hopping term, no
solver), so both sides of every parity test consume bit-identical arrays that
neither side produced.

Canonical layout (the same one the C ABI takes):
  * ``dims = (N0, N1, N2, N3)``; axis 0 is time; site index is lexicographic
    with ``x3`` fastest.
  * gauge field ``[site][mu][row][col]`` complex128, ``U_mu(x)`` joins ``x`` to
    ``x + mu``.
  * spinor ``[site][spin 4][colour]`` complex128; several right-hand sides are
    stacked in front: ``[rhs][site][spin][colour]``.

Random numbers come from numpy's counter-based Philox bit generator keyed by
``(seed, stream)``, so every field is reproducible from its seed alone.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "volume",
    "haar_su_n",
    "near_thermal_su_n",
    "gauge_field",
    "gaussian_spinor",
    "point_smeared_sources",
    "random_gauge_transform",
    "unit_gauge",
]

# stream ids keep independent draws for one seed apart
_STREAM_GAUGE = 1
_STREAM_SPINOR = 2
_STREAM_SOURCE = 3
_STREAM_GTRANS = 4


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """Philox generator keyed by (seed, stream)."""
    ss = np.random.SeedSequence([int(seed), int(stream)])
    return np.random.Generator(np.random.Philox(ss))


def volume(dims) -> int:
    d = tuple(int(v) for v in dims)
    if len(d) != 4 or min(d) < 1:
        raise ValueError(f"dims must be four positive extents, got {dims!r}")
    return d[0] * d[1] * d[2] * d[3]


def _complex_normal(g: np.random.Generator, shape, var: float) -> np.ndarray:
    """Complex Gaussian with E|z|^2 = var (real and imaginary parts var/2 each)."""
    s = np.sqrt(var / 2.0)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re * s + 1j * (im * s)).astype(np.complex128)


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt on rows, then fix det to 1 via the last row.

    Changes an almost-unitary matrix only at the rounding level.
    """
    u = u.copy()
    n = u.shape[-1]
    for i in range(n):
        for j in range(i):
            proj = np.sum(np.conj(u[..., j, :]) * u[..., i, :], axis=-1)
            u[..., i, :] -= proj[..., None] * u[..., j, :]
        nrm = np.sqrt(np.sum(np.abs(u[..., i, :]) ** 2, axis=-1))
        u[..., i, :] /= nrm[..., None]
    det = np.linalg.det(u)
    u[..., n - 1, :] *= np.conj(det)[..., None]
    return u


def haar_su_n(nc: int, count: int, g: np.random.Generator) -> np.ndarray:
    """``count`` Haar-distributed SU(nc) matrices, shape (count, nc, nc).

    SU(2): a uniform point on S^3, U = a0 + i a.sigma.  SU(N>2): QR of a
    complex Ginibre matrix with the diagonal phases of R removed (Mezzadri,
    Notices AMS 54 (2007)), then divided by an N-th root of its determinant.
    """
    if nc == 1:
        return np.ones((count, 1, 1), dtype=np.complex128)
    if nc == 2:
        a = g.standard_normal((count, 4))
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        u = np.empty((count, 2, 2), dtype=np.complex128)
        u[:, 0, 0] = a[:, 0] + 1j * a[:, 3]
        u[:, 0, 1] = a[:, 2] + 1j * a[:, 1]
        u[:, 1, 0] = -a[:, 2] + 1j * a[:, 1]
        u[:, 1, 1] = a[:, 0] - 1j * a[:, 3]
        return u
    z = _complex_normal(g, (count, nc, nc), 1.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    q = q * ph[:, None, :]
    det = np.linalg.det(q)
    q = q * np.exp(-1j * np.angle(det) / nc)[:, None, None]
    return _reunitarise(q)


def _traceless_gue(nc: int, count: int, g: np.random.Generator) -> np.ndarray:
    """Traceless Hermitian H with density proportional to exp(-Tr H^2 / 2).

    Diagonal entries N(0,1), off-diagonal real and imaginary parts N(0,1/2),
    then the trace removed; <Tr H^2> = nc^2 - 1.
    """
    h = np.zeros((count, nc, nc), dtype=np.complex128)
    iu = np.triu_indices(nc, 1)
    off = _complex_normal(g, (count, len(iu[0])), 1.0)
    h[:, iu[0], iu[1]] = off
    h = h + np.conj(np.swapaxes(h, 1, 2))
    di = g.standard_normal((count, nc))
    idx = np.arange(nc)
    h[:, idx, idx] = di
    tr = np.trace(h, axis1=1, axis2=2).real / nc
    h[:, idx, idx] -= tr[:, None]
    return h


def near_thermal_su_n(nc: int, count: int, eps: float, g: np.random.Generator) -> np.ndarray:
    """U = exp(i eps H) with H traceless GUE, then reunitarised.

    The exponential uses the Hermitian eigendecomposition H = V diag(w) V^+.
    """
    if nc == 1:
        return np.ones((count, 1, 1), dtype=np.complex128)
    h = _traceless_gue(nc, count, g)
    out = np.empty_like(h)
    chunk = 1 << 20
    for s in range(0, count, chunk):
        w, v = np.linalg.eigh(h[s:s + chunk])
        ph = np.exp(1j * eps * w)
        out[s:s + chunk] = (v * ph[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))
    return _reunitarise(out)


def gauge_field(dims, nc: int, kind: str = "haar", seed: int = 1, eps: float = 0.3) -> np.ndarray:
    """Fundamental SU(nc) link field, canonical layout [V][4][nc][nc] complex128.

    kind: "haar" (Haar-random links), "thermal" (near-thermal exp(i eps H)) or
    "unit" (free field).
    """
    v = volume(dims)
    if kind == "unit":
        return unit_gauge(dims, nc)
    g = rng(seed, _STREAM_GAUGE)
    if kind == "haar":
        u = haar_su_n(nc, 4 * v, g)
    elif kind == "thermal":
        u = near_thermal_su_n(nc, 4 * v, eps, g)
    else:
        raise ValueError(f"unknown gauge kind {kind!r}")
    return np.ascontiguousarray(u.reshape(v, 4, nc, nc))


def unit_gauge(dims, nc: int) -> np.ndarray:
    v = volume(dims)
    u = np.zeros((v, 4, nc, nc), dtype=np.complex128)
    idx = np.arange(nc)
    u[:, :, idx, idx] = 1.0
    return u


def gaussian_spinor(dims, nr: int, seed: int = 2, n_rhs: int | None = None) -> np.ndarray:
    """Gaussian spinor field(s): real and imaginary parts N(0, 1/2).

    Shape [V][4][nr], or [n_rhs][V][4][nr] when n_rhs is given.
    """
    v = volume(dims)
    g = rng(seed, _STREAM_SPINOR)
    shape = (v, 4, nr) if n_rhs is None else (int(n_rhs), v, 4, nr)
    return _complex_normal(g, shape, 1.0)


def point_smeared_sources(dims, nr: int, n_rhs: int, seed: int = 4, width: float = 2.0,
                          which=None) -> np.ndarray:
    """Point sources at seeded sites, smeared with a spatial Gaussian profile.

    Source k sits at a seeded site x_k, in spin k mod 4 and colour
    (k // 4) mod nr; on the time slice of x_k it carries the weight
    exp(-|x - x_k|^2 / (2 width^2)) with the spatial distance taken with
    periodic wrap, and zero elsewhere; each source is normalised to unit
    2-norm.  Shape [n_rhs][V][4][nr]; with ``which`` (indices below n_rhs)
    only those sources are returned, identical to the full set's entries.
    """
    d = tuple(int(v) for v in dims)
    v = volume(d)
    g = rng(seed, _STREAM_SOURCE)
    ks = list(range(n_rhs)) if which is None else [int(k) for k in which]
    out = np.zeros((len(ks), v, 4, nr), dtype=np.complex128)
    x = np.indices(d).reshape(4, -1)  # coordinates of every site
    pos = [[int(g.integers(0, n)) for n in d] for _ in range(n_rhs)]
    for o, k in enumerate(ks):
        src = pos[k]
        on_slice = x[0] == src[0]
        r2 = np.zeros(v)
        for mu in (1, 2, 3):
            dx = np.abs(x[mu] - src[mu])
            dx = np.minimum(dx, d[mu] - dx)
            r2 += dx.astype(np.float64) ** 2
        w = np.where(on_slice, np.exp(-r2 / (2.0 * width * width)), 0.0)
        out[o, :, k % 4, (k // 4) % nr] = w
        out[o] /= np.sqrt(np.sum(np.abs(out[o]) ** 2))
    return out


def random_gauge_transform(dims, nc: int, seed: int = 7) -> np.ndarray:
    """Haar SU(nc) matrix per site, shape [V][nc][nc]."""
    v = volume(dims)
    return haar_su_n(nc, v, rng(seed, _STREAM_GTRANS))
