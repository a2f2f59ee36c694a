"""Pins for the CPU oracle: each check needs no other implementation of the method.

The paper (arXiv 2405.19294) prints no numeric example, so the oracle is pinned
by closed forms (free-field plane waves), invariants (gamma_5-hermiticity,
gauge covariance, representation identities), textbook special cases
(SU(2) adjoint = SO(3) rotation, diagonal links) and brute force (dense
matrices on tiny lattices).  A dropped term, a flipped sign, a link taken at
the wrong site, a transposed operand or a permuted axis each fails at least
one of them; ``test_pins_catch_planted_mistakes`` checks that claim directly.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc

THETA_AP = np.array([np.pi, 0.0, 0.0, 0.0])
THETA_TW = np.array([np.pi, 0.7, -0.4, 1.3])   # twisted in every direction


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def coords(dims):
    return np.indices(tuple(dims)).reshape(4, -1)


# ----------------------------------------------------------------- gamma basis

def test_gamma_clifford_and_chirality():
    g = [orc.gamma(m) for m in range(5)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(4))
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))
    for a in range(4):
        assert np.allclose(g[4] @ g[a], -g[a] @ g[4])


# ----------------------------------------------------------------- rep maps

REPS = [(2, "fund"), (3, "fund"), (4, "fund"), (2, "adj"), (3, "adj"), (4, "adj"),
        (2, "sym"), (3, "sym"), (4, "sym"), (3, "asym"), (4, "asym")]


@pytest.mark.parametrize("nc,rep", REPS)
def test_rep_unitary_det_homomorphism(nc, rep):
    u = fx.haar_su_n(nc, 6, fx.rng(11, nc))
    ur = orc.rep_map(nc, rep, u)
    nr = orc.rep_dim(nc, rep)
    for k in range(6):
        assert np.allclose(ur[k] @ ur[k].conj().T, np.eye(nr), atol=1e-13)
        assert abs(np.linalg.det(ur[k]) - 1) < 1e-12
    # homomorphism and adjoint
    for k in range(3):
        uv = orc.rep_map(nc, rep, u[k] @ u[k + 3])
        assert np.allclose(uv, ur[k] @ ur[k + 3], atol=1e-13)
        assert np.allclose(orc.rep_map(nc, rep, u[k].conj().T), ur[k].conj().T, atol=1e-13)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_rep_trace_relations(nc):
    u = fx.haar_su_n(nc, 8, fx.rng(12, nc))
    tr = np.trace(u, axis1=1, axis2=2)
    tr2 = np.trace(u @ u, axis1=1, axis2=2)
    adj = orc.rep_map(nc, "adj", u)
    assert np.allclose(adj.imag, 0, atol=1e-15)
    assert np.allclose(np.trace(adj, axis1=1, axis2=2), np.abs(tr) ** 2 - 1, atol=1e-12)
    sym = orc.rep_map(nc, "sym", u)
    assert np.allclose(np.trace(sym, axis1=1, axis2=2), (tr ** 2 + tr2) / 2, atol=1e-12)
    if nc > 2:
        asym = orc.rep_map(nc, "asym", u)
        ta = np.trace(asym, axis1=1, axis2=2)
        assert np.allclose(ta, (tr ** 2 - tr2) / 2, atol=1e-12)
        if nc == 3:
            assert np.allclose(ta, np.conj(tr), atol=1e-12)
        if nc == 4:
            assert np.allclose(ta.imag, 0, atol=1e-12)
    if nc == 2:
        assert np.allclose(np.trace(sym, axis1=1, axis2=2), np.trace(adj, axis1=1, axis2=2))
    assert np.allclose(orc.rep_map(nc, "fund", u), u)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_rep_centre_elements(nc):
    z = np.exp(2j * np.pi / nc) * np.eye(nc)
    assert np.allclose(orc.rep_map(nc, "adj", z), np.eye(nc * nc - 1), atol=1e-13)
    nr = orc.rep_dim(nc, "sym")
    assert np.allclose(orc.rep_map(nc, "sym", z), z[0, 0] ** 2 * np.eye(nr), atol=1e-13)
    if nc > 2:
        nr = orc.rep_dim(nc, "asym")
        assert np.allclose(orc.rep_map(nc, "asym", z), z[0, 0] ** 2 * np.eye(nr), atol=1e-13)


@pytest.mark.parametrize("nc,rep", [(2, "adj"), (3, "adj"), (4, "adj"), (3, "sym"), (4, "asym")])
def test_rep_basis_orthonormal(nc, rep):
    b = orc.rep_basis(nc, rep)
    gram = np.einsum("aij,bij->ab", b.conj(), b)
    scale = 0.5 if rep == "adj" else 1.0
    assert np.allclose(gram, scale * np.eye(len(b)), atol=1e-14)
    if rep == "adj":
        assert np.allclose(b, np.conj(np.swapaxes(b, 1, 2)))
        assert np.allclose(np.trace(b, axis1=1, axis2=2), 0)


def test_su2_adjoint_is_rotation():
    """exp(-i phi sigma_3 / 2) rotates the generators by phi about axis 3."""
    phi = 0.83
    u = np.diag([np.exp(-0.5j * phi), np.exp(0.5j * phi)])
    r = orc.rep_map(2, "adj", u)
    c, s = np.cos(phi), np.sin(phi)
    assert np.allclose(r, [[c, -s, 0], [s, c, 0], [0, 0, 1]], atol=1e-14)
    # and about axis 1: generators 2 and 3 rotate
    u1 = np.array([[np.cos(phi / 2), -1j * np.sin(phi / 2)], [-1j * np.sin(phi / 2), np.cos(phi / 2)]])
    r1 = orc.rep_map(2, "adj", u1)
    assert np.allclose(r1, [[1, 0, 0], [0, c, -s], [0, s, c]], atol=1e-14)


def test_two_index_diagonal_links_fix_basis_order():
    """Diagonal U = diag(u_j): e_(jk) picks up u_j u_k, in lexicographic pair order."""
    ph = np.exp(1j * np.array([0.3, -1.1, 0.5, 0.3]))
    ph[-1] = 1 / np.prod(ph[:-1])
    u = np.diag(ph)
    sym = [ph[j] * ph[k] for j in range(4) for k in range(j, 4)]
    asym = [ph[j] * ph[k] for j in range(4) for k in range(j + 1, 4)]
    assert np.allclose(orc.rep_map(4, "sym", u), np.diag(sym), atol=1e-14)
    assert np.allclose(orc.rep_map(4, "asym", u), np.diag(asym), atol=1e-14)
    # a permutation-like link moves basis vectors: U = [[0,1],[-1,0]] swaps E00 and E11
    w = np.array([[0, 1], [-1, 0]], dtype=complex)
    assert np.allclose(orc.rep_map(2, "sym", w), [[0, 0, 1], [0, -1, 0], [1, 0, 0]], atol=1e-14)


# ----------------------------------------------------------------- free field (closed form)

def plane_wave(dims, n, theta, spin_colour):
    """exp(i p.x) u with p_mu = (2 pi n_mu + theta_mu) / N_mu."""
    x = coords(dims)
    p = (2 * np.pi * np.asarray(n) + theta) / np.asarray(dims)
    phase = np.exp(1j * np.tensordot(p, x, axes=(0, 0)))
    return phase[:, None, None] * spin_colour[None], p


def free_symbol(p, kappa, dagger=False):
    g = [orc.gamma(m) for m in range(4)]
    s = 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
    return (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4) + (-s if dagger else s)


@pytest.mark.parametrize("dims,nr,theta", [((4, 4, 4, 4), 2, THETA_AP), ((6, 4, 2, 8), 3, THETA_TW),
                                           ((4, 2, 6, 4), 6, THETA_TW)])
@pytest.mark.parametrize("dagger", [False, True])
def test_free_field_plane_waves(dims, nr, theta, dagger):
    kappa = 0.137
    u = np.zeros((fx.volume(dims), 4, nr, nr), complex)
    u[:, :, np.arange(nr), np.arange(nr)] = 1
    g = fx.rng(3, nr)
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 3, 1, 2)]:
        sc = g.standard_normal((4, nr)) + 1j * g.standard_normal((4, nr))
        psi, p = plane_wave(dims, n, theta, sc)
        out = orc.dw(dims, u, kappa, psi, theta, dagger=dagger)
        expect = np.einsum("ab,sbc->sac", free_symbol(p, kappa, dagger), psi)
        assert rel(out, expect) < 1e-13


# ----------------------------------------------------------------- gamma_5-hermiticity

def _random_setup(dims, nc, rep, seed=5, kind="haar"):
    uf = fx.gauge_field(dims, nc, kind, seed=seed)
    return orc.rep_map(nc, rep, uf)


def inner(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


@pytest.mark.parametrize("nc,rep", [(2, "fund"), (3, "fund"), (2, "adj"), (3, "sym"), (4, "asym")])
def test_gamma5_hermiticity(nc, rep):
    dims = (4, 2, 4, 6)
    ur = _random_setup(dims, nc, rep)
    nr = ur.shape[-1]
    chi = fx.gaussian_spinor(dims, nr, seed=8)
    psi = fx.gaussian_spinor(dims, nr, seed=9)
    kappa = 0.13
    d_psi = orc.dw(dims, ur, kappa, psi, THETA_TW)
    g5dg5_chi = orc.gamma5(orc.dw(dims, ur, kappa, orc.gamma5(chi), THETA_TW))
    lhs = inner(chi, d_psi)
    assert abs(lhs - inner(g5dg5_chi, psi)) < 1e-13 * abs(lhs) * 10
    assert abs(lhs - np.conj(inner(psi, g5dg5_chi))) < 1e-13 * abs(lhs) * 10
    # the dagger flag is the adjoint: D^+ = g5 D g5
    assert rel(orc.dw(dims, ur, kappa, chi, THETA_TW, dagger=True), g5dg5_chi) < 1e-14


# ----------------------------------------------------------------- gauge covariance

@pytest.mark.parametrize("nc,rep", [(2, "fund"), (3, "fund"), (2, "adj"), (3, "sym"), (4, "asym")])
def test_gauge_covariance(nc, rep):
    dims = (4, 4, 2, 6)
    v = fx.volume(dims)
    uf = fx.gauge_field(dims, nc, "haar", seed=21)
    gt = fx.random_gauge_transform(dims, nc, seed=22)
    x = coords(dims)
    ugf = np.empty_like(uf)
    for mu in range(4):
        y = x.copy()
        y[mu] = (y[mu] + 1) % dims[mu]
        fwd = np.ravel_multi_index(tuple(y), dims)
        ugf[:, mu] = gt @ uf[:, mu] @ np.conj(np.swapaxes(gt[fwd], 1, 2))
    ur = orc.rep_map(nc, rep, uf)
    urg = orc.rep_map(nc, rep, ugf)
    rg = orc.rep_map(nc, rep, gt)
    nr = ur.shape[-1]
    psi = fx.gaussian_spinor(dims, nr, seed=23)
    rot = lambda f: np.einsum("sab,sib->sia", rg, f)
    kappa = 0.125
    lhs = orc.dw(dims, urg, kappa, rot(psi), THETA_TW)
    rhs = rot(orc.dw(dims, ur, kappa, psi, THETA_TW))
    assert rel(lhs, rhs) < 1e-13
    assert v == len(psi)


# ----------------------------------------------------------------- layout conventions

def test_point_source_layout():
    """Point source: D maps delta_x0 e to x0 and its eight neighbours only.

    Checks the canonical indexing (axis 0 = time, x3 fastest) and which link
    each hop uses; extent 3 keeps forward and backward neighbours distinct.
    """
    dims = (3, 4, 5, 6)
    nc = 3
    ur = _random_setup(dims, nc, "fund", seed=31)
    v = fx.volume(dims)
    x0 = (0, 3, 2, 5)
    s0 = np.ravel_multi_index(x0, dims)
    assert s0 == ((x0[0] * dims[1] + x0[1]) * dims[2] + x0[2]) * dims[3] + x0[3]
    e = fx.rng(1, 32).standard_normal((4, nc)) + 0j
    psi = np.zeros((v, 4, nc), complex)
    psi[s0] = e
    kappa = 0.11
    out = orc.dw(dims, ur, kappa, psi, THETA_TW)
    g = [orc.gamma(m) for m in range(4)]
    expect = np.zeros_like(out)
    expect[s0] += e
    for mu in range(4):
        xm = list(x0); xm[mu] = (x0[mu] - 1) % dims[mu]
        xp = list(x0); xp[mu] = (x0[mu] + 1) % dims[mu]
        sm, sp = np.ravel_multi_index(xm, dims), np.ravel_multi_index(xp, dims)
        # site x0 - mu reaches x0 forward through U_mu(x0 - mu)
        ph = np.exp(1j * THETA_TW[mu]) if xm[mu] == dims[mu] - 1 else 1
        expect[sm] += -kappa * ph * (np.eye(4) - g[mu]) @ (e @ ur[sm, mu].T)
        # site x0 + mu reaches x0 backward through U_mu(x0)^+
        ph = np.exp(-1j * THETA_TW[mu]) if xp[mu] == 0 else 1
        expect[sp] += -kappa * ph * (np.eye(4) + g[mu]) @ (e @ ur[s0, mu].conj())
    assert rel(out, expect) < 1e-14


# ----------------------------------------------------------------- brute force

def dense(fn, n_sites, nr):
    n = n_sites * 4 * nr
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        cols.append(fn(e.reshape(n_sites, 4, nr)).reshape(-1))
    return np.stack(cols, axis=1)


def test_dense_adjoint_and_schur():
    dims = (2, 2, 4, 2)
    nc, rep = 3, "fund"
    ur = _random_setup(dims, nc, rep, seed=41)
    nr = 3
    v = fx.volume(dims)
    kappa = 0.14
    d = dense(lambda f: orc.dw(dims, ur, kappa, f, THETA_TW), v, nr)
    dd = dense(lambda f: orc.dw(dims, ur, kappa, f, THETA_TW, dagger=True), v, nr)
    assert np.allclose(dd, d.conj().T, atol=1e-14)
    # Schur complement of the dense blocks equals D_hat
    par = np.repeat(orc.parity_of_sites(dims), 4 * nr)
    ev, od = np.where(par == 0)[0], np.where(par == 1)[0]
    schur = d[np.ix_(ev, ev)] - d[np.ix_(ev, od)] @ np.linalg.solve(d[np.ix_(od, od)], d[np.ix_(od, ev)])
    dhat = dense(lambda f: orc.deo(dims, ur, kappa, f, THETA_TW), v // 2, nr)
    assert np.allclose(dhat, schur, atol=1e-13)
    dhat_dag = dense(lambda f: orc.deo(dims, ur, kappa, f, THETA_TW, dagger=True), v // 2, nr)
    assert np.allclose(dhat_dag, dhat.conj().T, atol=1e-13)
    # the hop blocks are -1/kappa times the off-diagonal blocks of D
    heo = dense(lambda f: orc.hop_eo(dims, ur, f, 0, THETA_TW), v // 2, nr)
    assert np.allclose(heo, -d[np.ix_(ev, od)] / kappa, atol=1e-13)


def test_cg_matches_dense_solve_full_and_eo():
    dims = (4, 2, 2, 4)
    ur = _random_setup(dims, 2, "fund", seed=51)
    nr = 2
    v = fx.volume(dims)
    kappa = 0.12
    eta = fx.gaussian_spinor(dims, nr, seed=52)
    a = dense(lambda f: orc.dw(dims, ur, kappa, orc.dw(dims, ur, kappa, f, THETA_AP), THETA_AP, dagger=True),
              v, nr)
    x_ref = np.linalg.solve(a, eta.reshape(-1)).reshape(eta.shape)
    x, info = orc.cg(dims, ur, kappa, eta, THETA_AP, orc.SYSTEM_FULL, tol=1e-12)
    assert info["status"] == 0 and info["true_rel_resid"] <= 1e-12
    assert rel(x, x_ref) < 1e-10
    # e/o: D x = b through the Schur complement and reconstruction
    dm = dense(lambda f: orc.dw(dims, ur, kappa, f, THETA_AP), v, nr)
    b = fx.gaussian_spinor(dims, nr, seed=53)
    xs, info = orc.solve_d_eo(dims, ur, kappa, b, THETA_AP, tol=1e-12)
    assert info["status"] == 0
    assert rel(xs.reshape(-1), np.linalg.solve(dm, b.reshape(-1))) < 1e-10


def test_cg_plane_wave_one_iteration_and_k_waves():
    dims = (8, 4, 4, 4)
    nr = 3
    u = np.zeros((fx.volume(dims), 4, nr, nr), complex)
    u[:, :, np.arange(nr), np.arange(nr)] = 1
    kappa = 0.12
    g = fx.rng(4, 61)
    sc = g.standard_normal((4, nr)) + 1j * g.standard_normal((4, nr))
    psi, p = plane_wave(dims, (1, 0, 2, 1), THETA_AP, sc)
    x, info = orc.cg(dims, u, kappa, psi, THETA_AP, orc.SYSTEM_FULL, tol=1e-12)
    lam = (1 - 2 * kappa * np.cos(p).sum()) ** 2 + 4 * kappa ** 2 * (np.sin(p) ** 2).sum()
    assert info["iters"] == 1
    assert rel(x, psi / lam) < 1e-13
    # three waves with distinct eigenvalues -> three iterations
    waves = [plane_wave(dims, n, THETA_AP, sc)[0] for n in [(0, 0, 0, 0), (1, 1, 0, 0), (3, 1, 2, 1)]]
    x, info = orc.cg(dims, u, kappa, sum(waves), THETA_AP, orc.SYSTEM_FULL, tol=1e-10)
    assert info["iters"] == 3


def test_lanczos_extremes_match_dense_spectrum():
    dims = (4, 2, 2, 4)
    ur = _random_setup(dims, 2, "fund", seed=71)
    kappa = 0.12
    v = fx.volume(dims)
    eta = fx.gaussian_spinor(dims, 2, seed=72)
    ee, _ = orc.split_eo(dims, eta)
    x, info = orc.cg(dims, ur, kappa, ee, THETA_AP, orc.SYSTEM_EO, tol=1e-13)
    a = dense(lambda f: orc.deo(dims, ur, kappa, orc.deo(dims, ur, kappa, f, THETA_AP), THETA_AP, dagger=True),
              v // 2, 2)
    ev = np.linalg.eigvalsh((a + a.conj().T) / 2)
    lo, hi = orc.lanczos_extremes(info["alpha"], info["beta"])
    # Ritz values lie inside the spectrum and approach its ends
    assert ev[0] * (1 - 1e-12) <= lo and hi <= ev[-1] * (1 + 1e-12)
    assert (ev[-1] - hi) / ev[-1] < 1e-2 and (lo - ev[0]) / ev[0] < 1e-2


# ----------------------------------------------------------------- BiCGstab

def test_bicgstab_matches_dense_solve_and_scipy():
    """The oracle's BiCGstab against a dense solve on D_hat, D and the Schur route,
    and its iteration count against scipy's independent implementation of the
    same method (van der Vorst 1992) run on the dense D_hat."""
    sla = pytest.importorskip("scipy.sparse.linalg")
    dims = (4, 2, 2, 4)
    ur = _random_setup(dims, 2, "fund", seed=55)
    nr, kappa, v = 2, 0.13, fx.volume(dims)
    dhat = dense(lambda f: orc.deo(dims, ur, kappa, f, THETA_AP), v // 2, nr)
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, nr, seed=56))[0]
    x, info = orc.bicgstab(dims, ur, kappa, be, THETA_AP, orc.BICG_EO, tol=1e-12)
    assert info["status"] == 0 and info["true_rel_resid"] <= 1e-12
    assert rel(x.reshape(-1), np.linalg.solve(dhat, be.reshape(-1))) <= np.linalg.cond(dhat) * 1e-12
    steps = []
    xs, flag = sla.bicgstab(dhat, be.reshape(-1), rtol=1e-12, atol=0.0, maxiter=1000,
                            callback=lambda xk: steps.append(1))
    assert flag == 0
    assert abs(len(steps) - info["iters"]) <= 1, (len(steps), info["iters"])
    # full lattice, directly and through the Schur complement
    dm = dense(lambda f: orc.dw(dims, ur, kappa, f, THETA_AP), v, nr)
    b = fx.gaussian_spinor(dims, nr, seed=57)
    ref = np.linalg.solve(dm, b.reshape(-1))
    bound = np.linalg.cond(dm) * 1e-12
    xf, info = orc.bicgstab(dims, ur, kappa, b, THETA_AP, orc.BICG_FULL, tol=1e-12)
    assert info["status"] == 0 and rel(xf.reshape(-1), ref) <= bound
    xe, info = orc.solve_d_eo_bicgstab(dims, ur, kappa, b, THETA_AP, tol=1e-12)
    assert info["status"] == 0 and rel(xe.reshape(-1), ref) <= bound


def test_bicgstab_pins_catch_planted_mistakes():
    """Typical slips in a BiCGstab recurrence still converge (the stop is on the
    residual) but take more iterations: the iteration-count pin against scipy
    rejects each.  The mutants are numpy re-statements written here; the
    oracle is untouched."""
    sla = pytest.importorskip("scipy.sparse.linalg")
    dims = (4, 2, 2, 4)
    ur = _random_setup(dims, 2, "fund", seed=55)
    a = dense(lambda f: orc.deo(dims, ur, 0.13, f, THETA_AP), fx.volume(dims) // 2, 2)
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 2, seed=56))[0].reshape(-1)

    def iterations(mutant, tol=1e-12):
        x, r = np.zeros_like(b), b.copy()
        r0, p, v = b.copy(), b.copy(), np.zeros_like(b)
        rho, rho_old, al, om = np.vdot(b, b), 1.0, 1.0, 1.0
        for it in range(1, 500):
            if it > 1:
                beta = rho / rho_old * (1 if mutant == "beta_without_alpha_over_omega" else al / om)
                p = r + beta * (p + om * v if mutant == "p_sign" else p - om * v)
            v = a @ p
            al = rho / np.vdot(r0, v)
            s_ = r - al * v
            t = a @ s_
            om = (np.vdot(s_, t) if mutant == "omega_conjugated" else np.vdot(t, s_)) / np.vdot(t, t).real
            x, r = x + al * p + om * s_, s_ - om * t
            rho_old, rho = rho, (np.vdot(r, r0) if mutant == "rho_conjugated" else np.vdot(r0, r))
            if np.vdot(r, r).real <= tol ** 2 * np.vdot(b, b).real:
                return it
        return 500

    steps = []
    sla.bicgstab(a, b, rtol=1e-12, atol=0.0, maxiter=1000, callback=lambda xk: steps.append(1))
    assert abs(iterations(None) - len(steps)) <= 1
    for m in ["beta_without_alpha_over_omega", "p_sign", "omega_conjugated", "rho_conjugated"]:
        assert abs(iterations(m) - len(steps)) > 1, m


def test_bicgstab_special_cases():
    """kappa = 0 (D_hat = 1): one iteration gives x = b exactly; a free-field plane
    wave (two distinct eigenvalues of the symbol) converges in at most two
    iterations to the analytic solution; zero and non-finite sources."""
    dims = (4, 4, 2, 4)
    ur = _random_setup(dims, 3, "fund", seed=58)
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=59))[0]
    x, info = orc.bicgstab(dims, ur, 0.0, be, THETA_AP, orc.BICG_EO)
    assert info["iters"] == 1 and info["status"] == 0 and np.array_equal(x, be)
    unit = fx.unit_gauge(dims, 3)
    sc = fx.rng(4, 60).standard_normal((4, 3)) + 1j * fx.rng(4, 61).standard_normal((4, 3))
    pw, pm = plane_wave(dims, (1, 0, 1, 1), THETA_TW, sc)
    kappa = 0.12
    x, info = orc.bicgstab(dims, unit, kappa, pw, THETA_TW, orc.BICG_FULL, tol=1e-13)
    exact = np.einsum("ab,sbc->sac", np.linalg.inv(free_symbol(pm, kappa)), pw)
    assert info["status"] == 0 and info["iters"] <= 2
    assert rel(x, exact) < 1e-12
    zero = np.zeros_like(be)
    x, info = orc.bicgstab(dims, ur, 0.12, zero, THETA_AP)
    assert info["status"] == 0 and info["iters"] == 0 and not np.abs(x).max()
    bad = be.copy()
    bad[1, 2, 0] = np.nan
    _, info = orc.bicgstab(dims, ur, 0.12, bad, THETA_AP)
    assert info["status"] == -5


def test_bicgstab_and_cg_solve_the_same_system():
    """D x = b solved through the Schur complement by BiCGstab on D_hat and by CG
    on its normal equations: the solution is unique, so both agree to the
    tolerance; BiCGstab needs fewer D_hat applications here."""
    dims = (4, 4, 4, 4)
    ur = _random_setup(dims, 3, "fund", seed=62, kind="thermal")
    b = fx.gaussian_spinor(dims, 3, seed=63)
    kappa = 0.135
    xb, ib = orc.solve_d_eo_bicgstab(dims, ur, kappa, b, THETA_AP, tol=1e-11)
    xc, ic = orc.solve_d_eo(dims, ur, kappa, b, THETA_AP, tol=1e-12)
    assert ib["status"] == 0 and ic["status"] == 0
    assert np.linalg.norm(b - orc.dw(dims, ur, kappa, xb, THETA_AP)) / np.linalg.norm(b) <= 1e-10
    assert rel(xb, xc) < 1e-8
    assert 2 * ib["iters"] < 2 * ic["iters"]


# ----------------------------------------------------------------- QMR-g5

def test_qmr_g5_iterates_match_explicit_least_squares():
    """After n steps the oracle's QMR-g5 iterate equals V_n y with y the least-squares solution of
    |rho_1 e_1 - T y|, where V is built here independently by g5-Gram-Schmidt of the Krylov vectors
    b, A b, A^2 b, ... (normalised in the 2-norm) and T = [V_{n+1}, A V_n]_g5 / [v_i, v_i]_g5; and
    the converged solution equals a dense solve, for D_hat and for D."""
    dims = (4, 2, 2, 4)
    ur = _random_setup(dims, 2, "fund", seed=65)
    kappa, v = 0.13, fx.volume(dims)
    dhat = dense(lambda f: orc.deo(dims, ur, kappa, f, THETA_AP), v // 2, 2)
    g5 = np.kron(np.eye(v // 2), np.kron(orc.gamma(4), np.eye(2)))
    jdot = lambda a, c: np.vdot(a, g5 @ c)
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, 2, seed=66))[0]
    b = be.reshape(-1)
    basis = []
    k = b.copy()
    for _ in range(9):
        w = k.copy()
        for q in basis:
            w = w - jdot(q, w) / jdot(q, q) * q
        basis.append(w / np.linalg.norm(w))
        k = dhat @ basis[-1]
    for n in (1, 2, 4, 8):
        vn = np.stack(basis[:n], axis=1)
        vn1 = np.stack(basis[:n + 1], axis=1)
        avn = dhat @ vn
        t = np.array([[jdot(vn1[:, i], avn[:, j]) / jdot(vn1[:, i], vn1[:, i]) for j in range(n)]
                      for i in range(n + 1)])
        rhs = np.zeros(n + 1, complex)
        rhs[0] = np.linalg.norm(b)
        y = np.linalg.lstsq(t, rhs, rcond=None)[0]
        x, info = orc.qmr_g5(dims, ur, kappa, be, THETA_AP, orc.BICG_EO, tol=0.0, max_iter=n)
        assert info["iters"] == n
        assert rel(x.reshape(-1), vn @ y) < 1e-10, n
    x, info = orc.qmr_g5(dims, ur, kappa, be, THETA_AP, orc.BICG_EO, tol=1e-12)
    assert info["status"] == 0 and rel(x.reshape(-1), np.linalg.solve(dhat, b)) <= np.linalg.cond(dhat) * 1e-12
    dm = dense(lambda f: orc.dw(dims, ur, kappa, f, THETA_AP), v, 2)
    bf = fx.gaussian_spinor(dims, 2, seed=67)
    x, info = orc.qmr_g5(dims, ur, kappa, bf, THETA_AP, orc.BICG_FULL, tol=1e-12)
    assert info["status"] == 0
    assert rel(x.reshape(-1), np.linalg.solve(dm, bf.reshape(-1))) <= np.linalg.cond(dm) * 1e-12


def test_qmr_g5_stops_on_the_residual_bound():
    """Regression: stopping on the quasi-residual alone left this system restarting from a residual
    at rounding level (where [v, v]_g5 is near zero and a step is almost empty) until it gave up;
    stopping when sqrt(k + 1) times the quasi-residual reaches tol converges without a restart."""
    dims = (4, 4, 4, 8)
    ur = orc.rep_map(3, "fund", fx.gauge_field(dims, 3, "thermal", seed=93))
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=95, n_rhs=3))[0][1]
    x, info = orc.qmr_g5(dims, ur, 0.125, be, THETA_AP, tol=1e-10)
    assert info["status"] == 0 and info["restarts"] == 0 and info["true_rel_resid"] <= 1e-10


def test_qmr_g5_special_cases():
    """kappa = 0: one step returns b; zero and non-finite sources; agreement with BiCGstab."""
    dims = (4, 4, 2, 4)
    ur = _random_setup(dims, 3, "fund", seed=68, kind="thermal")
    be = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=69))[0]
    x, info = orc.qmr_g5(dims, ur, 0.0, be, THETA_AP)
    assert info["iters"] == 1 and info["status"] == 0 and rel(x, be) < 1e-15
    x, info = orc.qmr_g5(dims, ur, 0.12, np.zeros_like(be), THETA_AP)
    assert info["status"] == 0 and info["iters"] == 0 and not np.abs(x).max()
    bad = be.copy()
    bad[0, 0, 0] = np.inf
    assert orc.qmr_g5(dims, ur, 0.12, bad, THETA_AP)[1]["status"] == -5
    xq, iq = orc.qmr_g5(dims, ur, 0.135, be, THETA_AP, tol=1e-12)
    xb, ib = orc.bicgstab(dims, ur, 0.135, be, THETA_AP, tol=1e-12)
    assert iq["status"] == 0 and rel(xq, xb) < 1e-9


# ----------------------------------------------------------------- clover (Sheikholeslami-Wohlert)

def _gauge_transformed(dims, nc, uf, gt):
    x = coords(dims)
    ugf = np.empty_like(uf)
    for mu in range(4):
        y = x.copy()
        y[mu] = (y[mu] + 1) % dims[mu]
        fwd = np.ravel_multi_index(tuple(y), dims)
        ugf[:, mu] = gt @ uf[:, mu] @ np.conj(np.swapaxes(gt[fwd], 1, 2))
    return ugf


@pytest.mark.parametrize("nc,rep", [(2, "fund"), (3, "fund"), (2, "adj"), (3, "sym"), (4, "asym")])
def test_clover_hermitian_chiral_and_covariant(nc, rep):
    """A is Hermitian, block-diagonal in the chiral basis (commutes with g5), equals 1 on the free
    field and for c_sw = 0, and transforms as A -> (1 x Omega_R) A (1 x Omega_R)^+; D_sw is
    g5-Hermitian and gauge covariant."""
    dims = (4, 2, 4, 2)
    uf = fx.gauge_field(dims, nc, "haar", seed=31)
    ur = orc.rep_map(nc, rep, uf)
    nr = ur.shape[-1]
    kappa, csw = 0.13, 1.3
    a = orc.clover(dims, ur, kappa, csw)
    assert np.abs(a - np.conj(np.swapaxes(a, 1, 2))).max() < 1e-15
    assert np.abs(a[:, :2 * nr, 2 * nr:]).max() == 0 and np.abs(a[:, 2 * nr:, :2 * nr]).max() == 0
    assert np.abs(a - np.eye(4 * nr)).max() > 1e-2
    assert np.array_equal(orc.clover(dims, orc.rep_map(nc, rep, fx.unit_gauge(dims, nc)), kappa, csw),
                          np.broadcast_to(np.eye(4 * nr), a.shape))
    assert np.array_equal(orc.clover(dims, ur, kappa, 0.0), np.broadcast_to(np.eye(4 * nr), a.shape))
    psi = fx.gaussian_spinor(dims, nr, seed=32)
    chi = fx.gaussian_spinor(dims, nr, seed=33)
    assert rel(orc.dsw(dims, ur, kappa, 0.0, psi, THETA_TW), orc.dw(dims, ur, kappa, psi, THETA_TW)) < 1e-15
    g5 = orc.gamma5
    lhs = inner(chi, orc.dsw(dims, ur, kappa, csw, psi, THETA_TW))
    rhs = inner(g5(orc.dsw(dims, ur, kappa, csw, g5(chi), THETA_TW)), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    gt = fx.random_gauge_transform(dims, nc, seed=34)
    urg = orc.rep_map(nc, rep, _gauge_transformed(dims, nc, uf, gt))
    rg = orc.rep_map(nc, rep, gt)
    big = np.einsum("ij,sab->siajb", np.eye(4), rg).reshape(-1, 4 * nr, 4 * nr)
    ag = orc.clover(dims, urg, kappa, csw)
    assert np.abs(ag - big @ a @ np.conj(np.swapaxes(big, 1, 2))).max() < 1e-13
    rot = lambda f: np.einsum("sab,sib->sia", rg, f)
    assert rel(orc.dsw(dims, urg, kappa, csw, rot(psi), THETA_TW), rot(orc.dsw(dims, ur, kappa, csw, psi, THETA_TW))) < 1e-13


@pytest.mark.parametrize("n", [1, 3])
def test_clover_constant_abelian_field(n):
    """U_1(x) = exp(i b x_0 sigma_3) (b = 2 pi n / N_0, the others 1): every leaf of the 0-1 plane is
    exp(i b sigma_3), so F_01 = i sin(b) sigma_3 everywhere, the other planes vanish, and
    A = 1 - kappa c_sw (g_0 g_1) (x) (i sin b sigma_3).  Pins the leaf paths, their orientation,
    the 1/8 normalisation, the order g_mu g_nu and the sign of the term."""
    dims = (6, 4, 2, 2)
    v = fx.volume(dims)
    x = coords(dims)
    b = 2 * np.pi * n / dims[0]
    u = fx.unit_gauge(dims, 2)
    ph = np.exp(1j * b * x[0])
    u[:, 1, 0, 0] = ph
    u[:, 1, 1, 1] = np.conj(ph)
    kappa, csw = 0.12, 1.7
    a = orc.clover(dims, u, kappa, csw)
    s3 = np.diag([1.0, -1.0])
    g01 = orc.gamma(0) @ orc.gamma(1)
    expect = np.eye(8) - kappa * csw * np.kron(g01, 1j * np.sin(b) * s3)
    assert np.abs(a - expect[None]).max() < 1e-14
    assert v == len(a)


def test_clover_schur_complement_and_solves():
    """D_hat_sw equals the Schur complement of the dense D_sw (and its adjoint that of D_sw^+);
    clover_apply's A^-1 inverts A; BiCGstab on D_sw and through the Schur route match a dense solve."""
    dims = (2, 2, 4, 2)
    nc, rep = 3, "fund"
    uf = fx.gauge_field(dims, nc, "haar", seed=35)
    ur = orc.rep_map(nc, rep, uf)
    nr, v = 3, fx.volume(dims)
    kappa, csw = 0.12, 1.1
    d = dense(lambda f: orc.dsw(dims, ur, kappa, csw, f, THETA_TW), v, nr)
    dd = dense(lambda f: orc.dsw(dims, ur, kappa, csw, f, THETA_TW, dagger=True), v, nr)
    assert np.allclose(dd, d.conj().T, atol=1e-14)
    par = np.repeat(orc.parity_of_sites(dims), 4 * nr)
    ev, od = np.where(par == 0)[0], np.where(par == 1)[0]
    schur = d[np.ix_(ev, ev)] - d[np.ix_(ev, od)] @ np.linalg.solve(d[np.ix_(od, od)], d[np.ix_(od, ev)])
    dhat = dense(lambda f: orc.dsw_eo(dims, ur, kappa, csw, f, THETA_TW), v // 2, nr)
    assert np.allclose(dhat, schur, atol=1e-13)
    dhat_dag = dense(lambda f: orc.dsw_eo(dims, ur, kappa, csw, f, THETA_TW, dagger=True), v // 2, nr)
    assert np.allclose(dhat_dag, dhat.conj().T, atol=1e-13)
    t = fx.gaussian_spinor(dims, nr, seed=36)
    to = orc.split_eo(dims, t)[1]
    back = orc.clover_apply(dims, ur, kappa, csw, 1, orc.clover_apply(dims, ur, kappa, csw, 1, to, inverse=True))
    assert rel(back, to) < 1e-14
    b = fx.gaussian_spinor(dims, nr, seed=37)
    ref = np.linalg.solve(d, b.reshape(-1))
    bound = np.linalg.cond(d) * 1e-12
    xf, info = orc.bicgstab_sw(dims, ur, kappa, csw, b, THETA_TW, orc.BICG_FULL, tol=1e-12)
    assert info["status"] == 0 and rel(xf.reshape(-1), ref) <= bound
    xs, info = orc.solve_dsw_eo_bicgstab(dims, ur, kappa, csw, b, THETA_TW, tol=1e-12)
    assert info["status"] == 0 and rel(xs.reshape(-1), ref) <= bound


# ----------------------------------------------------------------- rounding to storage formats

def test_round_f32_and_f16_match_ieee_casts():
    g = fx.rng(9, 81)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.integers(-9, 6, 20000),
                        [0.0, -0.0, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 65519.99, 65520.0, 2.0 ** -25,
                         3 * 2.0 ** -26, 1 + 2 ** -24, 1 + 3 * 2 ** -24, 2.0 ** -149, 2.0 ** -150]])
    with np.errstate(over="ignore"):
        assert np.array_equal(orc.round_to("f32", x), x.astype(np.float32).astype(np.float64))
        assert np.array_equal(orc.round_to("f16", x), x.astype(np.float16).astype(np.float64))


def test_round_bf16_ties_and_torch_cast():
    torch = pytest.importorskip("torch")
    g = fx.rng(9, 82)
    x32 = (g.standard_normal(20000) * 10.0 ** g.integers(-30, 30, 20000)).astype(np.float32)
    x = x32.astype(np.float64)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(orc.round_to("bf16", x), ref)
    # ties go to the even significand
    assert orc.round_to("bf16", np.array([1 + 2 ** -8]))[0] == 1.0
    assert orc.round_to("bf16", np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    # a value just above the tie (not representable in float32) rounds up
    assert orc.round_to("bf16", np.array([1 + 2 ** -8 + 2 ** -40]))[0] == 1 + 2 ** -7


# ----------------------------------------------------------------- the pins catch planted mistakes

def test_pins_catch_planted_mistakes():
    """Plant typical mistakes in a numpy re-statement of the hop and check the pins reject them.

    The mutants are written here (CPU only); the oracle itself is untouched.  The
    unmutated re-statement passes the free-field, gamma_5 and gauge-covariance
    checks; each mutant must fail at least one of them.  Agreement with the
    oracle is not one of the criteria, so the pins alone reject every mutant.
    """
    dims = (4, 2, 2, 4)
    nc = 2
    x = coords(dims)
    g = [orc.gamma(m) for m in range(4)]
    fwd = [None] * 4
    bwd = [None] * 4
    for mu in range(4):
        y = x.copy(); y[mu] = (y[mu] + 1) % dims[mu]; fwd[mu] = np.ravel_multi_index(tuple(y), dims)
        y = x.copy(); y[mu] = (y[mu] - 1) % dims[mu]; bwd[mu] = np.ravel_multi_index(tuple(y), dims)

    def dw_variant(u, kappa, psi, theta, mutant):
        out = np.zeros_like(psi)
        for mu in range(4):
            php = np.where(x[mu] == dims[mu] - 1, np.exp(1j * theta[mu]), 1)
            phm = np.where(x[mu] == 0, np.exp(-1j * theta[mu]), 1)
            gm = g[mu].T if mutant == "transposed_gamma" else g[mu]
            sgn = -1 if mutant == "gamma_sign" else 1
            uf = u[:, mu]
            ub = np.conj(np.swapaxes(u[bwd[mu], mu], 1, 2))
            if mutant == "backward_link_at_x":
                ub = np.conj(np.swapaxes(u[:, mu], 1, 2))
            if mutant == "backward_no_dagger":
                ub = u[bwd[mu], mu]
            if mutant == "no_phase":
                php = phm = np.ones(x.shape[1])
            tf = np.einsum("sab,sib->sia", uf, psi[fwd[mu]])
            tb = np.einsum("sab,sib->sia", ub, psi[bwd[mu]])
            out += php[:, None, None] * (tf - sgn * np.einsum("ij,sjc->sic", gm, tf))
            out += phm[:, None, None] * (tb + sgn * np.einsum("ij,sjc->sic", gm, tb))
        return psi - kappa * out

    uf = fx.gauge_field(dims, nc, "haar", seed=91)
    psi = fx.gaussian_spinor(dims, nc, seed=92)
    chi = fx.gaussian_spinor(dims, nc, seed=93)
    kappa = 0.13

    def passes_all(mutant):
        # free field
        unit = fx.unit_gauge(dims, nc)
        sc = fx.rng(1, 94).standard_normal((4, nc)) + 0j
        pw, p = plane_wave(dims, (1, 1, 0, 1), THETA_TW, sc)
        ok = rel(dw_variant(unit, kappa, pw, THETA_TW, mutant),
                 np.einsum("ab,sbc->sac", free_symbol(p, kappa), pw)) < 1e-12
        # gamma_5
        lhs = inner(chi, dw_variant(uf, kappa, psi, THETA_TW, mutant))
        g5 = orc.gamma5
        rhs = inner(g5(dw_variant(uf, kappa, g5(chi), THETA_TW, mutant)), psi)
        ok &= abs(lhs - rhs) < 1e-12 * abs(lhs)
        # gauge covariance: D[U^g] g psi = g D[U] psi
        ugf = np.empty_like(uf)
        for mu in range(4):
            ugf[:, mu] = gt @ uf[:, mu] @ np.conj(np.swapaxes(gt[fwd[mu]], 1, 2))
        rot = lambda f: np.einsum("sab,sib->sia", gt, f)
        ok &= rel(dw_variant(ugf, kappa, rot(psi), THETA_TW, mutant),
                  rot(dw_variant(uf, kappa, psi, THETA_TW, mutant))) < 1e-13
        return bool(ok)

    gt = fx.random_gauge_transform(dims, nc, seed=95)
    assert passes_all(None)
    # the unmutated re-statement is the oracle's operator (a check of the re-statement, not a criterion)
    assert rel(dw_variant(uf, kappa, psi, THETA_TW, None), orc.dw(dims, uf, kappa, psi, THETA_TW)) < 1e-13
    for m in ["transposed_gamma", "gamma_sign", "backward_link_at_x", "backward_no_dagger", "no_phase"]:
        assert not passes_all(m), m


def test_hop_abs_bounds_the_hop():
    """|H psi| <= |H| |psi| componentwise (triangle inequality), with equality for
    non-negative inputs on a free field with no phases."""
    dims = (4, 2, 4, 2)
    ur = _random_setup(dims, 3, "fund", seed=95)
    psi = fx.gaussian_spinor(dims, 3, seed=96)
    h = orc.hop(dims, ur, psi, THETA_TW)
    ha = orc.hop_abs(dims, np.abs(ur), np.abs(psi))
    assert np.all(np.abs(h) <= ha * (1 + 1e-12))
    unit = fx.unit_gauge(dims, 3)
    pos = np.abs(psi)
    # free field, positive spinor: projector entries (1 -+ g) have mixed signs, so
    # only the diagonal spin part is exact; check the scale instead
    assert np.allclose(orc.hop_abs(dims, np.abs(unit), pos).sum(), 2 * 8 * pos.sum(), rtol=1e-12)


def test_hop_abs_real_bounds_the_hop_and_free_field_closed_form():
    """The real-arithmetic |H||psi| (oracle.hop_abs_real): it bounds |Re H psi| and |Im H psi|
    componentwise and is at least the sum of the absolute entries of the real embedding of H (built
    column by column, brute force); on unit links, zero phases and a real non-negative spinor it has
    a closed form: the real part collects, per direction, the spinor's own spin component and the
    partner spin of a real gamma entry (mu = 0, 2); the imaginary part the partner of an imaginary
    entry (mu = 1, 3)."""
    dims = (2, 2, 2, 4)
    ur = _random_setup(dims, 3, "fund", seed=97)
    psi = fx.gaussian_spinor(dims, 3, seed=98)
    for dagger in (False, True):
        h = orc.hop(dims, ur, psi, THETA_TW, dagger)
        b = orc.hop_abs_real(dims, ur, psi, THETA_TW, dagger)
        assert np.all(np.abs(h.real) <= b.real * (1 + 1e-12)) and np.all(np.abs(h.imag) <= b.imag * (1 + 1e-12))
    n = psi.size
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        cols.append(orc.hop(dims, ur, e.reshape(psi.shape), THETA_TW).reshape(-1))
    hm = np.stack(cols, axis=1)
    pr, pi_ = np.abs(psi.real).reshape(-1), np.abs(psi.imag).reshape(-1)
    b = orc.hop_abs_real(dims, ur, psi, THETA_TW).reshape(-1)
    assert np.all(np.abs(hm.real) @ pr + np.abs(hm.imag) @ pi_ <= b.real * (1 + 1e-12))
    assert np.all(np.abs(hm.imag) @ pr + np.abs(hm.real) @ pi_ <= b.imag * (1 + 1e-12))
    # free field, real non-negative spinor: partner spin of spin s under gamma_mu
    unit = fx.unit_gauge(dims, 3)
    pos = np.abs(psi.real)
    b = orc.hop_abs_real(dims, unit, pos)
    p4 = pos.reshape(tuple(dims) + (4, 3))
    partner = {0: [2, 3, 0, 1], 1: [3, 2, 1, 0], 2: [3, 2, 1, 0], 3: [2, 3, 0, 1]}
    er = np.zeros_like(p4)
    ei = np.zeros_like(p4)
    for mu in range(4):
        for sh in (-1, 1):
            q = np.roll(p4, sh, axis=mu)
            er += q + (q[..., partner[mu], :] if mu in (0, 2) else 0)
            ei += q[..., partner[mu], :] if mu in (1, 3) else 0
    assert np.allclose(b.real, er.reshape(pos.shape), rtol=1e-14)
    assert np.allclose(b.imag, ei.reshape(pos.shape), rtol=1e-14, atol=0)
