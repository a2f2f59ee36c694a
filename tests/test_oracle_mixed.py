"""Pins for the oracle's emulation of reliable-update mixed-precision CG (CPU only).

The emulation (``oracle.cg_mixed``; the mixed-precision form of the Sec. 3.3 CG,
reliable updates after Clark et al., CPC 181 (2010)) is pinned by what does not
depend on it:

  * with FP64 inner arithmetic and no scheduled updates it is the same
    computation as the plain CG, so its solution equals ``oracle.cg``'s bit for
    bit; with scheduled updates (exact arithmetic: r64 equals the recursive
    residual, so the p shift is zero) it keeps CG's iteration count and
    solution to rounding;
  * in FP32, bfloat16 and binary16 storage the solve reaches the FP64 true
    residual, recomputed with the dense matrix of the operator (brute force),
    and its error against a dense LU solve is within cond(A) tol;
  * the update log follows the trigger rule: an "every" update falls exactly
    `every` iterations after the previous one, a "delta" update at the first
    iteration whose |r|^2 fell below delta^2 times |r|^2 at the last update;
  * binary16 storage with its per-system scale is invariant under scaling the
    source by a power of two (bit for bit), far into the range where unscaled
    binary16 would underflow;
  * ``test_mixed_pins_catch_planted_mistakes`` plants eight mistakes in the
    emulation and checks that these pins reject every one.
"""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc

THETA_AP = (np.pi, 0.0, 0.0, 0.0)
DELTA = {"f32": 1e-3, "bf16": 1e-1, "f16": 1e-2}


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def system(dims, nc, rep, seed, kappa, kind="thermal"):
    uf = fx.gauge_field(dims, nc, kind, seed=seed, eps=0.3)
    ur = orc.rep_map(nc, rep, uf)
    nr = ur.shape[-1]
    eta = orc.split_eo(dims, fx.gaussian_spinor(dims, nr, seed=seed + 1))[0]
    return ur, nr, eta


def dense_normal(dims, ur, nr, kappa):
    """Dense D_hat^+ D_hat on the even sites, column by column from unit vectors."""
    h = fx.volume(dims) // 2
    n = h * 4 * nr
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        d = orc.deo(dims, ur, kappa, e.reshape(h, 4, nr), THETA_AP)
        cols.append(orc.deo(dims, ur, kappa, d, THETA_AP, dagger=True).reshape(-1))
    return np.stack(cols, axis=1)


# small e/o systems: SU(3) fund, SU(2) adj, SU(4) asym (N_R = 6)
CASES = [((2, 2, 2, 4), 3, "fund", 11, 0.135), ((4, 2, 2, 2), 2, "adj", 13, 0.135),
         ((2, 2, 2, 2), 4, "asym", 17, 0.13)]


@pytest.fixture(scope="module")
def dense_cases():
    out = []
    for dims, nc, rep, seed, kappa in CASES:
        ur, nr, eta = system(dims, nc, rep, seed, kappa)
        a = dense_normal(dims, ur, nr, kappa)
        ev = np.linalg.eigvalsh(a)
        x_ref = np.linalg.solve(a, eta.reshape(-1)).reshape(eta.shape)
        out.append(dict(dims=dims, ur=ur, nr=nr, eta=eta, kappa=kappa, a=a, cond=ev[-1] / ev[0], x_ref=x_ref))
    return out


# ----------------------------------------------------------------- FP64 inner arithmetic

@pytest.mark.parametrize("dims,nc,rep,seed,kappa", [((4, 4, 4, 4), 3, "fund", 3, 0.135),
                                                      ((4, 2, 4, 6), 2, "adj", 5, 0.13),
                                                      ((4, 4, 2, 4), 4, "asym", 7, 0.125)])
def test_mixed_f64_equals_plain_cg(dims, nc, rep, seed, kappa):
    ur, nr, eta = system(dims, nc, rep, seed, kappa)
    x0, i0 = orc.cg(dims, ur, kappa, eta, THETA_AP)
    assert i0["status"] == 0 and i0["restarts"] == 0
    x, info = orc.cg_mixed(dims, ur, kappa, eta, THETA_AP, inner="f64", every=0, delta=0.0)
    assert np.array_equal(x, x0)
    assert info["iters"] == i0["iters"] and info["updates"] == 1
    assert info["log"] == [(i0["iters"], "converged", i0["true_rel_resid"])]
    # scheduled updates do not change CG in exact arithmetic
    x, info = orc.cg_mixed(dims, ur, kappa, eta, THETA_AP, inner="f64", every=7, delta=0.0)
    assert info["status"] == 0 and abs(info["iters"] - i0["iters"]) <= 1
    assert info["updates"] >= i0["iters"] // 7
    assert rel(x, x0) <= 1e-11


# ----------------------------------------------------------------- low precision against brute force

def converges_to_dense(c, inner, every, delta, iter_cap):
    x, info = orc.cg_mixed(c["dims"], c["ur"], c["kappa"], c["eta"], THETA_AP, tol=1e-10, max_iter=iter_cap,
                           inner=inner, every=every, delta=delta)
    if info["status"] != 0:
        return False, info
    r = rel(c["a"] @ x.reshape(-1), c["eta"].reshape(-1))
    err = rel(x, c["x_ref"])
    return bool(r <= 1.01e-10 and err <= c["cond"] * 1e-10 and abs(r - info["true_rel_resid"]) <= 1e-3 * r), info


SCHEDULES = {"every": lambda inner: (10, 0.0), "trigger": lambda inner: (50, DELTA[inner]),
             "at_convergence": lambda inner: (0, 0.0)}


@pytest.mark.parametrize("inner,sched", [(i, s) for i in ("f32", "bf16", "f16") for s in ("every", "trigger")]
                         + [("f32", "at_convergence"), ("bf16", "at_convergence")])
def test_mixed_reaches_fp64_residual_against_dense(dense_cases, inner, sched):
    """(binary16 needs updates before the recursion converges: its recursion stalls above 1e-10)"""
    for c in dense_cases:
        every, delta = SCHEDULES[sched](inner)
        _, i0 = orc.cg(c["dims"], c["ur"], c["kappa"], c["eta"], THETA_AP)
        ok, info = converges_to_dense(c, inner, every, delta, 4 * i0["iters"] + 40)
        assert ok, (c["dims"], info["status"], info["true_rel_resid"], info["iters"])


# ----------------------------------------------------------------- the update schedule

def schedule_ok(info, every, delta):
    """The update log against the trigger rule (see the module docstring)."""
    prev = 0
    drop = info["drop"]
    for it, cause, _ in info["log"]:
        span = drop[prev:it]          # iterations prev+1 .. it
        if cause == "every" and not (every > 0 and it - prev == every):
            return False
        if cause == "delta" and not (delta > 0 and span[-1] < delta ** 2):
            return False
        # no trigger fired earlier in the span
        if delta > 0 and np.any(span[:-1] < delta ** 2):
            return False
        if every > 0 and it - prev > every:
            return False
        prev = it
    return True


@pytest.mark.parametrize("inner", ["f32", "bf16", "f16"])
def test_mixed_update_schedule_follows_trigger(inner):
    ur, nr, eta = system((4, 4, 4, 4), 3, "fund", 3, 0.135)
    for every, delta in [(9, 0.0), (0, DELTA[inner]), (13, DELTA[inner])]:
        _, info = orc.cg_mixed((4, 4, 4, 4), ur, 0.135, eta, THETA_AP, inner=inner, every=every, delta=delta)
        assert info["status"] == 0
        assert info["log"][-1][1] != "every" or info["log"][-1][2] <= 1e-10
        causes = {c for _, c, _ in info["log"]}
        assert causes <= ({"every"} if every else set()) | ({"delta"} if delta else set()) | {"converged"}
        assert schedule_ok(info, every, delta), (every, delta, info["log"])
        assert len(info["log"]) == info["updates"]


# ----------------------------------------------------------------- binary16 scaling

def scale_invariant(ur, eta, k):
    dims = (4, 4, 4, 4)
    x1, i1 = orc.cg_mixed(dims, ur, 0.135, eta, THETA_AP, inner="f16", every=50, delta=DELTA["f16"])
    x2, i2 = orc.cg_mixed(dims, ur, 0.135, eta * 2.0 ** k, THETA_AP, inner="f16", every=50, delta=DELTA["f16"])
    return i1["status"] == 0 and np.array_equal(x2, x1 * 2.0 ** k) and i1["iters"] == i2["iters"]


def test_mixed_f16_scale_invariance():
    ur, nr, eta = system((4, 4, 4, 4), 3, "fund", 3, 0.135)
    for k in (-30, -12, 20):
        assert scale_invariant(ur, eta, k), k


# ----------------------------------------------------------------- planted mistakes

def test_mixed_pins_catch_planted_mistakes(dense_cases):
    """Each planted mistake in the emulation fails at least one pin above (checked here on
    the small dense systems, the schedule rule and the binary16 scaling)."""
    ur, nr, eta = system((4, 4, 4, 4), 3, "fund", 3, 0.135)

    def pins_pass():
        for c in dense_cases:
            _, i0 = orc.cg(c["dims"], c["ur"], c["kappa"], c["eta"], THETA_AP)
            for inner, sched in (("f32", "trigger"), ("bf16", "trigger"), ("f16", "trigger"),
                                 ("f32", "at_convergence")):
                every, delta = SCHEDULES[sched](inner)
                ok, _ = converges_to_dense(c, inner, every, delta, 4 * i0["iters"] + 40)
                if not ok:
                    return False
        for inner in ("f32", "f16"):
            _, info = orc.cg_mixed((4, 4, 4, 4), ur, 0.135, eta, THETA_AP, inner=inner, every=9, delta=0.0,
                                   max_iter=400)
            if info["status"] != 0 or not schedule_ok(info, 9, 0.0):
                return False
        return scale_invariant(ur, eta, -30)

    try:
        orc.set_mixed_mutation(0)
        assert pins_pass()
        # 1 x_lo kept after the fold, 2 fold without 1/scale, 3 x accumulated in binary32,
        # 4 stop on the recursive residual, 5 schedule one iteration late, 6 no binary16 scale,
        # 7 true residual with the low-precision operator, 8 residual reseeded without its scale
        for k in range(1, 9):
            orc.set_mixed_mutation(k)
            assert not pins_pass(), k
    finally:
        orc.set_mixed_mutation(0)
