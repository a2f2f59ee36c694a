"""Continuous-batching sessions: systems join and leave a running session at
step boundaries; each result must equal the standalone solve bit for bit."""

import numpy as np
import pytest

import fixtures as fx
import oracle as orc
from paper_2405_19294_amd import hrw

from gpu_helpers import THETA_AP, setup, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_session_staggered_requests_bitwise_equal_standalone(inner):
    dims = (4, 4, 4, 8)
    uf, ur, g = setup(dims, 2, "adj", "thermal", seed=81, dtypes=("f64", "f32"))
    prm = hrw.solve_params(tol=1e-10, max_iter=3000, system="ddag_d_eo", inner_dtype=inner, reliable_every=25,
                           theta=THETA_AP)
    half = fx.volume(dims) // 2
    reqs = []  # (n_rhs, kappas, sources)
    for k, n in enumerate([2, 1, 3, 1, 2]):
        b = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=90 + k, n_rhs=n))[0]
        ks = [0.12 + 0.003 * ((k + j) % 6) for j in range(n)]
        reqs.append((n, ks, b))
    s = hrw.Session(g, prm, n_slots=5)
    pending = list(range(len(reqs)))
    where = {}          # request -> first slot
    results = {}
    free = [True] * 5
    steps = 0
    while pending or where:
        # admit while slots are free (a request needs n consecutive slots)
        for r in list(pending):
            n = reqs[r][0]
            for a in range(5 - n + 1):
                if all(free[a:a + n]):
                    s.load(a, to_dev(reqs[r][2]), reqs[r][1])
                    for j in range(a, a + n):
                        free[j] = False
                    where[r] = a
                    pending.remove(r)
                    break
            break  # at most one admission per step: requests join while others run
        s.step(7)
        steps += 1
        state = s.slots()
        for r, a in list(where.items()):
            n = reqs[r][0]
            if all(state[j] == 2 for j in range(a, a + n)):
                x, res, rc = s.read(a, n)
                results[r] = (x.cpu().numpy(), res, rc)
                for j in range(a, a + n):
                    free[j] = True
                del where[r]
        assert steps < 2000
    s.close()
    for r, (n, ks, b) in enumerate(reqs):
        x_mix, res_mix, rc = results[r]
        assert rc == 0, res_mix
        x1, res1, rc1 = hrw.cg_solve(g, to_dev(b), ks, prm)
        assert np.array_equal(x_mix, x1.cpu().numpy()), r
        assert [q["iters"] for q in res_mix] == [q["iters"] for q in res1]
        for j in range(n):
            assert res_mix[j]["true_rel_resid"] <= 1e-10


def test_session_failure_isolated():
    dims = (4, 4, 4, 4)
    uf, ur, g = setup(dims, 3, "fund", "thermal", seed=83, dtypes=("f64",))
    prm = hrw.solve_params(tol=1e-10, max_iter=2000, system="ddag_d_eo", theta=THETA_AP)
    b = orc.split_eo(dims, fx.gaussian_spinor(dims, 3, seed=84, n_rhs=2))[0]
    bad = b[1].copy()
    bad[5, 2, 1] = np.inf
    s = hrw.Session(g, prm, n_slots=3)
    s.load(0, to_dev(b[0]), 0.13)
    s.load(1, to_dev(bad), 0.13)
    s.step(3)
    s.load(2, to_dev(b[1]), 0.125)
    while s.step(50):
        pass
    assert s.slots() == [2, 2, 2]
    x0, r0, rc0 = s.read(0, 1)
    xb, rb, rcb = s.read(1, 1)
    x2, r2, rc2 = s.read(2, 1)
    assert rc0 == 0 and rc2 == 0 and rcb == hrw.EBREAKDOWN
    assert s.slots() == [0, 0, 0]
    # a freed slot takes a new request
    s.load(1, to_dev(b[0]), 0.13)
    while s.step(50):
        pass
    x3, r3, rc3 = s.read(1, 1)
    assert rc3 == 0 and np.array_equal(x3.cpu().numpy(), x0.cpu().numpy())
    s.close()


def test_served_stream_results_equal_standalone():
    """A small Poisson stream through the continuous-batching server on the GPU:
    each request's solution equals its standalone solve bit for bit, and the
    oracle, given the request's links and sources copied to the host, finds every
    source's FP64 true residual within the tolerance and the solution within
    cond(A) tol of its own FP64 CG solution."""
    from paper_2405_19294_amd import serve
    be = serve.GpuBackend(inner_dtype="f32", tol=1e-10)
    reqs = serve.poisson_stream(10, rate=100.0, seed=9, volumes=[(4, 4, 4, 8), (8, 4, 4, 4)],
                                reps=[(2, "fund"), (2, "adj"), (3, "fund"), (4, "asym")], max_rhs=4)
    srv = serve.Server(be, hbm_budget=8 << 30, n_slots=6, step_iters=10, keep_x=True)
    rep = srv.run(reqs, realtime=True)
    assert rep["done"] == len(reqs), rep
    theta = be.theta
    for r in reqs:
        x, res, rc = be.solve_alone(r)
        assert rc == 0
        xs = r.x.cpu().numpy()
        assert np.array_equal(xs, x.cpu().numpy()), r.rid
        assert max(r.true_rel_resid) <= 1e-10
        ur = orc.rep_map(r.nc, r.rep, be._links(r.dims, r.nc).cpu().numpy())
        b = be.sources(r).cpu().numpy()
        xs = xs.reshape(b.shape)
        for j in range(r.n_rhs):
            d = orc.deo(r.dims, ur, r.kappa, xs[j], theta)
            ax = orc.deo(r.dims, ur, r.kappa, d, theta, dagger=True)
            assert np.linalg.norm(ax - b[j]) <= 1.01e-10 * np.linalg.norm(b[j]), (r.rid, j)
            xo, info = orc.cg(r.dims, ur, r.kappa, b[j], theta, orc.SYSTEM_EO, tol=1e-12)
            lo, hi = orc.lanczos_extremes(info["alpha"], info["beta"])
            assert np.linalg.norm(xs[j] - xo) <= (hi / lo) * 1e-10 * np.linalg.norm(xo), (r.rid, j)
