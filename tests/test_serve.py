"""Serving-loop logic on the CPU stand-in backend (the CPU oracle behind the
session interface): completion, slot reuse, admission by footprint, refusal,
failure isolation and latency accounting."""

import numpy as np

from paper_2405_19294_amd import serve
from serve_fakes import OracleBackend

SMALL = [(4, 4, 4, 4), (2, 4, 4, 4)]
REPS = [(2, "fund"), (3, "fund")]


def stream(n=12, rate=200.0, max_rhs=3, seed=3):
    return serve.poisson_stream(n, rate=rate, seed=seed, volumes=SMALL, reps=REPS, max_rhs=max_rhs)


def test_stream_is_seeded_and_poisson_like():
    a, b = serve.poisson_stream(400, seed=5), serve.poisson_stream(400, seed=5)
    assert [(r.dims, r.rep, r.n_rhs, r.kappa) for r in a] == [(r.dims, r.rep, r.n_rhs, r.kappa) for r in b]
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 1 / 20.0) < 0.15 / 20.0 * 4
    assert all(0.12 <= r.kappa <= 0.135 and 1 <= r.n_rhs <= 12 for r in a)


def test_all_served_results_equal_standalone_and_slots_reused():
    be = OracleBackend()
    reqs = stream()
    srv = serve.Server(be, hbm_budget=1 << 40, n_slots=4, keep_x=True)
    rep = srv.run(reqs, realtime=False)
    assert rep["done"] == len(reqs) and rep["refused"] == 0 and rep["failed"] == 0
    assert sum(r.n_rhs for r in reqs) > 4 * len({r.key for r in reqs})  # slots had to be reused
    for r in reqs:
        x, res, rc = be.solve_alone(r)
        assert np.array_equal(r.x, x)
        assert max(r.true_rel_resid) <= 1e-10
    lat = [r.latency() for r in reqs]
    assert min(lat) >= 0 and rep["latency_s"]["p50"] <= rep["latency_s"]["p99"] <= rep["latency_s"]["max"]


def test_admission_by_footprint_parks_then_serves():
    be = OracleBackend(session_bytes_per_slot=100)
    reqs = stream(n=10)
    keys = {r.key for r in reqs}
    assert len(keys) > 1
    budget = 4 * 100 + max(be.gauge_bytes(k) for k in keys)  # room for one session at a time
    srv = serve.Server(be, hbm_budget=budget, n_slots=4)
    rep = srv.run(reqs, realtime=False)
    assert rep["done"] == len(reqs)
    assert rep["hbm_peak"] <= budget


def test_resident_gauges_count_against_the_budget():
    """Gauge fields are charged when their first session opens: a budget that holds one
    gauge field and one session serves two keys one after the other, evicting the first
    key's gauge field for the second, and the peak of sessions plus gauges stays within it."""
    be = OracleBackend(session_bytes_per_slot=100)
    a, b = serve.poisson_stream(2, rate=200.0, seed=3, volumes=[(4, 4, 4, 4)], reps=[(2, "fund")], max_rhs=2)
    b.dims = (2, 4, 4, 4)
    b.arrival = a.arrival + 1e-3
    big = max(be.gauge_bytes(a.key), be.gauge_bytes(b.key))
    budget = 4 * 100 + big
    srv = serve.Server(be, hbm_budget=budget, n_slots=4)
    rep = srv.run([a, b], realtime=False)
    assert rep["done"] == 2 and rep["refused"] == 0
    assert rep["hbm_peak"] <= budget
    assert be.dropped == [a.key]                      # evicted to admit the second key
    assert list(srv.resident) == [b.key] and srv.gauge_used == be.gauge_bytes(b.key)
    # both gauges fit: nothing is evicted and both stay resident
    be2 = OracleBackend(session_bytes_per_slot=100)
    a2, b2 = serve.poisson_stream(2, rate=200.0, seed=3, volumes=[(4, 4, 4, 4)], reps=[(2, "fund")], max_rhs=2)
    b2.dims = (2, 4, 4, 4)
    srv2 = serve.Server(be2, hbm_budget=2 * (4 * 100) + be2.gauge_bytes(a2.key) + be2.gauge_bytes(b2.key),
                        n_slots=4)
    rep2 = srv2.run([a2, b2], realtime=False)
    assert rep2["done"] == 2 and be2.dropped == [] and len(srv2.resident) == 2


def test_gauge_larger_than_budget_is_refused():
    be = OracleBackend(session_bytes_per_slot=100)
    reqs = stream(n=4)
    k = reqs[0].key
    srv = serve.Server(be, hbm_budget=be.gauge_bytes(k) + 4 * 100 - 1, n_slots=4)  # session fits, gauge + session do not
    srv.run([reqs[0]], realtime=False)
    assert reqs[0].status == "refused"
    assert srv.gauge_used == 0 and not srv.resident


def test_refusals():
    be = OracleBackend(session_bytes_per_slot=100)
    reqs = stream(n=6, max_rhs=3)
    reqs[0].n_rhs = 9                      # more sources than slots
    srv = serve.Server(be, hbm_budget=1 << 30, n_slots=4)
    rep = srv.run(reqs, realtime=False)
    assert reqs[0].status == "refused" and rep["refused"] == 1 and rep["done"] == len(reqs) - 1
    tiny = serve.Server(OracleBackend(session_bytes_per_slot=10 ** 9), hbm_budget=10 ** 6, n_slots=4)
    rep = tiny.run(stream(n=3), realtime=False)
    assert rep["refused"] == 3


def test_failure_is_isolated():
    reqs = stream(n=12)
    bad = reqs[0].key
    be = OracleBackend(fail_keys=[bad])
    srv = serve.Server(be, hbm_budget=1 << 40, n_slots=4)
    rep = srv.run(reqs, realtime=False)
    n_bad = sum(r.key == bad for r in reqs)
    assert rep["failed"] == n_bad and rep["done"] == len(reqs) - n_bad
    assert all(r.status.startswith("failed") for r in reqs if r.key == bad)


def test_realtime_latency_includes_queueing():
    be = OracleBackend(iters_per_step=5)
    reqs = stream(n=8, rate=50.0, max_rhs=2)
    srv = serve.Server(be, hbm_budget=1 << 40, n_slots=2)
    rep = srv.run(reqs, realtime=True)
    assert rep["done"] == 8
    for r in reqs:
        assert r.t_admit >= r.t_arrive - 1e-6 and r.t_done >= r.t_admit
