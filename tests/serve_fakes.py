"""CPU stand-in for the serving backend, used by the scheduling tests.

It solves each slot's system with the CPU oracle when the slot is loaded and
reports it finished after a number of steps that grows with its iteration
count, behind the same interface as ``serve.GpuBackend``.  Test code only.
"""

import math

import numpy as np

import fixtures
import oracle


class OracleBackend:
    """CPU stand-in with the same interface: each slot solves its system with the
    CPU oracle when loaded and reports it finished after a number of steps that
    grows with its iteration count.  For tiny lattices and tests only."""

    def __init__(self, tol=1e-10, session_bytes_per_slot=1 << 20, fail_keys=(), theta=(math.pi, 0, 0, 0),
                 iters_per_step=20):
        self.fx, self.orc = fixtures, oracle
        self.tol, self.per_slot, self.fail_keys = tol, session_bytes_per_slot, set(fail_keys)
        self.theta, self.iters_per_step = theta, iters_per_step
        self.gauges = {}
        self.dropped = []   # keys whose gauge field the server evicted, in order

    def gauge(self, key):
        if key not in self.gauges:
            dims, nc, rep = key
            uf = self.fx.gauge_field(dims, nc, "thermal", seed=7, eps=0.3)
            self.gauges[key] = self.orc.rep_map(nc, rep, uf)
        return self.gauges[key]

    def gauge_bytes(self, key):
        dims, nc, rep = key
        return int(np.prod(dims)) * 4 * self.orc.rep_dim(nc, rep) ** 2 * 16 * 2

    def drop_gauge(self, key):
        self.gauges.pop(key, None)
        self.dropped.append(key)

    def session_bytes(self, key, n_slots):
        return n_slots * self.per_slot

    def sources(self, req):
        nr = self.orc.rep_dim(req.nc, req.rep)
        full = self.fx.gaussian_spinor(req.dims, nr, seed=req.seed, n_rhs=req.n_rhs)
        return self.orc.split_eo(req.dims, full)[0]

    def open_session(self, key, n_slots):
        return _OracleSession(self, key, n_slots)

    def solve_alone(self, req):
        ur = self.gauge(req.key)
        b = self.sources(req)
        xs, res = [], []
        for j in range(req.n_rhs):
            x, info = self.orc.cg(req.dims, ur, req.kappa, b[j], self.theta, self.orc.SYSTEM_EO, tol=self.tol)
            xs.append(x)
            res.append({"iters": info["iters"], "true_rel_resid": info["true_rel_resid"],
                        "status": 0 if info["status"] == 0 else -5})
        return np.stack(xs), res, 0


class _OracleSession:
    def __init__(self, be, key, n_slots):
        if key in be.fail_keys:
            raise RuntimeError(f"injected failure opening a session for {key}")
        self.be, self.key, self.n_slots = be, key, n_slots
        self.slot = [None] * n_slots  # (x, result, steps left)

    def load(self, slot, req):
        x, res, _ = self.be.solve_alone(req)
        for j in range(req.n_rhs):
            left = max(1, math.ceil(res[j]["iters"] / self.be.iters_per_step))
            self.slot[slot + j] = [x[j], res[j], left]

    def step(self, k):
        running = 0
        for s in self.slot:
            if s is not None and s[2] > 0:
                s[2] -= 1
                running += s[2] > 0
        return running

    def slots(self):
        return [0 if s is None else (1 if s[2] > 0 else 2) for s in self.slot]

    def read(self, slot, n, keep_x=False):
        xs = np.stack([self.slot[slot + j][0] for j in range(n)])
        res = [self.slot[slot + j][1] for j in range(n)]
        for j in range(n):
            self.slot[slot + j] = None
        rc = -5 if any(r["status"] < 0 for r in res) else 0
        return (xs if keep_x else None), res, rc

    def close(self):
        pass
