"""Serving loop: continuous batching of CG solve requests on one GPU.

Requests (lattice, representation, kappa, number of sources) arrive over time.
Gauge fields stay resident.  Requests that share a gauge field are served by
one solver session (a multi-slot CG, ``hrw.Session``): a request joins a
running session as soon as enough slots are free, its iterations share every
operator launch with the requests already there, and it leaves the session
when its own systems have converged.  Sessions of different gauge fields run
on their own HIP streams from their own host threads, so their work overlaps
on the device.  Admission is by HBM footprint: the resident gauge fields and
the open sessions' workspaces together stay within the budget.  A session is
opened only when its workspace, plus its gauge field if that is not resident
yet, fits; idle sessions are closed and the gauge fields of keys without a
session are evicted, least recently used first, to make room; a request that
cannot fit even on an empty device is refused.

Each request's result is the same as a standalone solve of that request,
because every slot keeps its own recurrence (see ``hrw.Session``).

The backend is pluggable: ``GpuBackend`` drives libhrw.  Any object with the
same methods (gauge, gauge_bytes, drop_gauge, session_bytes, sources,
open_session, solve_alone) can stand in for it, e.g. to test the scheduling on
a CPU.
"""

from __future__ import annotations

import collections
import dataclasses
import json
import math
import queue
import threading
import time
from typing import Callable

import numpy as np

C5_VOLUMES = [(8, 8, 8, 8), (16, 16, 16, 16), (32, 16, 16, 16), (48, 24, 24, 24), (64, 32, 32, 32)]
C5_REPS = [(2, "fund"), (2, "adj"), (3, "fund"), (4, "asym")]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the stream
    dims: tuple
    nc: int
    rep: str
    kappa: float
    n_rhs: int
    seed: int
    # filled in by the server
    t_arrive: float | None = None   # host clock at arrival
    t_admit: float | None = None
    t_done: float | None = None
    status: str = "pending"         # pending | running | done | failed | refused
    iters: list | None = None
    true_rel_resid: list | None = None
    x: object = None

    @property
    def key(self):
        return (tuple(self.dims), self.nc, self.rep)

    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive


def poisson_stream(n_requests=400, rate=20.0, seed=5, volumes=C5_VOLUMES, reps=C5_REPS,
                   kappa=(0.12, 0.135), max_rhs=12) -> list:
    """Seeded request stream: exponential inter-arrival times (rate per second);
    volume, representation and source count uniform, kappa uniform in the range."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 55])))
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(g.exponential(1.0 / rate))
        dims = volumes[int(g.integers(len(volumes)))]
        nc, rep = reps[int(g.integers(len(reps)))]
        out.append(Request(rid=rid, arrival=t, dims=tuple(dims), nc=nc, rep=rep,
                           kappa=float(g.uniform(*kappa)), n_rhs=int(g.integers(1, max_rhs + 1)),
                           seed=1000 + rid))
    return out


# ---------------------------------------------------------------- backends

def near_thermal_links(torch, dev, dims, nc, eps, seed):
    """Seeded near-thermal SU(nc) links U = exp(i eps H), H traceless GUE (density
    exp(-Tr H^2 / 2)), generated on the device; canonical [V][4][nc][nc] complex128."""
    v = int(np.prod(dims))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    n = 4 * v
    a = torch.randn((n, nc, nc), generator=gen, device=dev, dtype=torch.float64)
    b = torch.randn((n, nc, nc), generator=gen, device=dev, dtype=torch.float64)
    h = torch.complex(a, b) / math.sqrt(2.0)
    h = torch.triu(h, 1)
    h = h + h.conj().transpose(1, 2)
    d = torch.randn((n, nc), generator=gen, device=dev, dtype=torch.float64)
    h = h + torch.diag_embed(d.to(torch.complex128))
    tr = torch.diagonal(h, dim1=1, dim2=2).sum(-1) / nc
    h = h - tr[:, None, None] * torch.eye(nc, dtype=torch.complex128, device=dev)
    u = torch.linalg.matrix_exp(1j * eps * h)
    return u.reshape(v, 4, nc, nc).contiguous()


class GpuBackend:
    """libhrw sessions on torch-owned device memory, one HIP stream per session."""

    def __init__(self, inner_dtype="f32", tol=1e-10, max_iter=20000, reliable_every=50, reliable_delta=None,
                 eps=0.3, theta=(math.pi, 0.0, 0.0, 0.0), gauge_seed=7):
        import torch

        from . import hrw
        self.torch, self.hrw = torch, hrw
        hrw.load()
        self.dev = torch.device("cuda:0")
        self.inner, self.eps, self.theta, self.gauge_seed = inner_dtype, eps, theta, gauge_seed
        if reliable_delta is None:
            reliable_delta = hrw.RELIABLE_DELTA[inner_dtype]
        self.params = hrw.solve_params(tol=tol, max_iter=max_iter, system="ddag_d_eo", inner_dtype=inner_dtype,
                                       reliable_every=reliable_every, reliable_delta=reliable_delta, theta=theta)
        self.gauges = {}
        self.lock = threading.Lock()

    # inputs are generated on the device from seeded torch generators
    def _links(self, dims, nc):
        return near_thermal_links(self.torch, self.dev, dims, nc, self.eps,
                                  self.gauge_seed * 1000 + nc * 100 + sum(dims))

    def gauge(self, key):
        with self.lock:
            if key not in self.gauges:
                dims, nc, rep = key
                uf = self._links(dims, nc)
                self.gauges[key] = self.hrw.Gauge(dims, nc, rep, uf, dtypes=("f64", self.inner))
                del uf
            return self.gauges[key]

    def gauge_bytes(self, key):
        dims, nc, rep = key
        return self.hrw.gauge_storage_size(dims, nc, rep, ("f64", self.inner))

    def drop_gauge(self, key):
        """Release a resident gauge field (its key has no open session)."""
        with self.lock:
            g = self.gauges.pop(key, None)
        if g is not None:
            g.close()
            g.storage = None  # its session has closed and synchronised: nothing reads it any more

    def session_bytes(self, key, n_slots):
        dims, nc, rep = key
        return self.hrw.workspace_size(dims, nc, rep, n_slots, self.params)

    def sources(self, req):
        torch = self.torch
        g = self.gauge(req.key)
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(req.seed)
        half = g.volume // 2
        shape = (req.n_rhs, half, 4, g.nr)
        re = torch.randn(shape, generator=gen, device=self.dev, dtype=torch.float64)
        im = torch.randn(shape, generator=gen, device=self.dev, dtype=torch.float64)
        return torch.complex(re, im) * math.sqrt(0.5)

    def open_session(self, key, n_slots):
        return _GpuSession(self, key, n_slots)

    def solve_alone(self, req):
        """Standalone solve of one request (for the alone-vs-mix check)."""
        x, res, rc = self.hrw.cg_solve(self.gauge(req.key), self.sources(req), [req.kappa] * req.n_rhs, self.params)
        return x, res, rc


class _GpuSession:
    def __init__(self, be: GpuBackend, key, n_slots):
        self.be, self.key, self.n_slots = be, key, n_slots
        self.stream = be.torch.cuda.Stream()
        with be.torch.cuda.stream(self.stream):
            self.s = be.hrw.Session(be.gauge(key), be.params, n_slots, stream=self.stream)

    def load(self, slot, req):
        with self.be.torch.cuda.stream(self.stream):
            b = self.be.sources(req)
            self.s.load(slot, b, [req.kappa] * req.n_rhs)
            self.stream.synchronize()

    def step(self, k):
        return self.s.step(k)

    def slots(self):
        return self.s.slots()

    def read(self, slot, n, keep_x=False):
        with self.be.torch.cuda.stream(self.stream):
            x, res, rc = self.s.read(slot, n)
            self.stream.synchronize()
        return (x if keep_x else None), res, rc

    def close(self):
        self.s.close()
        self.stream.synchronize()


# ---------------------------------------------------------------- server

class _Worker(threading.Thread):
    """Runs one session: admits queued requests into free slots between steps."""

    def __init__(self, server, key, sess, n_slots):
        super().__init__(daemon=True)
        self.server, self.key, self.sess, self.n_slots = server, key, sess, n_slots
        self.q = queue.Queue()
        self.waiting = []
        self.where = {}           # rid -> (first slot, request)
        self.free = [True] * n_slots
        self.stop_flag = False
        self.last_busy = time.perf_counter()

    def idle(self):
        return not self.where and not self.waiting and self.q.empty()

    def _admit(self):
        while True:
            try:
                self.waiting.append(self.q.get_nowait())
            except queue.Empty:
                break
        for req in list(self.waiting):
            n = req.n_rhs
            for a in range(self.n_slots - n + 1):
                if all(self.free[a:a + n]):
                    try:
                        self.sess.load(a, req)
                    except Exception as e:  # a bad request fails alone
                        req.status, req.t_done = f"failed: {e}", time.perf_counter()
                        self.waiting.remove(req)
                        self.server._finish(req)
                        break
                    for j in range(a, a + n):
                        self.free[j] = False
                    req.t_admit, req.status = time.perf_counter(), "running"
                    self.where[req.rid] = (a, req)
                    self.waiting.remove(req)
                    break

    def _collect(self):
        state = self.sess.slots()
        for rid, (a, req) in list(self.where.items()):
            n = req.n_rhs
            if all(state[j] == 2 for j in range(a, a + n)):
                x, res, rc = self.sess.read(a, n, keep_x=self.server.keep_x)
                req.x = x
                req.iters = [r["iters"] for r in res]
                req.true_rel_resid = [r["true_rel_resid"] for r in res]
                req.status = "done" if rc == 0 else f"failed: status {rc}"
                req.t_done = time.perf_counter()
                for j in range(a, a + n):
                    self.free[j] = True
                del self.where[rid]
                self.server._finish(req)

    def run(self):
        while not self.stop_flag:
            self._admit()
            if self.where:
                self.sess.step(self.server.step_iters)
                self._collect()
                self.last_busy = time.perf_counter()
            else:
                try:
                    self.waiting.append(self.q.get(timeout=0.002))
                except queue.Empty:
                    pass
        self.sess.close()


class Server:
    """Continuous-batching server over a backend.

    hbm_budget: bytes that the resident gauge fields and the sessions'
    workspaces may occupy together (a gauge field is charged when the first
    session of its key opens and released when it is evicted); n_slots: slots
    per session; step_iters: CG iterations per session step (requests join and
    leave between steps)."""

    def __init__(self, backend, hbm_budget: int, n_slots: int = 12, step_iters: int = 20, keep_x: bool = False,
                 idle_close: float = 0.5):
        self.be, self.budget, self.n_slots = backend, int(hbm_budget), int(n_slots)
        self.step_iters, self.keep_x, self.idle_close = int(step_iters), keep_x, idle_close
        self.workers = {}
        self.used = 0                           # bytes of open sessions' workspaces
        self.gauge_used = 0                     # bytes of resident gauge fields
        self.resident = collections.OrderedDict()  # key -> gauge bytes, least recently used first
        self.session_cost = {}
        self.parked = []          # requests waiting for HBM to open their session
        self.done = []
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.peak_used = 0

    def _finish(self, req):
        with self.cv:
            self.done.append(req)
            self.cv.notify_all()

    def _cost(self, key):
        if key not in self.session_cost:
            self.session_cost[key] = self.be.session_bytes(key, self.n_slots)
        return self.session_cost[key]

    def _route(self, req):
        """Admission by footprint: returns 'queued', 'parked', 'refused' or 'failed'."""
        key = req.key
        if req.n_rhs > self.n_slots or self._cost(key) + self.be.gauge_bytes(key) > self.budget:
            return "refused"
        w = self.workers.get(key)
        if w is None:
            need = self._cost(key) + (0 if key in self.resident else self.be.gauge_bytes(key))
            if self.used + self.gauge_used + need > self.budget:
                self._make_room(need, key)
            if self.used + self.gauge_used + need > self.budget:
                return "parked"
            try:
                sess = self.be.open_session(key, self.n_slots)
            except Exception as e:
                req.status, req.t_done = f"failed: {e}", time.perf_counter()
                return "failed"
            if key not in self.resident:
                self.resident[key] = self.be.gauge_bytes(key)
                self.gauge_used += self.resident[key]
            self.used += self._cost(key)
            self.peak_used = max(self.peak_used, self.used + self.gauge_used)
            w = _Worker(self, key, sess, self.n_slots)
            self.workers[key] = w
            w.start()
        self.resident.move_to_end(key)
        w.q.put(req)
        return "queued"

    def _make_room(self, need, keep):
        """Close idle sessions, then evict the gauge fields of keys without a
        session (least recently used first, never ``keep``), until ``need``
        more bytes fit or nothing more can go."""
        for key, w in sorted(self.workers.items(), key=lambda kw: kw[1].last_busy):
            if self.used + self.gauge_used + need <= self.budget:
                return
            if w.idle():
                w.stop_flag = True
                w.join()
                del self.workers[key]
                self.used -= self._cost(key)
        for key in list(self.resident):
            if self.used + self.gauge_used + need <= self.budget:
                return
            if key == keep or key in self.workers:
                continue
            self.gauge_used -= self.resident.pop(key)
            self.be.drop_gauge(key)

    def run(self, requests: list, realtime: bool = True, on_progress: Callable | None = None) -> dict:
        """Replay the stream (sleeping until each arrival when realtime) and wait
        until every request is done, failed or refused.  Returns the report."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        refused = []
        i = 0
        n = len(reqs)
        while i < n or self.parked:
            now = time.perf_counter() - t0
            while i < n and (not realtime or reqs[i].arrival <= now):
                r = reqs[i]
                r.t_arrive = t0 + r.arrival if realtime else time.perf_counter()
                with self.lock:
                    out = self._route(r)
                if out == "refused":
                    r.status, r.t_done = "refused", r.t_arrive
                    refused.append(r)
                elif out == "parked":
                    self.parked.append(r)
                elif out == "failed":
                    self._finish(r)
                i += 1
            if self.parked:
                with self.lock:
                    still = []
                    for r in self.parked:
                        out = self._route(r)
                        if out == "parked":
                            still.append(r)
                    self.parked = still
            if on_progress:
                on_progress(len(self.done), n)
            if i < n:
                wait = reqs[i].arrival - (time.perf_counter() - t0) if realtime else 0
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif self.parked:
                time.sleep(0.002)
        with self.cv:
            while len(self.done) + len(refused) < n:
                self.cv.wait(timeout=1.0)
                if on_progress:
                    on_progress(len(self.done), n)
        t_end = time.perf_counter()
        for w in self.workers.values():
            w.stop_flag = True
        for w in self.workers.values():
            w.join()
        self.workers.clear()
        return self.report(reqs, t_end - t0)

    def report(self, reqs, wall):
        ok = [r for r in reqs if r.status == "done"]
        lat = np.array([r.latency() for r in ok]) if ok else np.zeros(0)
        svc = np.array([r.t_done - r.t_admit for r in ok]) if ok else np.zeros(0)
        rhs = sum(r.n_rhs for r in ok)
        return {
            "requests": len(reqs),
            "done": len(ok),
            "failed": sum(1 for r in reqs if r.status.startswith("failed")),
            "refused": sum(1 for r in reqs if r.status == "refused"),
            "wall_s": wall,
            "rhs_solves_per_s": rhs / wall if wall > 0 else 0.0,
            "requests_per_s": len(ok) / wall if wall > 0 else 0.0,
            "latency_s": {"p50": float(np.percentile(lat, 50)) if len(lat) else None,
                          "p99": float(np.percentile(lat, 99)) if len(lat) else None,
                          "max": float(lat.max()) if len(lat) else None},
            "service_s": {"p50": float(np.percentile(svc, 50)) if len(svc) else None,
                          "p99": float(np.percentile(svc, 99)) if len(svc) else None},
            "hbm_budget": self.budget,
            "hbm_peak": self.peak_used,
            "max_true_rel_resid": max((max(r.true_rel_resid) for r in ok), default=None),
        }


def jsonl(reqs, path):
    with open(path, "w") as f:
        for r in reqs:
            f.write(json.dumps({"rid": r.rid, "dims": r.dims, "nc": r.nc, "rep": r.rep, "kappa": r.kappa,
                                "n_rhs": r.n_rhs, "status": r.status, "arrival": r.arrival,
                                "latency_s": r.latency(), "iters": r.iters,
                                "true_rel_resid": r.true_rel_resid}) + "\n")
