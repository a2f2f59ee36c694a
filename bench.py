"""Benchmark: one full solve request on the SU(3) fundamental 32^4 workload.

A step is one pass of the whole hot path over one batch of synthetic input:
representation map + packing of the resident gauge field, packing of the
source, b'_e = b_e + kappa H_eo b_o, FP64 CG on the even/odd Schur normal
equations to a true relative residual of 1e-10, reconstruction of the odd
sites, the FP64 residual of the full D_W, and unpacking of the solution.
Inputs (links U = exp(i 0.3 H), H traceless GUE, reunitarised; Gaussian
source) are seeded and already resident in HBM when the timed region starts.

Prints one JSON line: solves/s as ``value``, the roofline of the dominant
hopping-kernel instance measured with HIP events inside the timed steps, and
the CPU oracle timed on a bounded sample as ``cpu_baseline``.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D_W GB/s & % HBM roofline; CG solves/s at 1e-10 resid vs FP64; p99 latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hop_traffic_su3_fund_32x4_f64.json")

WORKLOAD = {
    "workload": "su3_fund_32^4_eo_cg_fp64",
    "lattice": [32, 32, 32, 32],
    "gauge": "SU(3) fundamental, near-thermal U = exp(i 0.3 H), H traceless GUE, reunitarised",
    "source": "Gaussian complex spinor, Re/Im ~ N(0, 1/2)",
    "kappa": 0.135,
    "theta": "antiperiodic time (pi, 0, 0, 0)",
    "system": "D x = b via even/odd Schur complement, CG on its normal equations",
    "inner_dtype": "f64",
    "tol": 1e-10,
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle CG iterations in the CPU sample (0 = auto)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import fixtures as fx
    from paper_2405_19294_amd import hrw

    hrw.load()
    dev = torch.device("cuda:0")
    dims = tuple(WORKLOAD["lattice"])
    nc, rep, kappa = 3, "fund", WORKLOAD["kappa"]
    theta = (np.pi, 0.0, 0.0, 0.0)

    t0 = time.time()
    uf = fx.gauge_field(dims, nc, "thermal", seed=2, eps=0.3)
    b = fx.gaussian_spinor(dims, 3, seed=3)
    log(f"inputs generated in {time.time() - t0:.1f}s")
    uf_d = torch.from_numpy(uf).to(dev)
    b_d = torch.from_numpy(b).to(dev)
    prm = hrw.solve_params(tol=WORKLOAD["tol"], max_iter=5000, system="d_cgnr_eo", inner_dtype="f64",
                           theta=theta)
    # buffers sized once; steps reuse them (torch's caching allocator holds them)
    storage = hrw.gauge_storage_size(dims, nc, rep, ("f64",))
    ws = hrw.Workspace(hrw.workspace_size(dims, nc, rep, 1, prm), dev)
    x_d = torch.empty_like(b_d)
    stream = torch.cuda.current_stream()

    def step():
        g = hrw.Gauge(dims, nc, rep, uf_d, dtypes=("f64",))
        x, res, rc = hrw.cg_solve(g, b_d, kappa, prm, x=x_d, ws=ws)
        g.close()
        if rc != 0:
            raise RuntimeError(f"solve failed: {res}")
        return res[0]

    for _ in range(args.warmup):
        r = step()
        log(f"warmup solve: {r['iters']} iterations, true residual {r['true_rel_resid']:.2e}")

    torch.cuda.synchronize()
    hrw.timing_enable(True)
    lat = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        r = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        log(f"step {k}: {lat[-1] * 1e3:.1f} ms, {r['iters']} iterations, |b-Dx|/|b| = {r['d_rel_resid']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    classes = {name: hrw.timing_read(k) for k, name in [(0, "hop_all"), (3, "hop_plain"), (4, "hop_axpy"),
                                                         (5, "hop_cg")]}
    hrw.timing_enable(False)
    ms_per_step = elapsed / args.steps * 1e3

    # dominant hopping-kernel instance class (largest summed time)
    dom_name = max(("hop_plain", "hop_axpy", "hop_cg"), key=lambda n: classes[n]["ms"])
    dom = classes[dom_name]
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9 if dom["ms"] > 0 else 0.0
    allhop = classes["hop_all"]
    # HBM bytes per launch from the committed counter record, if it was taken
    # with the current kernel sources (None otherwise)
    from paper_2405_19294_amd import profsum
    epi_tag = {"hop_plain": ", 0>", "hop_axpy": ", 1>", "hop_cg": ", 2>"}[dom_name]
    traffic = profsum.traffic_for("hop_kernel<3, 3, double, false" + epi_tag, TRAFFIC_RECORD)
    roofline = {
        "bound": "hbm",
        "kernel": f"hop_kernel<N_R=3, RS=3, double, {dom_name[4:]} epilogue>",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": round(traffic) if traffic else None,
        "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE, calibrated on a 1 GiB copy)",
        "avg_launch_us": round(dom["ms"] / max(dom["launches"], 1) * 1e3, 2),
        "bytes_per_launch": round(dom["bytes"] / max(dom["launches"], 1)),
        "launches": dom["launches"],
        "all_hop_kernels_gbs": round(allhop["bytes"] / (allhop["ms"] * 1e-3) / 1e9, 1) if allhop["ms"] else 0,
        "hop_share_of_step": round(allhop["ms"] / (elapsed * 1e3), 3),
    }

    out = {
        "metric": METRIC,
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": WORKLOAD,
        "roofline": roofline,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "solve": {"iters": r["iters"], "true_rel_resid": r["true_rel_resid"], "d_rel_resid": r["d_rel_resid"]},
    }

    out["hbm_copy_reference"] = copy_reference(torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dims, uf, b, kappa, theta, r["iters"], args.cpu_iters)
    print(json.dumps(out), flush=True)


def copy_reference(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy of 1 GiB (torch's copy kernel): the attainable
    streaming bandwidth on this GPU, and the known-size kernel the HBM byte
    counters are calibrated against."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    bb = torch.empty_like(a)
    bb.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bb.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_per_copy": 2 * nbytes, "avg_us": round(ms * 1e3, 2),
            "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def cpu_baseline(dims, uf, b, kappa, theta, gpu_iters, cpu_iters):
    """The CPU oracle (as it stands) on a bounded sample of the same solve.

    Times a few iterations of the oracle's FP64 CG on the same even/odd system
    and extrapolates to the iteration count of the full solve.
    """
    import oracle as orc

    threads = orc.num_threads()
    ur = orc.rep_map(3, "fund", uf)
    be, bo = orc.split_eo(dims, b)
    t0 = time.perf_counter()
    bpe = be + kappa * orc.hop_eo(dims, ur, bo, 0, theta)
    eta = orc.deo(dims, ur, kappa, bpe, theta, dagger=True)
    t_prep = time.perf_counter() - t0
    n = cpu_iters or 0
    if n <= 0:
        # size the sample to roughly 15 s from the cost of one D_hat apply
        t1 = time.perf_counter()
        orc.deo(dims, ur, kappa, be, theta)
        t_apply = time.perf_counter() - t1
        n = int(max(1, min(20, 15.0 / max(2 * t_apply, 1e-3))))
    t1 = time.perf_counter()
    orc.cg(dims, ur, kappa, eta, theta, orc.SYSTEM_EO, tol=1e-10, max_iter=n)
    t_cg = time.perf_counter() - t1
    per_iter = t_cg / n
    est_solve = t_prep + per_iter * gpu_iters
    log(f"cpu oracle: {n} CG iterations in {t_cg:.1f}s on {threads} threads ({cpu_model()})")
    return {
        "value": round(1.0 / est_solve, 6),
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{n} iterations of the oracle's FP64 CG on the same 32^4 even/odd system "
                   f"({per_iter:.2f} s/iteration incl. the final true-residual check) plus the "
                   f"b' and eta preparation ({t_prep:.2f} s), extrapolated to the GPU solve's "
                   f"{gpu_iters} iterations; host CPU: {cpu_model()}"),
    }


if __name__ == "__main__":
    main()
