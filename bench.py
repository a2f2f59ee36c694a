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
                       [--workload c2|c1|c3|c4|c5|ops|bicgstab]

The default workload (c2) is the one the headline numbers are quoted on; the
others print the same kind of JSON line for the remaining configurations:
c1 SU(2) fund 4^4 (latency-bound), c3 SU(2) adj / SU(4) asym 24^3x48 mixed
precision, c4 SU(3) sym 32^4 multi-source, c5 the serving stream, ops the operator table
over the four representations, bicgstab the default request solved by BiCGstab, clover the
same request with the clover term (c_sw = 1) solved by BiCGstab.
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
# inside timed solves the library times one hopping launch in TIMING_EVERY of each epilogue
# class with HIP events (odd, so launches that repeat in pairs are both sampled): timing every
# launch added two event records per hop, about 4 ms to a 78 ms solve
TIMING_EVERY = 9
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
    "links": "SU(3) two-row: the hops read two rows of each link and rebuild the third",
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
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed solve (and the 1 GiB copy the counters are calibrated on): no "
                         "stored-link, operator, BiCGstab, four-representation or multi-source rows")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle CG iterations in the CPU sample (0 = auto)")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "ops", "bicgstab", "clover"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload != "c2":
        out = {"c1": workload_c1, "c3": workload_c3, "c4": workload_c4, "c5": workload_c5,
               "ops": workload_ops, "bicgstab": workload_bicgstab, "clover": workload_clover}[args.workload](args)
        print(json.dumps(out), flush=True)
        return

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
        g = hrw.Gauge(dims, nc, rep, uf_d, dtypes=("f64",), two_rows=True)
        x, res, rc = hrw.cg_solve(g, b_d, kappa, prm, x=x_d, ws=ws)
        g.close()
        if rc != 0:
            raise RuntimeError(f"solve failed: {res}")
        return res[0]

    for _ in range(args.warmup):
        r = step()
        log(f"warmup solve: {r['iters']} iterations, true residual {r['true_rel_resid']:.2e}")

    torch.cuda.synchronize()
    hrw.timing_enable(True, every=TIMING_EVERY)
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
    # (the instance name continues with the staging flag: "<double, false, 0, false>")
    epi_tag = {"hop_plain": "false, 0,", "hop_axpy": "false, 1,", "hop_cg": "true, 2,"}[dom_name]
    traffic = profsum.traffic_for("hop_su3_kernel<double, " + epi_tag, TRAFFIC_RECORD)
    roofline = {
        "bound": "hbm",
        "kernel": f"hop_su3_kernel<double, {dom_name[4:]} epilogue> (two rows of each link read, third rebuilt)",
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
        # the timed launches are one in TIMING_EVERY of each class
        "hop_share_of_step": round(allhop["ms"] * TIMING_EVERY / (elapsed * 1e3), 3),
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
    # after the timed steps (context; the timed region above is unchanged): the same request
    # with stored links, single operator applies, BiCGstab, the operator table over the four
    # representations and the multi-source workload's ratios
    if not args.no_extras:
        out["stored_links"] = stored_link_row(torch, hrw, dims, nc, rep, uf_d, b_d, kappa, prm, ws, x_d,
                                              out["value"], max(2, min(args.steps, 5)))
        out["operators"] = operator_table(torch, hrw, dev, dims, nc, rep, uf_d, kappa, theta,
                                          out["hbm_copy_reference"]["gbs"])
        out["bicgstab"] = bicgstab_rows(torch, hrw, dev, dims, nc, rep, uf_d, b_d, kappa, theta, out["value"],
                                        max(2, min(args.steps, 5)))
        del x_d, ws
        torch.cuda.empty_cache()
        out["operators_4_reps"] = four_rep_table(torch, hrw, dev, kappa, theta, out["hbm_copy_reference"]["gbs"])
        c4 = c4_rows(torch, hrw, dev, 1, extras=False)
        out["c4_multi_source"] = {"fp64_cg": c4["fp64_cg"], "multi_source": c4["multi_source"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dims, uf, b, kappa, theta, r["iters"], args.cpu_iters)
    print(json.dumps(out), flush=True)


def workload_bicgstab(args):
    """The default workload's request solved by BiCGstab on D_hat (BF16 inner storage with FP32
    arithmetic and FP64 reliable updates as the line's value; FP32 inner and plain FP64 beside it),
    against FP64 CG on the normal equations; the roofline is that of the hopping kernel inside the
    BF16-inner solves."""
    import torch

    import fixtures as fx
    from paper_2405_19294_amd import hrw
    dev = torch.device("cuda:0")
    dims = tuple(WORKLOAD["lattice"])
    kappa, theta = WORKLOAD["kappa"], (np.pi, 0.0, 0.0, 0.0)
    uf_d = torch.from_numpy(fx.gauge_field(dims, 3, "thermal", seed=2, eps=0.3)).to(dev)
    b_d = torch.from_numpy(fx.gaussian_spinor(dims, 3, seed=3)).to(dev)
    prm = hrw.solve_params(tol=WORKLOAD["tol"], max_iter=5000, system="d_cgnr_eo", inner_dtype="f64", theta=theta)
    g = hrw.Gauge(dims, 3, "fund", uf_d, dtypes=("f64",), two_rows=True)
    _, _, per_cg, _ = _solve_timed(hrw, torch, g, b_d, kappa, prm, max(1, args.steps // 2), 1)
    g.close()
    rows = bicgstab_rows(torch, hrw, dev, dims, 3, "fund", uf_d, b_d, kappa, theta, 1.0 / per_cg, args.steps,
                         order=("bf16", "f32", "f64"), timed="bf16")
    roof = rows.pop("roofline")
    # the same request by QMR-g5 (FP64, one D_hat application per iteration)
    g = hrw.Gauge(dims, 3, "fund", uf_d, dtypes=("f64",), two_rows=True)
    prm_q = hrw.solve_params(tol=WORKLOAD["tol"], max_iter=5000, system="d_eo", theta=theta)
    _, res_q, per_q, _ = _solve_timed(hrw, torch, g, b_d, kappa, prm_q, max(1, args.steps // 2), 1,
                                      solver=hrw.qmr_g5_solve)
    g.close()
    rows["qmr_g5_f64"] = {"solves_per_s": round(1.0 / per_q, 3), "ms_per_solve": round(per_q * 1e3, 2),
                          "iters": res_q[0]["iters"], "dhat_applies": res_q[0]["iters"],
                          "restarts": res_q[0]["restarts"], "true_rel_resid": res_q[0]["true_rel_resid"],
                          "d_rel_resid": res_q[0]["d_rel_resid"], "vs_fp64_cg": round(per_cg / per_q, 3)}
    log(f"QMR-g5 f64: {rows['qmr_g5_f64']}")
    cfg = dict(WORKLOAD, workload="su3_fund_32^4_eo_bicgstab_mixed_bf16",
               system="D x = b via even/odd Schur complement, BiCGstab on D_hat",
               inner_dtype="bf16 storage, f32 arithmetic", reliable_every=50,
               reliable_delta=hrw.RELIABLE_DELTA["bf16"])
    m = rows["bf16"]
    return _line(m["solves_per_s"], "solves/s", args.steps, 1, m["ms_per_solve"], "bf16", cfg, roof,
                 bicgstab=rows, fp64_cg_solves_per_s=round(1.0 / per_cg, 3))


def workload_clover(args):
    """The default workload's gauge field and source with the clover term (c_sw = 1): clover setup,
    D_sw and D_hat_sw applies in FP64 and FP32, and D_sw x = b by BiCGstab on D_hat_sw (FP64, and
    FP32 inner fields with FP64 reliable updates; the line's value) beside the same request
    without the clover term.  The field is flagged special unitary: the hops read two rows of each
    SU(3) link (the clover builder reads the stored three)."""
    import torch

    import fixtures as fx
    from paper_2405_19294_amd import hrw
    dev = torch.device("cuda:0")
    dims = tuple(WORKLOAD["lattice"])
    kappa, csw, theta = WORKLOAD["kappa"], 1.0, (np.pi, 0.0, 0.0, 0.0)
    uf_d = torch.from_numpy(fx.gauge_field(dims, 3, "thermal", seed=2, eps=0.3)).to(dev)
    b_d = torch.from_numpy(fx.gaussian_spinor(dims, 3, seed=3)).to(dev)
    g = hrw.Gauge(dims, 3, "fund", uf_d, dtypes=("f64", "f32"), two_rows=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = hrw.Clover(g, kappa, csw, dtypes=("f64", "f32"))
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    v = int(np.prod(dims))
    pe = b_d[: v // 2].contiguous()
    ops = {}
    for dt in ("f64", "f32"):
        for name, fn, arg in (("dsw", hrw.dsw_apply, b_d), ("dsw_eo", hrw.dsw_eo_apply, pe)):
            out = torch.empty_like(arg)
            ws = hrw.Workspace.for_apply(g, 1)
            for _ in range(3):
                fn(c, arg, theta, dt, out=out, ws=ws)
            torch.cuda.synchronize()
            hrw.timing_enable(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn(c, arg, theta, dt, out=out, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            hop = hrw.timing_read(0)
            hrw.timing_enable(False)
            ops[f"{name}_{dt}"] = {"call_us": round(e0.elapsed_time(e1) * 1e3 / 20, 1),
                                   "hop_us": round(hop["ms"] * 1e3 / 20, 1)}
            log(f"clover {name} {dt}: {ops[f'{name}_{dt}']}")
    rows, roof = {}, None
    for inner in ("f32", "f64"):
        prm = hrw.solve_params(tol=WORKLOAD["tol"], max_iter=5000, system="d_eo", inner_dtype=inner, theta=theta,
                               reliable_delta=hrw.RELIABLE_DELTA[inner])
        hrw.clover_bicgstab_solve(c, b_d, prm)
        torch.cuda.synchronize()
        if inner == "f32":
            hrw.timing_enable(True, every=TIMING_EVERY)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, res, rc = hrw.clover_bicgstab_solve(c, b_d, prm)
            if rc != 0:
                raise RuntimeError(f"clover solve failed: {res}")
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.steps
        if inner == "f32":
            roof = _hop_roofline(hrw, "hop_su3_kernel<float> (two rows of each link read; with the FP64 launches "
                                      "of the updates)")
            hrw.timing_enable(False)
        r = res[0]
        rows[inner] = {"solves_per_s": round(1.0 / per, 3), "ms_per_solve": round(per * 1e3, 2), "iters": r["iters"],
                       "reliable_updates": r["reliable_updates"], "restarts": r["restarts"],
                       "true_rel_resid": r["true_rel_resid"], "d_rel_resid": r["d_rel_resid"]}
        log(f"clover BiCGstab {inner}: {rows[inner]}")
    c.close()
    # the same request without the clover term
    prm = hrw.solve_params(tol=WORKLOAD["tol"], max_iter=5000, system="d_eo", inner_dtype="f32", theta=theta,
                           reliable_delta=hrw.RELIABLE_DELTA["f32"])
    _, res0, per0, _ = _solve_timed(hrw, torch, g, b_d, kappa, prm, max(1, args.steps // 2), 1,
                                    solver=hrw.bicgstab_solve)
    g.close()
    cfg = dict(WORKLOAD, workload="su3_fund_32^4_clover_eo_bicgstab_mixed_f32", c_sw=csw,
               system="D_sw x = b via even/odd Schur complement (A_ee - kappa^2 H_eo A_oo^-1 H_oe), BiCGstab",
               inner_dtype="f32", reliable_every=50, reliable_delta=1e-3,
               links="SU(3) two-row: the hops read two rows of each link and rebuild the third")
    m = rows["f32"]
    return _line(m["solves_per_s"], "solves/s", args.steps, 1, m["ms_per_solve"], "f32", cfg, roof,
                 clover_setup_ms=round(setup_ms, 1), operators=ops, bicgstab=rows,
                 without_clover_f32={"solves_per_s": round(1.0 / per0, 3), "iters": res0[0]["iters"]})


def stored_link_row(torch, hrw, dims, nc, rep, uf_d, b_d, kappa, prm, ws, x_d, two_row_value, steps):
    """The same FP64 CG request with the hops reading all three stored rows of each link (the
    paper's full-link storage), beside the line's two-row solve."""
    def step():
        g = hrw.Gauge(dims, nc, rep, uf_d, dtypes=("f64",))
        x, res, rc = hrw.cg_solve(g, b_d, kappa, prm, x=x_d, ws=ws)
        g.close()
        if rc != 0:
            raise RuntimeError(f"stored-link solve failed: {res}")
        return res[0]

    step()
    torch.cuda.synchronize()
    hrw.timing_enable(True, every=TIMING_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    roof = _hop_roofline(hrw, "hop_kernel<N_R=3, RS=3, double> (all three rows read)")
    hrw.timing_enable(False)
    row = {"solves_per_s": round(steps / el, 3), "ms_per_solve": round(el / steps * 1e3, 2), "iters": r["iters"],
           "true_rel_resid": r["true_rel_resid"], "d_rel_resid": r["d_rel_resid"],
           "two_row_speedup": round(two_row_value / (steps / el), 3), "steps": steps, "hop_roofline": roof}
    log(f"FP64 CG, stored links (three rows): {row}")
    return row


def bicgstab_rows(torch, hrw, dev, dims, nc, rep, uf_d, b_d, kappa, theta, cg_value, steps,
                  order=("f64", "f32"), timed=None, two_rows=True):
    """The same request (D x = b through the even/odd Schur complement, |b'_e - D_hat x_e| <= 1e-10
    |b'_e| in FP64) solved by BiCGstab on D_hat itself: plain FP64, and FP32 inner fields with FP64
    reliable updates (BF16 storage with FP32 arithmetic likewise).  A step is the whole request as in the main line (gauge field built, solve,
    reconstruction, |b - D x|); solves/s beside CG's."""
    rows = {}
    for inner in order:
        dtypes = ("f64",) if inner == "f64" else ("f64", inner)
        prm = hrw.solve_params(tol=WORKLOAD["tol"], max_iter=5000, system="d_eo", inner_dtype=inner, theta=theta,
                               reliable_delta=hrw.RELIABLE_DELTA[inner])
        ws = hrw.Workspace(hrw.workspace_size(dims, nc, rep, 1, prm), dev)
        x_d = torch.empty_like(b_d)

        def step():
            g = hrw.Gauge(dims, nc, rep, uf_d, dtypes=dtypes, two_rows=two_rows)
            x, res, rc = hrw.bicgstab_solve(g, b_d, kappa, prm, x=x_d, ws=ws)
            g.close()
            if rc != 0:
                raise RuntimeError(f"BiCGstab solve failed: {res}")
            return res[0]

        step()
        torch.cuda.synchronize()
        if timed == inner:
            hrw.timing_enable(True, every=TIMING_EVERY)
        t0 = time.perf_counter()
        for _ in range(steps):
            r = step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if timed == inner:
            kt = {"f64": "double", "f32": "float", "bf16": "bf16"}[inner]
            extra = "" if inner == "f64" else " (the class also holds the few FP64 launches of the reliable updates)"
            name = f"hop_su3_kernel<{kt}> (two rows of each link read)" if two_rows else f"hop_kernel<N_R=3, RS=3, {kt}>"
            rows["roofline"] = _hop_roofline(hrw, name + extra)
            hrw.timing_enable(False)
        rows[inner] = {"solves_per_s": round(steps / el, 3), "ms_per_solve": round(el / steps * 1e3, 2),
                       "iters": r["iters"], "dhat_applies": 2 * r["iters"],
                       "reliable_updates": r["reliable_updates"], "restarts": r["restarts"],
                       "true_rel_resid": r["true_rel_resid"], "d_rel_resid": r["d_rel_resid"],
                       "vs_fp64_cg": round(steps / el / cg_value, 3), "steps": steps}
        log(f"BiCGstab {inner}: {rows[inner]}")
        del ws
    return rows


def operator_table(torch, hrw, dev, dims, nc, rep, uf_d, kappa, theta, copy_gbs, reps=20, fused=False,
                   two_rows=False):
    """Single applies of D_W (full lattice) and D_hat (even sites) in FP64 and FP32.

    fused: the gauge field keeps its fundamental links and the hops build U_R in registers; the
    byte models then count the N_F x N_F fundamental links (N_F^2 in place of N^2 in the link terms).
    two_rows (SU(3) fundamental): the hops read two rows of each link, 6 complex in place of N^2.

    Per call: the hopping kernels' time from HIP events on the launch stream
    (library timing) and the whole call (canonical-layout packing included).
    Byte and flop models per unit, N = N_R, c = bytes per complex:
      D_W   per site:      min traffic (every link once) c (4N^2 + 8N);
                           as streamed (each link read by both of its sites) c (8N^2 + 12N);
                           flops 128N^2 + 72N
      D_hat per even site: c (16N^2 + 20N) (min traffic = as streamed);
                           flops 2 (128N^2 + 56N) + 8N
    """
    v = int(np.prod(dims))
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    g = hrw.Gauge(dims, nc, rep, uf_d, dtypes=("f64", "f32"), fused=fused, two_rows=two_rows)
    n = g.nr
    nl = nc if fused else n  # dimension of the streamed links
    lc = 6 if two_rows else nl * nl  # complex numbers of each link the hops read
    psi = torch.complex(torch.randn((v, 4, n), generator=gen, device=dev, dtype=torch.float64),
                        torch.randn((v, 4, n), generator=gen, device=dev, dtype=torch.float64)) * np.sqrt(0.5)
    pe = psi[: v // 2].contiguous()
    out_f, out_e = torch.empty_like(psi), torch.empty_like(pe)
    ws = hrw.Workspace.for_apply(g, 1)
    rows = {}
    for dt, cb in (("f64", 16), ("f32", 8)):
        for op in ("dw", "deo"):
            def call():
                if op == "dw":
                    hrw.dw_apply(g, kappa, psi, theta, dt, out=out_f, ws=ws)
                else:
                    hrw.deo_apply(g, kappa, pe, theta, dt, out=out_e, ws=ws)
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            hrw.timing_enable(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            hop = hrw.timing_read(0)
            hrw.timing_enable(False)
            hop_us = hop["ms"] * 1e3 / reps
            if op == "dw":
                b_min = cb * (4 * lc + 8 * n) * v
                b_str = cb * (8 * lc + 12 * n) * v
                flops = (128 * n * n + 72 * n) * v
            else:
                b_min = b_str = cb * (16 * lc + 20 * n) * (v // 2)
                flops = (2 * (128 * n * n + 56 * n) + 8 * n) * (v // 2)
            gbs = b_min / (hop_us * 1e-6) / 1e9
            rows[f"{op}_{dt}"] = {
                "hop_us": round(hop_us, 1), "call_us": round(e0.elapsed_time(e1) * 1e3 / reps, 1),
                "bytes_min": b_min, "GBs_min": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                "frac_of_copy": round(gbs / copy_gbs, 3),
                "GBs_as_streamed": round(b_str / (hop_us * 1e-6) / 1e9, 1),
                "GFLOPs": round(flops / (hop_us * 1e-6) / 1e9, 1)}
            log(f"{op} {dt}{' fused' if fused else ''}{' two-row' if two_rows else ''}: {rows[f'{op}_{dt}']}")
    g.close()
    return rows


# ---------------------------------------------------------------- other workloads

def _line(metric_value, unit, steps, warmup, ms_per_step, dtype, config, roofline, **extra):
    out = {"metric": METRIC, "value": metric_value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline}
    out.update(extra)
    return out


def _hop_roofline(hrw, kernel_label):
    """Roofline of the hopping-kernel class with the most summed time since timing_enable."""
    classes = {n: hrw.timing_read(k) for k, n in [(3, "plain"), (4, "axpy"), (5, "cg")]}
    name = max(classes, key=lambda n: classes[n]["ms"])
    c = classes[name]
    if not c["ms"]:
        return None
    ach = c["bytes"] / (c["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": f"{kernel_label}, {name} epilogue", "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_us": round(c["ms"] / c["launches"] * 1e3, 2),
            "bytes_per_launch": round(c["bytes"] / c["launches"]), "launches": c["launches"]}


def _even_part(dims, full):
    x = np.indices(tuple(dims)).reshape(4, -1)
    return np.ascontiguousarray(full[..., (x.sum(axis=0) & 1) == 0, :, :])


def _solve_timed(hrw, torch, g, b, kappa, prm, steps, warmup, solver=None):
    solver = solver or hrw.cg_solve
    for _ in range(warmup):
        solver(g, b, kappa, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    for _ in range(steps):
        ts = time.perf_counter()
        x, res, rc = solver(g, b, kappa, prm)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        if rc != 0:
            raise RuntimeError(f"solve failed: {res}")
    return x, res, (time.perf_counter() - t0) / steps, lat


def workload_c1(args):
    """SU(2) fund 4^4, Haar links, kappa 0.12, antiperiodic: D_W apply + FP64 CG on D^+D (full lattice)."""
    import torch

    import fixtures as fx
    from paper_2405_19294_amd import hrw
    dev = torch.device("cuda:0")
    dims, kappa, theta = (4, 4, 4, 4), 0.12, (np.pi, 0, 0, 0)
    uf = torch.from_numpy(fx.gauge_field(dims, 2, "haar", seed=1)).to(dev)
    psi = torch.from_numpy(fx.gaussian_spinor(dims, 2, seed=2)).to(dev)
    g = hrw.Gauge(dims, 2, "fund", uf, dtypes=("f64",))
    ws = hrw.Workspace.for_apply(g, 1)
    out = torch.empty_like(psi)
    for _ in range(10):
        hrw.dw_apply(g, kappa, psi, theta, out=out, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(200):
        hrw.dw_apply(g, kappa, psi, theta, out=out, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    apply_us = e0.elapsed_time(e1) / 200 * 1e3
    prm = hrw.solve_params(tol=1e-10, system="ddag_d_full", theta=theta)
    for _ in range(args.warmup):
        hrw.cg_solve(g, psi, kappa, prm)
    torch.cuda.synchronize()
    hrw.timing_enable(True, every=TIMING_EVERY)
    x, res, per, lat = _solve_timed(hrw, torch, g, psi, kappa, prm, max(args.steps, 20), 0)
    roof = _hop_roofline(hrw, "hop_kernel<N_R=2, double>")
    hrw.timing_enable(False)
    return _line(round(1.0 / per, 2), "solves/s", max(args.steps, 20), args.warmup, round(per * 1e3, 3), "f64",
                 {"workload": "su2_fund_4^4_cg_fp64_full", "lattice": list(dims), "kappa": kappa,
                  "gauge": "Haar SU(2)", "system": "D^+D x = b, full lattice", "tol": 1e-10},
                 roof, dw_apply_us=round(apply_us, 2),
                 note="latency-bound: 256 sites (0.13 MB per apply), so no GB/s claim; the apply time includes "
                      "packing and unpacking of the canonical fields",
                 latency_ms={"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
                 solve={"iters": res[0]["iters"], "true_rel_resid": res[0]["true_rel_resid"]})


def workload_c3(args):
    """24^3x48 SU(2) adj and SU(4) asym, U_R built on the device: FP64 / FP32 / BF16 / FP16-storage CG,
    each with the stored U_R and with the representation map fused into the hop."""
    import torch

    import fixtures as fx
    from paper_2405_19294_amd import hrw
    dev = torch.device("cuda:0")
    dims, kappa, theta = (48, 24, 24, 24), 0.135, (np.pi, 0, 0, 0)
    cases, roof, main = [], None, None
    for nc, rep in [(2, "adj"), (4, "asym")]:
        t0 = time.time()
        uf = torch.from_numpy(fx.gauge_field(dims, nc, "thermal", seed=3, eps=0.3)).to(dev)
        log(f"c3 SU({nc}) links in {time.time() - t0:.1f}s")
        g = hrw.Gauge(dims, nc, rep, uf, dtypes=("f64", "f32", "bf16", "f16"))
        # the same field with the representation map fused into the single-source hops
        gf = hrw.Gauge(dims, nc, rep, uf, dtypes=("f64", "f32", "bf16", "f16"), fused=True)
        del uf
        b = torch.from_numpy(_even_part(dims, fx.gaussian_spinor(dims, g.nr, seed=4))).to(dev)
        ref = None
        stored_rate = {}
        for fused, inner in [(False, d) for d in ("f64", "f32", "bf16", "f16")] + \
                            [(True, d) for d in ("f64", "f32", "bf16", "f16")]:
            gg = gf if fused else g
            prm = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype=inner,
                                   reliable_every=50, reliable_delta=hrw.RELIABLE_DELTA[inner], theta=theta)
            for _ in range(args.warmup):
                hrw.cg_solve(gg, b, kappa, prm)
            torch.cuda.synchronize()
            hrw.timing_enable(True, every=TIMING_EVERY)
            x, res, per, lat = _solve_timed(hrw, torch, gg, b, kappa, prm, args.steps, 0)
            kname = "hop_fused_kernel" if fused else "hop_kernel"
            r = _hop_roofline(hrw, f"{kname}<N_R={g.nr}, {inner}>")
            hrw.timing_enable(False)
            if inner == "f64" and not fused:
                ref = x.clone()
            err = float((torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref)).item())
            case = {"rep": f"SU({nc}) {rep}", "n_r": g.nr, "inner": inner, "fused_rep_map": fused,
                    "solves_per_s": round(1.0 / per, 3),
                    "ms_per_solve": round(per * 1e3, 2), "iters": res[0]["iters"],
                    "reliable_updates": res[0]["reliable_updates"], "true_rel_resid": res[0]["true_rel_resid"],
                    "rel_error_vs_fp64": err, "hop_roofline": r}
            if fused:
                case["speedup_vs_stored_links"] = round(1.0 / per / stored_rate[inner], 3)
                case["speedup_vs_stored_fp64"] = round(1.0 / per / stored_rate["f64"], 3)
            else:
                stored_rate[inner] = 1.0 / per
            cases.append(case)
            log(f"c3 {case}")
            if nc == 4 and inner == "f32" and fused:
                main, roof = case, r
        # D_W (full lattice) apply bandwidth in FP64 and FP32 on this representation
        psi = torch.from_numpy(fx.gaussian_spinor(dims, g.nr, seed=5)).to(dev)
        ws = hrw.Workspace.for_apply(g, 1)
        out_ = torch.empty_like(psi)
        for dt in ["f64", "f32"]:
            hrw.dw_apply(g, kappa, psi, theta, dt, out=out_, ws=ws)
            torch.cuda.synchronize()
            hrw.timing_enable(True)
            for _ in range(10):
                hrw.dw_apply(g, kappa, psi, theta, dt, out=out_, ws=ws)
            torch.cuda.synchronize()
            c = hrw.timing_read(4)
            hrw.timing_enable(False)
            cases.append({"rep": f"SU({nc}) {rep}", "dw_apply_hop_" + dt: {
                "us": round(c["ms"] / c["launches"] * 1e3, 1),
                "GBs_dup_link_model": round(c["bytes"] / (c["ms"] * 1e-3) / 1e9, 1)}})
        gf.close()
        del g, gf, b, psi, ws, out_
        torch.cuda.empty_cache()
    return _line(main["solves_per_s"], "solves/s", args.steps, args.warmup, main["ms_per_solve"], "f32",
                 {"workload": "su4_asym_24^3x48_mixed_cg", "lattice": list(dims), "kappa": kappa,
                  "reps": ["SU(2) adj", "SU(4) asym"], "inner": ["f64", "f32", "bf16", "f16"],
                  "value_case": "SU(4) asym, FP32 inner, representation map fused into the hop",
                  "reliable_every": 50, "reliable_delta": hrw.RELIABLE_DELTA, "tol": 1e-10}, roof, cases=cases)


def c4_rows(torch, hrw, dev, steps, extras=True):
    """SU(3) sym 32^4, 12 and 24 point-smeared sources: multi-source mixed CG (FP32 inner,
    FP64 reliable updates) against two FP64 CG baselines on the same system, one source at a
    time and all 24 batched (links shared).  extras: also FP16 storage and BiCGstab rows."""
    import fixtures as fx
    dims, kappa, theta = (32, 32, 32, 32), 0.135, (np.pi, 0, 0, 0)
    t0 = time.time()
    uf_h = fx.gauge_field(dims, 3, "thermal", seed=6, eps=0.3)
    uf = torch.from_numpy(uf_h).to(dev)
    g = hrw.Gauge(dims, 3, "sym", uf, dtypes=("f64", "f32"))
    g_fused = hrw.Gauge(dims, 3, "sym", uf, dtypes=("f64",), fused=True) if extras else None
    del uf
    nmax = 24
    srcs = torch.empty((nmax, fx.volume(dims) // 2, 4, g.nr), dtype=torch.complex128, device=dev)
    for k in range(nmax):
        full = fx.point_smeared_sources(dims, g.nr, nmax, seed=7, which=[k])
        srcs[k] = torch.from_numpy(_even_part(dims, full)[0])
    log(f"c4 inputs in {time.time() - t0:.1f}s")
    # plain FP64 CG, one source at a time (the reference rate)
    prm64 = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype="f64", theta=theta)
    x64, res64, per64, _ = _solve_timed(hrw, torch, g, srcs[0:1].contiguous(), kappa, prm64, steps, 1)
    fp64_rate = 1.0 / per64
    # the same FP64 CG batched over all sources (links shared through LDS); one batched apply
    # first runs the launch-shape search of this source count outside the timed solve
    hrw.deo_apply(g, kappa, srcs, theta, "f64")
    torch.cuda.synchronize()
    _, res64b, per64b, _ = _solve_timed(hrw, torch, g, srcs, kappa, prm64, 1, 0)
    fp64_batched_rate = nmax / per64b
    fp64 = {"solves_per_s": round(fp64_rate, 3), "iters": res64[0]["iters"],
            "batched_24_rhs_solves_per_s": round(fp64_batched_rate, 3),
            "batched_max_iters": max(q["iters"] for q in res64b)}
    if extras:
        # FP64 CG, one source at a time, with the representation map fused into the hop
        _, res64f, per64f, _ = _solve_timed(hrw, torch, g_fused, srcs[0:1].contiguous(), kappa, prm64, steps, 1)
        g_fused.close()
        fp64["fused_rep_map_solves_per_s"] = round(1.0 / per64f, 3)
    out = {}
    roof = None
    for n in (12, 24):
        prm = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype="f32",
                               reliable_every=50, reliable_delta=hrw.RELIABLE_DELTA["f32"], theta=theta)
        b = srcs[:n].contiguous()
        # the warm-up solve runs the first-use launch-shape search, whose trial launches
        # stay out of the hop statistics
        hrw.cg_solve(g, b, kappa, prm)
        torch.cuda.synchronize()
        hrw.timing_enable(True, every=TIMING_EVERY)
        x, res, per, lat = _solve_timed(hrw, torch, g, b, kappa, prm, steps, 0)
        r = _hop_roofline(hrw, f"hop_mrhs_kernel<N_R=6, float, {n} sources>")
        hrw.timing_enable(False)
        err0 = float((torch.linalg.vector_norm(x[0] - x64[0]) / torch.linalg.vector_norm(x64[0])).item())
        out[n] = {"rhs_solves_per_s": round(n / per, 3), "ms_per_batch": round(per * 1e3, 1),
                  "speedup_vs_fp64_cg": round(n / per / fp64_rate, 2),
                  "speedup_vs_fp64_cg_batched": round(n / per / fp64_batched_rate, 2),
                  "max_iters": max(q["iters"] for q in res),
                  "max_reliable_updates": max(q["reliable_updates"] for q in res),
                  "max_true_rel_resid": max(q["true_rel_resid"] for q in res),
                  "rel_error_vs_fp64_source0": err0, "hop_roofline": r}
        if extras:
            out[n]["speedup_vs_fp64_cg_fused_rep_map"] = round(n / per * 1.0 / fp64["fused_rep_map_solves_per_s"], 2)
        log(f"c4 n={n}: {out[n]}")
        roof = r
    rows = {"fp64_cg": fp64, "multi_source": out, "roofline": roof}
    if extras:
        # the same 24 sources with FP16 storage of the inner fields (FP32 arithmetic)
        prm16 = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype="f16",
                                 reliable_every=50, reliable_delta=hrw.RELIABLE_DELTA["f16"], theta=theta)
        g16 = hrw.Gauge(dims, 3, "sym", torch.from_numpy(uf_h).to(dev), dtypes=("f64", "f16"))
        x16, res16, per16, _ = _solve_timed(hrw, torch, g16, srcs, kappa, prm16, steps, 1)
        rows["multi_source_24_f16_storage"] = {
            "rhs_solves_per_s": round(nmax / per16, 3), "ms_per_batch": round(per16 * 1e3, 1),
            "speedup_vs_fp64_cg": round(nmax / per16 / fp64_rate, 2),
            "speedup_vs_fp64_cg_batched": round(nmax / per16 / fp64_batched_rate, 2),
            "max_iters": max(q["iters"] for q in res16),
            "max_true_rel_resid": max(q["true_rel_resid"] for q in res16),
            "rel_error_vs_fp64_source0": float((torch.linalg.vector_norm(x16[0] - x64[0]) /
                                                torch.linalg.vector_norm(x64[0])).item())}
        log(f"c4 n=24 f16 storage: {rows['multi_source_24_f16_storage']}")
        g16.close()
        rows["bicgstab_propagators"] = _c4_bicgstab(hrw, torch, g, srcs, kappa, theta, steps)
    g.close()
    del srcs
    torch.cuda.empty_cache()
    return rows


def workload_c4(args):
    """SU(3) sym 32^4, 12 and 24 point-smeared sources: multi-source mixed CG vs plain FP64 CG."""
    import torch

    from paper_2405_19294_amd import hrw
    dev = torch.device("cuda:0")
    steps = max(1, args.steps // 2)
    rows = c4_rows(torch, hrw, dev, steps, extras=True)
    out = rows["multi_source"]
    return _line(out[24]["rhs_solves_per_s"], "rhs-solves/s", steps, 1, out[24]["ms_per_batch"],
                 "f32", {"workload": "su3_sym_32^4_multi_source_mixed_cg", "lattice": [32, 32, 32, 32],
                         "kappa": 0.135, "sources": "point-smeared (Gaussian spatial profile, width 2), 12 and 24",
                         "inner": "f32", "reliable_every": 50, "reliable_delta": hrw.RELIABLE_DELTA["f32"],
                         "tol": 1e-10}, rows["roofline"],
                 fp64_cg=rows["fp64_cg"], multi_source=out,
                 multi_source_24_f16_storage=rows["multi_source_24_f16_storage"],
                 bicgstab_propagators=rows["bicgstab_propagators"], hbm_copy_reference=copy_reference(torch, dev))


def _c4_bicgstab(hrw, torch, g, srcs, kappa, theta, steps):
    """The same sources as propagators, D_hat y = eta: BiCGstab on D_hat (plain FP64 one source at a
    time, and 24 sources with FP32 inner fields and FP64 reliable updates) against FP64 CG on the
    normal equations D_hat^+ D_hat y = D_hat^+ eta of the same system."""
    n = srcs.shape[0]
    eta_dag = hrw.deo_apply(g, kappa, srcs[0:1].contiguous(), theta, "f64", dagger=True)
    prm_cg = hrw.solve_params(tol=1e-10, max_iter=20000, system="ddag_d_eo", inner_dtype="f64", theta=theta)
    _, res_cg, per_cg, _ = _solve_timed(hrw, torch, g, eta_dag, kappa, prm_cg, steps, 1)
    rows = {"fp64_cgnr_solves_per_s": round(1.0 / per_cg, 3), "fp64_cgnr_iters": res_cg[0]["iters"]}
    prm64 = hrw.solve_params(tol=1e-10, max_iter=20000, system="dhat_eo", inner_dtype="f64", theta=theta)
    y64, res64, per64, _ = _solve_timed(hrw, torch, g, srcs[0:1].contiguous(), kappa, prm64, steps, 1,
                                        solver=hrw.bicgstab_solve)
    rows["fp64_bicgstab"] = {"solves_per_s": round(1.0 / per64, 3), "iters": res64[0]["iters"],
                             "vs_fp64_cgnr": round(per_cg / per64, 2)}
    prm32 = hrw.solve_params(tol=1e-10, max_iter=20000, system="dhat_eo", inner_dtype="f32", theta=theta,
                             reliable_delta=hrw.RELIABLE_DELTA["f32"])
    y, res, per, _ = _solve_timed(hrw, torch, g, srcs, kappa, prm32, steps, 1, solver=hrw.bicgstab_solve)
    rows[f"mixed_f32_{n}_sources"] = {
        "rhs_solves_per_s": round(n / per, 3), "ms_per_batch": round(per * 1e3, 1),
        "vs_fp64_cgnr": round(n / per * per_cg, 2), "max_iters": max(q["iters"] for q in res),
        "max_true_rel_resid": max(q["true_rel_resid"] for q in res),
        "rel_error_vs_fp64_source0": float((torch.linalg.vector_norm(y[0] - y64[0]) /
                                            torch.linalg.vector_norm(y64[0])).item())}
    log(f"c4 BiCGstab propagators: {rows}")
    return rows


def workload_c5(args):
    """Serving: Poisson stream (20/s, seed 5) of CG requests over 5 volumes x 4 reps, continuous batching."""
    import torch

    from paper_2405_19294_amd import serve
    be = serve.GpuBackend(inner_dtype="f32", tol=1e-10)
    reqs = serve.poisson_stream(400, rate=20.0, seed=5)
    free, total = torch.cuda.mem_get_info()
    budget = int(min(free * 0.8, 200e9))
    t0 = time.time()
    for key in sorted({r.key for r in reqs}):
        be.gauge(key)
    log(f"c5: {len({r.key for r in reqs})} resident gauge fields in {time.time() - t0:.1f}s")
    srv = serve.Server(be, hbm_budget=budget, n_slots=12, step_iters=20)
    last = [0.0]

    def progress(done, n):
        if time.time() - last[0] > 10:
            last[0] = time.time()
            log(f"c5: {done}/{n} requests done")
    rep = srv.run(reqs, realtime=True, on_progress=progress)
    lat = rep["latency_s"]
    # arrival-rate sweep: 20 s of arrivals at each lower rate (the 20/s row is
    # the main stream above); the highest rate whose p99 latency stays within
    # twice the p99 service time (at most as much queueing as service) is
    # reported as sustainable
    sweep, bounded = [], None
    for rate in (1.0, 2.0, 5.0, 10.0, 20.0):
        if rate == 20.0:
            sreqs, r = reqs, rep
        else:
            sreqs = serve.poisson_stream(int(20 * rate), rate=rate, seed=5)
            r = serve.Server(be, hbm_budget=budget, n_slots=12, step_iters=20).run(sreqs, realtime=True)
        ms = lambda v: None if v is None else round(v * 1e3, 1)  # noqa: E731
        row = {"rate_per_s": rate, "p50_ms": ms(r["latency_s"]["p50"]), "p99_ms": ms(r["latency_s"]["p99"]),
               "service_p99_ms": ms(r["service_s"]["p99"]),
               "rhs_solves_per_s": round(r["rhs_solves_per_s"], 3), "done": r["done"], "refused": r["refused"]}
        sweep.append(row)
        log(f"c5 sweep: {row}")
        if r["done"] == len(sreqs) and r["latency_s"]["p99"] <= 2.0 * r["service_s"]["p99"]:
            bounded = rate
    return _line(round(rep["rhs_solves_per_s"], 3), "rhs-solves/s", len(reqs), 0,
                 round(rep["wall_s"] * 1e3 / max(rep["done"], 1), 3), "f32",
                 {"workload": "serving_poisson_20hz_400req", "rate_per_s": 20.0, "requests": len(reqs),
                  "volumes": ["8^4", "16^4", "16^3x32", "24^3x48", "32^3x64"],
                  "reps": ["SU(2) fund", "SU(2) adj", "SU(3) fund", "SU(4) asym"], "kappa": [0.12, 0.135],
                  "rhs_per_request": [1, 12], "slots_per_session": 12, "inner": "f32", "tol": 1e-10}, None,
                 latency_ms={"p50": round(lat["p50"] * 1e3, 1), "p99": round(lat["p99"] * 1e3, 1),
                             "max": round(lat["max"] * 1e3, 1)},
                 service_ms={k: round(v * 1e3, 1) for k, v in rep["service_s"].items()},
                 report={k: v for k, v in rep.items() if k not in ("latency_s", "service_s")},
                 rate_sweep=sweep, highest_rate_with_bounded_p99=bounded)


FOUR_REPS = [(3, "fund", (32, 32, 32, 32)), (2, "adj", (48, 24, 24, 24)), (4, "asym", (48, 24, 24, 24)),
             (3, "sym", (32, 32, 32, 32))]


def four_rep_table(torch, hrw, dev, kappa, theta, copy_gbs):
    """D_W and D_hat single applies in FP64 and FP32 for the four representations at the
    sizes of the solve workloads, with stored U_R (and, for SU(3) fund, two-row links),
    on near-thermal links generated on the device."""
    from paper_2405_19294_amd import serve
    table = {}
    for nc, rep, dims in FOUR_REPS:
        uf = serve.near_thermal_links(torch, dev, dims, nc, eps=0.3, seed=2)
        key = f"SU({nc}) {rep} {'x'.join(str(d) for d in dims[::-1])}"
        table[key] = operator_table(torch, hrw, dev, dims, nc, rep, uf, kappa, theta, copy_gbs)
        if rep == "fund":
            table[key + " two-row"] = operator_table(torch, hrw, dev, dims, nc, rep, uf, kappa, theta, copy_gbs,
                                                     two_rows=True)
        del uf
        torch.cuda.empty_cache()
    return table


def workload_ops(args):
    """Single D_W and D_hat applies in FP64 and FP32 for the four representations at the sizes of
    the solve workloads (SU(3) fund and sym 32^4, SU(2) adj and SU(4) asym 24^3x48)."""
    import torch

    import fixtures as fx
    from paper_2405_19294_amd import hrw
    hrw.load()
    dev = torch.device("cuda:0")
    theta, kappa = (np.pi, 0.0, 0.0, 0.0), 0.135
    copy = copy_reference(torch, dev)
    table, fused_table, two_row_table, worst = {}, {}, {}, None
    for nc, rep, dims in [(3, "fund", (32, 32, 32, 32)), (2, "adj", (48, 24, 24, 24)),
                          (4, "asym", (48, 24, 24, 24)), (3, "sym", (32, 32, 32, 32))]:
        uf = torch.from_numpy(fx.gauge_field(dims, nc, "thermal", seed=2, eps=0.3)).to(dev)
        rows = operator_table(torch, hrw, dev, dims, nc, rep, uf, kappa, theta, copy["gbs"])
        key = f"SU({nc}) {rep} {'x'.join(str(d) for d in dims[::-1])}"
        table[key] = rows
        if rep != "fund":
            # the same applies with the representation map fused into the hop
            fr = operator_table(torch, hrw, dev, dims, nc, rep, uf, kappa, theta, copy["gbs"], fused=True)
            for name, r in fr.items():
                r["speedup_vs_stored_links"] = round(rows[name]["hop_us"] / r["hop_us"], 3)
            fused_table[key] = fr
        else:
            # SU(3) fundamental links read as two rows (third rebuilt in the hop)
            tr = operator_table(torch, hrw, dev, dims, nc, rep, uf, kappa, theta, copy["gbs"], two_rows=True)
            for name, r in tr.items():
                r["speedup_vs_stored_links"] = round(rows[name]["hop_us"] / r["hop_us"], 3)
            two_row_table[key] = tr
        del uf
        torch.cuda.empty_cache()
        for name in ("deo_f64", "deo_f32"):
            if worst is None or rows[name]["frac_of_peak"] < worst[1]:
                worst = (f"{key} {name}", rows[name]["frac_of_peak"])
    fracs = [r["frac_of_peak"] for t in table.values() for n, r in t.items() if n.startswith("deo")]
    best = max(((k, n, r) for k, t in table.items() for n, r in t.items() if n.startswith("deo")),
               key=lambda v: v[2]["frac_of_peak"])
    roof = {"bound": "hbm", "kernel": f"D_hat apply (two e/o hops), {best[0]} {best[1]}",
            "achieved": best[2]["GBs_min"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": best[2]["frac_of_peak"], "traffic": None}
    return _line(round(sum(fracs) / len(fracs), 4), "mean fraction of 8 TB/s (D_hat, FP64 and FP32, 4 reps)", 20, 3,
                 None, "f64+f32", {"workload": "operator_sweep_4_reps", "kappa": kappa, "theta": "(pi,0,0,0)"}, roof,
                 operators=table, operators_fused_rep_map=fused_table, operators_two_row_links=two_row_table,
                 lowest=worst, hbm_copy_reference=copy)


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
    """The CPU oracle (as it stands, built -O3 -march=native on this host) on a bounded
    sample of the same solve, on all the host threads this process may use and on one.

    Times the b' and eta preparation and a few iterations of the oracle's FP64 CG on the
    same even/odd system with every thread, and extrapolates to the iteration count of
    the full solve.  The one-core figure scales that by the ratio of one D_hat apply
    timed on one thread to the same apply on all of them (a CG iteration is two D_hat
    applies plus site-wise vector work).
    """
    import tempfile

    import oracle as orc

    orc.load_native(tempfile.mkdtemp(prefix="oracle_native_"))
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", threads))
    orc.set_num_threads(threads)
    ur = orc.rep_map(3, "fund", uf)
    be, bo = orc.split_eo(dims, b)
    t0 = time.perf_counter()
    bpe = be + kappa * orc.hop_eo(dims, ur, bo, 0, theta)
    eta = orc.deo(dims, ur, kappa, bpe, theta, dagger=True)
    t_prep = time.perf_counter() - t0
    t1 = time.perf_counter()
    orc.deo(dims, ur, kappa, be, theta)
    t_apply = time.perf_counter() - t1
    n = cpu_iters or int(max(1, min(20, 10.0 / max(2 * t_apply, 1e-3))))
    t1 = time.perf_counter()
    orc.cg(dims, ur, kappa, eta, theta, orc.SYSTEM_EO, tol=1e-10, max_iter=n)
    t_cg = time.perf_counter() - t1
    per_iter = t_cg / n
    est_solve = t_prep + per_iter * gpu_iters
    orc.set_num_threads(1)
    t1 = time.perf_counter()
    orc.deo(dims, ur, kappa, be, theta)
    t_apply1 = time.perf_counter() - t1
    orc.set_num_threads(threads)
    scale = t_apply1 / t_apply
    log(f"cpu oracle (-O3 -march=native): {n} CG iterations in {t_cg:.1f}s on {threads} threads, "
        f"D_hat {t_apply:.2f}s ({threads} threads) / {t_apply1:.2f}s (1 thread) ({cpu_model()})")
    return {
        "value": round(1.0 / est_solve, 6),
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "build": "gcc -O3 -march=native -fopenmp",
        "sample": (f"{n} iterations of the oracle's FP64 CG on the same 32^4 even/odd system "
                   f"({per_iter:.2f} s/iteration incl. the final true-residual check) plus the "
                   f"b' and eta preparation ({t_prep:.2f} s), extrapolated to the GPU solve's "
                   f"{gpu_iters} iterations; {threads} threads; host CPU: {cpu_model()}"),
        "one_core": {
            "value": round(1.0 / (est_solve * scale), 6), "unit": "solves/s", "cores": 1,
            "sample": (f"the all-thread estimate scaled by one D_hat apply on 1 thread ({t_apply1:.2f} s) "
                       f"over the same apply on {threads} threads ({t_apply:.2f} s)")},
    }


if __name__ == "__main__":
    main()
