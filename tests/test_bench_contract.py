"""bench.py contract checks that need no GPU, and the counter summariser."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def _write_counters(path, name, rows):
    with open(path, "w") as f:
        f.write('"Kernel_Name","Counter_Name","Counter_Value"\n')
        for kernel, value in rows:
            f.write(f'"{kernel}","{name}",{value}\n')


def test_profsum_calibrates_on_the_copy_and_checks_the_source_hash(tmp_path):
    from paper_2405_19294_amd import profsum
    gib_kib = (1 << 30) / 1024
    hop = "void hrw::hop_kernel<3, 3, double, false, 0>(hrw::HopArgs<double>)"
    _write_counters(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", gib_kib / 2), (hop, 1000.0)])
    _write_counters(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", gib_kib), (hop, 100.0)])
    rec = profsum.summarize(None, str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "t"), "cmd")
    assert abs(rec["fetch_factor"] - 2.0) < 1e-12 and abs(rec["write_factor"] - 1.0) < 1e-12
    assert abs(rec["kernels"][0]["traffic_bytes"] - (2000.0 + 100.0) * 1024) < 1e-6
    assert profsum.traffic_for("hop_kernel<3, 3, double, false, 0>", str(tmp_path / "t.json")) == \
        rec["kernels"][0]["traffic_bytes"]
    data = json.load(open(tmp_path / "t.json"))
    data["source_hash"] = "stale"
    json.dump(data, open(tmp_path / "t.json", "w"))
    assert profsum.traffic_for("hop_kernel<3, 3, double, false, 0>", str(tmp_path / "t.json")) is None


def test_committed_traffic_record_names_the_dominant_instances():
    """The committed counter record holds the two-row FP64 hop instances under the names the
    bench looks up (the instance name carries the staging flag after the epilogue)."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "hop_traffic_su3_fund_32x4_f64.json")))
    names = [r["kernel"] for r in rec["kernels"]]
    for tag in ("false, 0,", "false, 1,", "true, 2,"):
        assert sum("hop_su3_kernel<double, " + tag in n for n in names) == 1, (tag, names)
