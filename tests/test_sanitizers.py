"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (CPU only).

* The oracle (plain C) is compiled with both sanitizers together with a driver
  that calls every entry point on tiny lattices, argument errors included
  (``oracle/sanitize_driver.c``); leak detection is on.
* libhrw's host code (argument validation, size planning, the launch-shape
  cache parser) is compiled with both sanitizers on the host pass only
  (``-Xarch_host``; device code unoptimised, never run) and linked with a
  driver that
  calls the C ABI on paths that return before anything reaches a device, and
  feeds the cache parser well-formed, malformed and hostile files
  (``tests/sanitize_abi_driver.cpp``).

A sanitizer report or a failed check fails the test.
"""

import concurrent.futures
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _run(exe, args, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=900, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "orc_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", *SAN_FLAGS, "-o", exe,
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "sanitize_driver.c"),
                    "-lm"], check=True, capture_output=True, timeout=600)
    out = _run(exe, [], {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})
    assert "ok" in out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2405_19294_amd", "csrc")
    # nothing here reaches a device: the device code is built unoptimised, only to link
    hip = ["hipcc", "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g", "-std=c++17", "-Xclang",
           "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    for f in SAN_FLAGS:
        hip += ["-Xarch_host", f]
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    srcs.append(os.path.join(ROOT, "tests", "sanitize_abi_driver.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        r = subprocess.run(hip + lang + ["-c", src, "-o", obj], capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stdout + r.stderr
        return obj

    with concurrent.futures.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "abi_san")
    link = ["hipcc", "--offload-arch=gfx950"]
    for f in SAN_FLAGS:
        link += ["-Xarch_host", f]
    r = subprocess.run(link + ["-o", exe, *objs], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    # the HIP runtime is not instrumented: its allocations are not the subject here
    out = _run(exe, [str(tmp_path)], {"ASAN_OPTIONS": "detect_leaks=0", "HIP_VISIBLE_DEVICES": ""})
    assert "ok" in out
