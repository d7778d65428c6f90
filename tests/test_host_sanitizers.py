"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every library source is compiled with the sanitizers on its host side only
(hipcc puts each -fsanitize= after -Xarch_host; the device code is the
ordinary gfx950 build) and linked into tests/sanitize/validate.cpp, which
calls every entry point with invalid arguments.  All of them must be
refused before any device work, so the program runs on a machine without a
GPU; a sanitizer finding aborts it.  LeakSanitizer is off: the HIP runtime
keeps allocations until exit."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1912_07962_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_validation_paths_are_clean_under_asan_and_ubsan(tmp_path):
    srcs = sorted(f for f in os.listdir(SRC) if f.endswith((".hip", ".cpp")))
    jobs = [[HIPCC, *FLAGS, *SAN, "-c", os.path.join(SRC, f), "-o", str(tmp_path / (f + ".o"))]
            for f in srcs]
    jobs.append([HIPCC, *FLAGS, *SAN, "-c", os.path.join(ROOT, "tests", "sanitize", "validate.cpp"),
                 "-o", str(tmp_path / "validate.o")])

    def run(cmd):
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(run, jobs))
    for cmd, r in zip(jobs, res):
        assert r.returncode == 0, (cmd[-3], r.stderr[-2000:])
    exe = tmp_path / "validate"
    link = [HIPCC, "--offload-arch=gfx950", *SAN, *[str(tmp_path / (f + ".o")) for f in srcs],
            str(tmp_path / "validate.o"), "-o", str(exe)]
    r = run(link)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
