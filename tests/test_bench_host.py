"""Host logic of bench.py (no GPU): the one-GPU refusal, the code digest that
gates the stored counter readings, the launch-shape mapping the roofline
uses, and the algorithmic work per window."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_code_digest_ignores_comments_and_layout(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) {  // twice\n  return 2 * x;\n}\n")
    b.write_text("/* doubles x */\nint f(int x) {\n\n    return 2 * x;   \n}\n// end\n")
    c.write_text("int f(int x) {\n  return 3 * x;\n}\n")
    assert bench.code_digest(str(a)) == bench.code_digest(str(b))
    assert bench.code_digest(str(a)) != bench.code_digest(str(c))


def test_counter_readings_are_reported_only_for_the_code_they_measured(monkeypatch):
    # the stored PMC readings are reported while the projector code is the
    # code they were taken on, and never for another code or instance
    t = dict(bench.PMC_TRAFFIC)
    current = bench.code_digest(os.path.join(ROOT, t["source"]))
    monkeypatch.setattr(bench, "PMC_TRAFFIC", dict(t, sha256=current))
    b4 = bench.pmc_traffic("cg_forward/4")
    assert b4 == (t["kib"]["cg_forward/4"][0] * 2.0 + t["kib"]["cg_forward/4"][1]) * 1024.0
    assert bench.pmc_traffic("cg_forward/5") is None
    monkeypatch.setattr(bench, "PMC_TRAFFIC", dict(t, sha256="0" * 64))
    assert bench.pmc_traffic("cg_forward/4") is None

    # the VALU instruction counts follow the same rule, and their issue
    # fraction is the count over the launch time against 1228.8 G/s
    monkeypatch.setattr(bench, "PMC_TRAFFIC", dict(t, sha256=current))
    monkeypatch.setattr(bench, "PMC_VALU", dict(bench.PMC_VALU, sha256=current))
    n = bench.PMC_VALU["insts"]["cg_forward/8"]
    v = bench.pmc_valu("cg_forward/8", 40e-6)
    assert v["insts_per_launch"] == n
    assert abs(v["frac"] - n / 40e-6 / 1228.8e9) < 1e-12
    assert bench.pmc_valu("cg_forward/6", 40e-6) is None
    monkeypatch.setattr(bench, "PMC_VALU", dict(bench.PMC_VALU, sha256="0" * 64))
    assert bench.pmc_valu("cg_forward/8", 40e-6) is None


def test_rays_per_lane_follows_the_launch_plan():
    # cap 0 means the maximum (8); the count is what the larger orientation
    # group needs at 512 lanes per workgroup, rounded up to an instantiated value
    assert bench.fwd_rays_per_lane(4, 44 * 1449) == 4
    assert bench.fwd_rays_per_lane(0, 44 * 1449) == 8
    assert bench.fwd_rays_per_lane(8, 600) == 2
    assert bench.fwd_rays_per_lane(8, 7 * 512) == 8
    assert bench.fwd_rays_per_lane(6, 100) == 1


def test_window_nnz_matches_the_oracle_matrix():
    # the roofline's algorithmic flops count 2 d N^2 non-zero weights per
    # angle; the oracle's CSR rows of the same angles hold that many to
    # 0.5% (it agrees to 2e-4: only border pixels differ)
    from oracle import system
    N, na = 64, 90
    P = system.Projector(N, na)
    ids = [0, 11, 22, 45, 67]
    th = np.array(ids) * np.pi / na
    nnz = P.rows(ids).nnz
    assert abs(bench.window_nnz(N, th) - nnz) <= 0.005 * nnz
