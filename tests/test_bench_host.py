"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the HBM
traffic taken from a committed profile only while the profiled kernel
source is unchanged, the algorithmic flop count of a solve, and the tau
error in scaled window coordinates."""

import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profiled_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k.md").write_text("- kernel_source_sha256_16: abcd\n- traffic_bytes: 123\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda sources=None: "abcd")
    assert bench.profiled_traffic("k.md") == 123       # the profile matches the source
    monkeypatch.setattr(bench, "kernel_source_sha", lambda sources=None: "0" * 16)
    assert bench.profiled_traffic("k.md") is None       # the kernel changed since the counters were taken
    assert bench.profiled_traffic("no_such_profile.md") is None


def test_every_registered_profile_names_its_source_and_traffic():
    """Each committed summary the bench lines read carries the kernel source
    hash it was taken on and the HBM bytes per launch, in the fields
    profiled_traffic parses."""
    for name in list(bench.PROFILES.values()) + ["k_rasl_rasl256x32x16x24.md"]:
        text = open(os.path.join(ROOT, "profiles", name)).read()
        fields = dict(line.strip().lstrip("- ").split(":", 1) for line in text.splitlines()
                      if line.strip().lstrip("- ").startswith(("kernel_source_sha256_16:", "traffic_bytes:")))
        assert len(fields["kernel_source_sha256_16"].strip()) == 16, name
        assert int(fields["traffic_bytes"]) > 0, name


def test_cold_jacobi_work_is_the_stated_model():
    """6 S m n^2 flops and 8 S m n^2 LDS bytes (n = min side), S summed
    over the patch's sweeps."""
    p = SimpleNamespace(m=30, n=50, model=8)
    res = {"counters": {"jacobi_sweeps": 7}}
    f, b = bench.cold_jacobi_work(res, p)
    assert f == 6 * 50 * 30 * 30 * 7 and b == 8 * 50 * 30 * 30 * 7


def test_solve_flops_counts_the_stated_terms():
    """2 nr per examined pair + 6 nr per rotation + 4 nc nr per kept row +
    (20 + 8 p') nc nr per inner iteration; warm adds 2 nc^2 nr per
    iteration and 6 nc per rotation."""
    p = SimpleNamespace(m=30, n=50, model=8)
    res = {"counters": {"jacobi_pairs": 1000, "jacobi_rotations": 400, "recon_rows": 70, "inner_iters": 3}}
    nr, nc, pp = 50, 30, 5
    cold = 2 * nr * 1000 + 6 * nr * 400 + 4 * nc * nr * 70 + (20 + 8 * pp) * nc * nr * 3
    assert bench.solve_flops(res, p) == cold
    assert bench.solve_flops(res, p, warm=True) == cold + 2 * nc * nc * nr * 3 + 6 * nc * 400


def test_tau_rel_err_in_scaled_coordinates():
    tau0 = np.array([[1.0, 0.0, 200.0], [0.0, 1.0, 150.0], [0.0, 0.0, 1.0]])
    assert bench.tau_rel_err(tau0, tau0, tau0, 100, 100) == 0.0
    H = tau0.copy()
    H[0, 2] += 0.5                                      # half a pixel shift: 0.5 / s in scaled units
    e = bench.tau_rel_err(H, tau0, tau0, 100, 100)
    assert abs(e - (0.5 / 50.0) / np.sqrt(3.0)) < 1e-12
