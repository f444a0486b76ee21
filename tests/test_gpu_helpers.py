"""Help for windows beyond LDS in the fused kernel: once the work queue is
empty, idle workgroups claim super-block pairs of the rounds that leaders
of tiled windows publish.  The pairs of a round touch disjoint rows, so
which workgroup takes which pair cannot change the arithmetic: a batch
solved with helpers must equal, bit for bit, the same batch solved with
one workgroup per window and the plain path, and it must match the oracle
as the one-workgroup path does.
"""

import os

import numpy as np
import pytest

import oracle as O
import tilt_synth as ts
from gpu_util import oracle_params, solve_on_device

pytestmark = pytest.mark.gpu

# Windows of the uneven workload: tiled ones (256x227 and 235x195: 8
# super-blocks, 4 pairs per round; 227x190: 6; 125x251: 4) and windows
# that fit LDS (warm-started where the rotation fits too).
TILED = [30, 7, 3, 67]
RESIDENT = [0, 1, 2, 4]


def _diff(a, b):
    """Names of the result fields in which a and b differ (empty: bitwise equal)."""
    out = [k for k in ("tau", "A", "E") if not np.array_equal(a[k], b[k])]
    if a["inner_iters_total"] != b["inner_iters_total"]:
        out.append("inner_iters_total")
    out += [f"counters.{k}={a['counters'][k]}/{b['counters'][k]}" for k in a["counters"]
            if a["counters"][k] != b["counters"][k]]
    return out


def _solve(tilt, ctx, ps, device, tp, helpers):
    old = os.environ.get("TILT_HELPERS")
    os.environ["TILT_HELPERS"] = "1" if helpers else "0"
    try:
        print(f"helpers={helpers}: {len(ps)} windows", flush=True)
        return solve_on_device(tilt, ctx, ps, device, tp)
    finally:
        if old is None:
            del os.environ["TILT_HELPERS"]
        else:
            os.environ["TILT_HELPERS"] = old


@pytest.mark.parametrize("svt_mode", [0, 1])
def test_helpers_equal_one_workgroup_bitwise(tilt, ctx, device, svt_mode):
    ps = ts.make_batch(2, TILED + RESIDENT)
    tp = tilt.default_params(fixed_iters=1, max_outer=2, max_inner=3, svt_mode=svt_mode)
    _, one = _solve(tilt, ctx, ps, device, tp, False)
    _, many = _solve(tilt, ctx, ps, device, tp, True)
    for k, (a, b) in enumerate(zip(one, many)):
        assert a["status"] == 0 and b["status"] == 0, k
        assert not _diff(a, b), (k, _diff(a, b))


@pytest.mark.parametrize("svt_mode", [0, 1])
def test_helpers_equal_plain_path_bitwise(tilt, ctx, device, svt_mode):
    ps = ts.make_batch(2, TILED[:2])
    tp = tilt.default_params(fixed_iters=1, max_outer=1, max_inner=3, svt_mode=svt_mode)
    _, fused = _solve(tilt, ctx, ps, device, tp, True)
    _, plain = solve_on_device(tilt, ctx, ps, device, tp, plain=True)
    for k, (a, b) in enumerate(zip(fused, plain)):
        assert not _diff(a, b), (k, _diff(a, b))


def test_many_tiled_windows_with_helpers(tilt, ctx, device):
    """Forty tiled windows and twenty-five that fit LDS in one launch, the
    small ones finishing first so that their workgroups help the tiled
    ones: every window equals its solve with one workgroup per window."""
    shapes = ts.make_config(2, count=300)
    tiled = [i for i, p in enumerate(shapes) if min(p.m, p.n) * ((max(p.m, p.n) + 3) // 4 * 4) > 40000][:40]
    small = [i for i, p in enumerate(shapes) if max(p.m, p.n) <= 100][:25]
    assert len(tiled) == 40 and len(small) == 25
    ps = [shapes[i] for i in tiled + small]
    tp = tilt.default_params(fixed_iters=1, max_outer=1, max_inner=2, svt_mode=1)
    _, one = _solve(tilt, ctx, ps, device, tp, False)
    _, many = _solve(tilt, ctx, ps, device, tp, True)
    for k, (a, b) in enumerate(zip(one, many)):
        assert a["status"] == 0, k
        assert not _diff(a, b), (k, _diff(a, b))


@pytest.mark.parametrize("svt_mode", [0, 1])
def test_helped_tiled_window_matches_oracle(tilt, ctx, device, svt_mode):
    """A 256x227 window solved with helpers for a fixed number of
    iterations against the FP64 oracle (the tolerances of the
    fixed-iteration parity tests), with the cold tiled Jacobi and with the
    tiled Jacobi warm-started from the staged rotation rows (which crosses
    a Newton-Schulz re-orthonormalisation at the fifth SVT)."""
    p = ts.make_batch(2, [30])[0]
    tp = tilt.default_params(fixed_iters=1, max_outer=1, max_inner=8, lam=p.lam, svt_mode=svt_mode)
    _, res = _solve(tilt, ctx, [p], device, tp, True)
    r = res[0]
    assert r["status"] == 0, r
    ref = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, oracle_params(O, tp), lam=p.lam)
    assert np.linalg.norm(r["A"] - ref.A) <= 1e-4 * np.linalg.norm(ref.A)
    assert np.linalg.norm(r["E"] - ref.E) <= 1e-3 * max(np.linalg.norm(ref.E), 1e-12)
    assert O.tau_rel_err(r["tau"], ref.tau_px, p.m, p.n) <= 1e-5


def test_full_uneven_batch_one_launch_against_oracle(tilt, ctx, device):
    """All 1024 windows of the uneven warm-started workload in one fused
    launch (svt_mode 1, idle workgroups helping the tiled windows), for a
    fixed 2 outer x 15 inner iterations so that the oracle can follow:
    every window returns TILT_OK, and sampled windows -- the two largest
    tiled ones, one each of the other SVT kinds (in LDS cold, in LDS warm)
    and the smallest -- match the FP64 oracle (fixed-count tolerances: A
    within 1e-4, tau within 1e-5)."""
    patches = ts.make_config(2)
    assert len(patches) == 1024
    tp = tilt.default_params(svt_mode=1, fixed_iters=1, max_outer=2, max_inner=15)
    _, res = solve_on_device(tilt, ctx, patches, device, tp)
    assert all(r["status"] == 0 for r in res)

    def cells(p):
        return min(p.m, p.n) * ((max(p.m, p.n) + 3) // 4 * 4)

    order = sorted(range(1024), key=lambda i: -cells(patches[i]))
    tiled = order[:2]
    mid = next(i for i in order if 20000 < cells(patches[i]) < 30000)       # in LDS, cold (rotation does not fit)
    warm = next(i for i in order if 8000 < cells(patches[i]) < 12000)       # in LDS, warm
    small = order[-1]
    for i in tiled + [mid, warm, small]:
        p, r = patches[i], res[i]
        ref = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, oracle_params(O, tp), lam=p.lam)
        err_a = np.linalg.norm(r["A"] - ref.A) / np.linalg.norm(ref.A)
        err_t = O.tau_rel_err(r["tau"], ref.tau_px, p.m, p.n)
        print(f"window {i} ({p.m}x{p.n}): A {err_a:.1e} tau {err_t:.1e}", flush=True)
        assert err_a <= 1e-4 and err_t <= 1e-5, (i, err_a, err_t)

