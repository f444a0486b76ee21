"""Gangs: several workgroups of the fused kernel share one window whose SVT
is tiled through device memory (the super-block pairs of each Jacobi round
are split over them, with a barrier between rounds).  The pairs of a round
touch disjoint rows, so which workgroup takes which pair cannot change the
arithmetic: a batch solved with gangs must equal, bit for bit, the same
batch solved with one workgroup per window and the plain path, and it must
match the oracle as the one-workgroup path does.
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


def _same(a, b):
    return (np.array_equal(a["tau"], b["tau"]) and np.array_equal(a["A"], b["A"]) and
            np.array_equal(a["E"], b["E"]) and a["inner_iters_total"] == b["inner_iters_total"] and
            a["counters"] == b["counters"])


def _solve(tilt, ctx, ps, device, tp, gang_max):
    old = os.environ.get("TILT_GANG_MAX")
    os.environ["TILT_GANG_MAX"] = str(gang_max)
    try:
        print(f"gang_max={gang_max}: {len(ps)} windows", flush=True)
        return solve_on_device(tilt, ctx, ps, device, tp)
    finally:
        if old is None:
            del os.environ["TILT_GANG_MAX"]
        else:
            os.environ["TILT_GANG_MAX"] = old


@pytest.mark.parametrize("gang_max", [2, 4, 8])
def test_gangs_equal_one_workgroup_bitwise(tilt, ctx, device, gang_max):
    ps = ts.make_batch(2, TILED + RESIDENT)
    tp = tilt.default_params(fixed_iters=1, max_outer=2, max_inner=3, svt_mode=1)
    _, one = _solve(tilt, ctx, ps, device, tp, 1)
    _, many = _solve(tilt, ctx, ps, device, tp, gang_max)
    for k, (a, b) in enumerate(zip(one, many)):
        assert a["status"] == 0 and b["status"] == 0, k
        assert _same(a, b), k


def test_gangs_equal_plain_path_bitwise(tilt, ctx, device):
    ps = ts.make_batch(2, TILED[:2])
    tp = tilt.default_params(fixed_iters=1, max_outer=1, max_inner=3)
    _, fused = _solve(tilt, ctx, ps, device, tp, 4)
    _, plain = solve_on_device(tilt, ctx, ps, device, tp, plain=True)
    for k, (a, b) in enumerate(zip(fused, plain)):
        assert _same(a, b), k


def test_many_concurrent_gangs(tilt, ctx, device):
    """Forty tiled windows (gangs of up to four, over a hundred workgroups
    at once) and twenty-five that fit LDS in one launch: every window
    equals its solve with one workgroup per window."""
    shapes = ts.make_config(2, count=300)
    tiled = [i for i, p in enumerate(shapes) if min(p.m, p.n) * ((max(p.m, p.n) + 3) // 4 * 4) > 40000][:40]
    small = [i for i, p in enumerate(shapes) if max(p.m, p.n) <= 100][:25]
    assert len(tiled) == 40 and len(small) == 25
    ps = [shapes[i] for i in tiled + small]
    tp = tilt.default_params(fixed_iters=1, max_outer=1, max_inner=2)
    _, one = _solve(tilt, ctx, ps, device, tp, 1)
    _, many = _solve(tilt, ctx, ps, device, tp, 4)
    for k, (a, b) in enumerate(zip(one, many)):
        assert a["status"] == 0, k
        assert _same(a, b), k


def test_gang_fixed_iterations_match_oracle(tilt, ctx, device):
    """A 256x227 window solved by a gang of four for a fixed number of
    iterations against the FP64 oracle (the tolerances of the
    fixed-iteration parity tests)."""
    p = ts.make_batch(2, [30])[0]
    tp = tilt.default_params(fixed_iters=1, max_outer=1, max_inner=6, lam=p.lam)
    _, res = _solve(tilt, ctx, [p], device, tp, 4)
    r = res[0]
    assert r["status"] == 0, r
    ref = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, oracle_params(O, tp), lam=p.lam)
    assert np.linalg.norm(r["A"] - ref.A) <= 1e-4 * np.linalg.norm(ref.A)
    assert np.linalg.norm(r["E"] - ref.E) <= 1e-3 * max(np.linalg.norm(ref.E), 1e-12)
    assert O.tau_rel_err(r["tau"], ref.tau_px, p.m, p.n) <= 1e-5
