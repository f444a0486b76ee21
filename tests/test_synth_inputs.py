"""The seeded input generators (tilt_synth): every workload can be drawn in
full, and the texture frequencies follow the stated recipe."""

import numpy as np
import pytest

import tilt_synth as ts
from tilt_synth import textures as tx


@pytest.mark.parametrize("r,L", [(8, 32), (7, 32), (8, 40), (6, 33), (1, 32), (5, 100)])
def test_texture_frequencies_are_separated_and_in_range(r, L):
    """r frequencies in [1, max(1 + 0.5 r + 0.5, L / 8)] cycles, pairwise at
    least 0.5 apart, also where r of them barely fit (rank 8 on 32 px)."""
    hi = max(1.0 + 0.5 * r + 0.5, L / 8.0)
    for seed in range(20):
        f = tx._freqs(np.random.default_rng(seed), r, L)
        assert f.shape == (r,)
        assert np.all(f >= 1.0) and np.all(f <= hi)
        if r > 1:
            assert np.min(np.diff(np.sort(f))) >= 0.5 - 1e-12


def test_tight_frequencies_fill_their_range():
    """The direct draw for tight cases is the uniform law on separated
    configurations: the smallest frequency spreads over the free span."""
    r, L = 8, 32
    lows = np.array([np.min(tx._freqs(np.random.default_rng(s), r, L)) for s in range(400)])
    span = (1.0 + 0.5 * r + 0.5 - 1.0) - 0.5 * (r - 1)
    # min of r uniforms on [0, span]: mean span / (r + 1)
    assert abs(np.mean(lows - 1.0) - span / (r + 1)) < 0.02


def test_uneven_workload_small_high_rank_windows_draw():
    """Indices of the uneven workload whose small windows have rank 7-8 (the
    rejection sampler alone could not draw them) are generated."""
    found = 0
    for i in range(200):
        rng = tx.patch_rng(2, i)
        m, n, r = int(rng.integers(32, 257)), int(rng.integers(32, 257)), int(rng.integers(1, 9))
        if r >= 7 and min(m, n) <= 48:
            p = ts.make_batch(2, [i])[0]
            assert p.image.shape == (2 * max(m, n), 2 * max(m, n)) and (p.m, p.n) == (m, n)
            assert np.all(np.isfinite(p.image))
            found += 1
    assert found >= 1
