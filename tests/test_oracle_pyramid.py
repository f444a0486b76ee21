"""Pins of the oracle's coarse-to-fine pyramid (CPU): the blur taps and the
even-pixel alignment from impulse responses, exactness on constant and
bilinear images, clamped borders, level shapes, the conjugation between
levels, and recovery of a deformation through three levels."""

import numpy as np
import pytest

import oracle as O
import tilt_synth as ts

P = O.pyramid


def test_constant_image_is_preserved():
    for H, W in [(7, 9), (8, 8), (2, 3)]:
        img = np.full((H, W), 0.37)
        out = P.blur_decimate(img)
        assert out.shape == ((H + 1) // 2, (W + 1) // 2)
        assert np.allclose(out, 0.37, rtol=0, atol=1e-15)


def test_impulse_responses_fix_taps_and_alignment():
    img = np.zeros((21, 23))
    img[10, 12] = 1.0                    # even row, even column: coarse (5, 6)
    out = P.blur_decimate(img)
    expect = np.zeros_like(out)
    expect[5, 6] = 36 / 256
    expect[4, 6] = expect[6, 6] = 6 / 256
    expect[5, 5] = expect[5, 7] = 6 / 256
    expect[4, 5] = expect[4, 7] = expect[6, 5] = expect[6, 7] = 1 / 256
    np.testing.assert_allclose(out, expect, rtol=0, atol=1e-16)
    img = np.zeros((21, 23))
    img[11, 12] = 1.0                    # odd row: shared by coarse rows 5 and 6 (taps 4/16)
    out = P.blur_decimate(img)
    assert abs(out[5, 6] - 24 / 256) < 1e-16 and abs(out[6, 6] - 24 / 256) < 1e-16
    assert abs(out[5, 5] - 4 / 256) < 1e-16 and abs(out[6, 7] - 4 / 256) < 1e-16
    # every second tap survives per axis: (1 + 6 + 1)/16 = (4 + 4)/16 = 1/2
    assert abs(out.sum() - 0.25) < 1e-15


def test_bilinear_images_are_sampled_exactly_in_the_interior():
    rng = np.random.default_rng(3)
    a, b, c, d = rng.standard_normal(4)
    H, W = 30, 34
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = a + b * x + c * y + d * x * y
    out = P.blur_decimate(img)
    yi, xi = np.mgrid[1:out.shape[0] - 1, 1:out.shape[1] - 1]
    want = a + b * (2 * xi) + c * (2 * yi) + d * (2 * xi) * (2 * yi)
    np.testing.assert_allclose(out[1:-1, 1:-1], want, rtol=0, atol=1e-12)


def test_borders_are_clamped():
    H, W = 6, 9
    img = np.tile(np.arange(W, dtype=np.float64) + 1.0, (H, 1))   # f(x) = x + 1
    out = P.blur_decimate(img)
    # column 0: taps at x = -2, -1 clamp to x = 0
    assert abs(out[2, 0] - (11 * 1 + 4 * 2 + 1 * 3) / 16) < 1e-15
    # last column of a width-9 image is pixel 8: taps 9, 10 clamp to 8
    assert abs(out[2, -1] - (1 * 7 + 4 * 8 + 11 * 9) / 16) < 1e-15


def test_level_shapes():
    assert P.level_shape(40, 37, 0) == (40, 37)
    assert P.level_shape(40, 37, 1) == (20, 19)
    assert P.level_shape(40, 37, 2) == (10, 10)
    assert [im.shape for im in P.build_pyramid(np.zeros((480, 640)), 3)] == [(480, 640), (240, 320), (120, 160)]
    assert [im.shape for im in P.build_pyramid(np.zeros((7, 5)), 3)] == [(7, 5), (4, 3), (2, 2)]


def test_conjugation_between_levels():
    rng = np.random.default_rng(5)
    H = np.array([[1.1, 0.2, 310.0], [-0.1, 0.9, 230.0], [2e-4, -1e-4, 1.0]])
    Hc = P.to_coarser(H)
    for _ in range(5):
        u = rng.uniform(-50, 50, 2)
        fine = H @ np.array([u[0], u[1], 1.0])
        coarse = Hc @ np.array([u[0] / 2, u[1] / 2, 1.0])
        np.testing.assert_allclose(coarse[:2] / coarse[2], fine[:2] / fine[2] / 2, rtol=1e-13)
    np.testing.assert_allclose(P.to_finer(Hc), H / H[2, 2], rtol=1e-14)
    A = np.array([[1.0, 0.3, 10.0], [0.0, 1.2, 5.0], [0.0, 0.0, 1.0]])
    assert np.allclose(P.to_coarser(A)[2], [0, 0, 1])


def test_pyramid_solve_recovers_deformation():
    """Three levels (64 -> 32 -> 16 samples per side) undo a 12 degree
    rotation with skew; the level-0 result is an axis-aligned scaling of the
    ground truth, like the single-level recovery pin."""
    rng = ts.patch_rng(79, 1)
    p = ts.make_patch(rng, m=64, n=64, height=192, width=192, rank=2, model=6, corruption=0.03,
                      theta_deg=12, skew=0.1)
    res, levels = P.tilt_solve_pyramid(p.image, p.tau0, p.m, p.n, p.model, O.Params(max_outer=30), levels=3)
    assert len(levels) == 3 and [r.A.shape for r in levels] == [(16, 16), (32, 32), (64, 64)]
    Mx = np.linalg.inv(p.meta["G_norm"]) @ res.tau_norm
    Mx = Mx / Mx[2, 2]
    off = max(abs(Mx[0, 1]), abs(Mx[1, 0])) / max(abs(Mx[0, 0]), abs(Mx[1, 1]))
    assert off < 2e-2, Mx
    M0 = np.linalg.inv(p.meta["G_norm"])
    assert max(abs(M0[0, 1]), abs(M0[1, 0])) > 0.05
