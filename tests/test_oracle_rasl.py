"""Pins of the RASL oracle (oracle/rasl.py) against what the mathematics
fixes: the block-diagonal projection equals the dense projector onto the
complement of a block-diagonal Jacobian; column k of the data matrix
depends on tau_k alone, with the Jacobian the finite differences give; the
inner loop's fixed point is a dual certificate of the constrained problem;
identical images are already aligned (the optimum is A = D, E = 0, so every
Delta tau is zero); planted misalignments are undone."""

import math

import numpy as np
import pytest

import oracle as O
import tilt_synth as ts

R = O.rasl


def _block_jacobians(rng, L, N, p):
    return [rng.standard_normal((L, p)) for _ in range(N)]


def test_column_annihilator_matches_dense_projector():
    rng = np.random.default_rng(31)
    L, N, p = 30, 5, 3
    Js = _block_jacobians(rng, L, N, p)
    P = R.ColumnAnnihilator(Js)
    # dense block-diagonal Jacobian acting on vec(V) (columns stacked)
    Jb = np.zeros((L * N, p * N))
    for k, J in enumerate(Js):
        Jb[k * L:(k + 1) * L, k * p:(k + 1) * p] = J
    Pd = np.eye(L * N) - Jb @ np.linalg.pinv(Jb)
    V = rng.standard_normal((L, N))
    W = rng.standard_normal((L, N))
    got = P(V)
    want = (Pd @ V.reshape(-1, order="F")).reshape((L, N), order="F")
    np.testing.assert_allclose(got, want, atol=1e-12)
    np.testing.assert_allclose(P(got), got, atol=1e-12)                  # idempotent
    assert abs(np.sum(P(V) * W) - np.sum(V * P(W))) < 1e-11               # self-adjoint
    for k, J in enumerate(Js):
        assert np.linalg.norm(J.T @ got[:, k]) < 1e-11                    # J_k^T (P V)_k = 0
        Vk = np.zeros((L, N))
        Vk[:, k] = J @ rng.standard_normal(p)
        assert np.linalg.norm(P(Vk)) < 1e-11                              # range(J_k) in column k is removed


def _smooth_image(rng, H, W):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.zeros((H, W))
    for _ in range(4):
        fx, fy = rng.uniform(0.05, 0.3, 2)
        ph = rng.uniform(0, 2 * math.pi)
        img += np.cos(fx * xs + fy * ys + ph)
    return img - img.min() + 0.5


@pytest.mark.parametrize("model", [O.AFFINE, O.PROJECTIVE])
def test_rasl_jacobian_is_block_diagonal_and_matches_finite_differences(model):
    rng = np.random.default_rng(32 + model)
    N, m, n, H, W = 3, 7, 5, 32, 32
    images = [_smooth_image(rng, H, W) for _ in range(N)]
    tau0 = []
    for _ in range(N):
        th = rng.uniform(-0.3, 0.3)
        Hp = np.array([[1.1 * math.cos(th), -math.sin(th), 15.3 + rng.uniform(-1, 1)],
                       [math.sin(th), 0.9 * math.cos(th), 14.7 + rng.uniform(-1, 1)],
                       [0.0, 0.0, 1.0]])
        if model == O.PROJECTIVE:
            Hp[2, :2] = rng.uniform(-2e-3, 2e-3, 2)
        tau0.append(Hp)
    frames = R.frames_from_px(tau0, m, n, model)
    D, Js = R.rasl_step1(images, frames, m, n, model)
    assert D.shape == (m * n, N)
    np.testing.assert_allclose(np.linalg.norm(D, axis=0), 1.0, rtol=1e-13)
    h = 1e-6
    for k in range(N):
        for j in range(model):
            cols = []
            for sgn in (1.0, -1.0):
                fr = [R.ImageFrame(f.tau.copy(), f.c, f.s) for f in frames]
                fr[k].tau[j] += sgn * h
                cols.append(R.rasl_step1(images, fr, m, n, model)[0])
            fd = (cols[0] - cols[1]) / (2 * h)
            # column k moves as J_k predicts, every other column not at all
            np.testing.assert_allclose(fd[:, k], Js[k][:, j], rtol=1e-5, atol=1e-6 * np.abs(Js[k]).max())
            others = np.delete(fd, k, axis=1)
            assert np.max(np.abs(others)) == 0.0


def test_rasl_inner_loop_fixed_point_is_a_dual_certificate():
    rng = np.random.default_rng(33)
    L, N, p = 24, 6, 3
    D = rng.uniform(0, 1, (L, N))
    D[rng.uniform(size=(L, N)) < 0.1] = 2.5
    D /= np.linalg.norm(D, axis=0)
    Js = _block_jacobians(rng, L, N, p)
    lam = 1 / math.sqrt(max(L, N))
    P = R.ColumnAnnihilator(Js)
    Z0 = np.zeros_like(D)
    prm = O.Params(eps1=1e-9, eps2=1e-8, max_inner=200000, rho0=1.2)
    r = O.ladmap_inner(D, P, lam, D, Z0, Z0, prm)
    assert r.cond1 < 1e-7 and r.cond2 < 1e-7
    Z = -r.Y
    f = O.objective(r.A, r.E, lam)
    assert np.linalg.norm(Z, 2) <= 1 + 1e-6
    assert np.max(np.abs(Z)) <= lam * (1 + 1e-6)
    for k, J in enumerate(Js):
        assert np.linalg.norm(J.T @ Z[:, k]) <= 1e-6
    nuc = np.sum(np.linalg.svd(r.A, compute_uv=False))
    assert abs(np.sum(Z * r.A) - nuc) <= 1e-6 * f
    assert abs(np.sum(Z * r.E) - lam * np.sum(np.abs(r.E))) <= 1e-6 * f
    assert abs(f - np.sum(Z * D)) <= 1e-6 * f
    assert np.linalg.norm(P(r.A + r.E - D)) <= 1e-7 * np.linalg.norm(P(D))


def test_identical_images_are_a_fixed_point():
    """N identical clean images: the normalised data matrix is d 1^T, and
    with J_k^T d = 0 every feasible A has ||A||_* >= ||A 1/sqrt(N)|| >=
    sqrt(N) = ||D||_*, while E != 0 costs more than it can save when
    lambda > ||d||_inf / sqrt(N); so A = D, E = 0 and Delta tau = 0."""
    rng = np.random.default_rng(34)
    N, m, n = 8, 10, 12
    img = _smooth_image(rng, 30, 34)
    tau0 = [np.array([[1.0, 0.05, 16.2], [-0.04, 1.0, 14.9], [0.0, 0.0, 1.0]])] * N
    frames = R.frames_from_px(tau0, m, n, O.AFFINE)
    D, _ = R.rasl_step1([img] * N, frames, m, n, O.AFFINE)
    lam = 1 / math.sqrt(m * n)
    assert lam > np.abs(D[:, 0]).max() / math.sqrt(N)
    prm = O.Params(eps1=1e-10, eps2=1e-9, max_inner=20000, max_outer=3, eps_outer=0.0)
    res = R.rasl_solve([img] * N, tau0, m, n, O.AFFINE, prm, lam=lam)
    for H in res.tau_px:
        assert np.max(np.abs(H - tau0[0])) < 1e-7
    np.testing.assert_allclose(res.A, D, atol=1e-8)
    assert np.max(np.abs(res.E)) < 1e-8


def test_rasl_undoes_planted_misalignment():
    """Images of one texture moved by planted rotations, scales and shifts
    of up to 1.5 px: after the solve, G_k^{-1} tau_k is the same transform
    for every k (a common transform is not identifiable): the window corners
    agree to within 0.15 px, from an initial spread above 1 px (the rest is
    the corruption and the bilinear interpolation of 12 x 14 windows)."""
    r = ts.rasl_set(1, count=10, m=12, n=14, height=32, width=36)
    prm = O.Params(max_outer=12, fixed_iters=False)
    res = R.rasl_solve(r.images, r.tau0, r.m, r.n, r.model, prm, lam=r.lam)

    def spread(taus):
        Ms = [np.linalg.inv(r.G_px[k]) @ taus[k] for k in range(r.count)]
        M0 = np.mean(Ms, axis=0)
        # displacement of the window corners, in px
        a, b = (r.n - 1) / 2.0, (r.m - 1) / 2.0
        corners = np.array([[-a, -b, 1], [a, -b, 1], [a, b, 1], [-a, b, 1]]).T
        ref = M0 @ corners
        ref = ref[:2] / ref[2]
        worst = 0.0
        for M in Ms:
            c = M @ corners
            worst = max(worst, float(np.max(np.linalg.norm(c[:2] / c[2] - ref, axis=0))))
        return worst

    assert spread(r.tau0) > 1.0
    assert spread(res.tau_px) < 0.15
    assert res.status >= 0
