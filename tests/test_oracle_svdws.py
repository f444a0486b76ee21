"""Pins of the oracle's SVD with warm start (Sec. 5, Alg. 2, Appendix A):
the closed-form f'(0) and f''(0) against finite differences of f(t) along
the Cayley curve, orthonormality of the curve, descent of the step, and the
pseudocontraction bound that guarantees the accuracy of the shrinkage."""

import numpy as np
import pytest

import oracle as O

W = O.svdws


def _previous(rng, m, n):
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    S = np.sort(rng.uniform(0.1, 2.0, n))[::-1]
    return U, S, V


@pytest.mark.parametrize("m,n,seed", [(7, 5, 0), (12, 12, 1), (20, 9, 2)])
def test_derivatives_match_finite_differences(m, n, seed):
    rng = np.random.default_rng(seed)
    U, S, V = _previous(rng, m, n)
    M = (U * S) @ V.T + 0.05 * rng.standard_normal((m, n))
    PU, PS, PV = W.projected_gradients(U, S, V, M)
    f1, f2 = W.derivatives(U, S, V, M, PU, PS, PV)
    h = 1e-4
    fp, f0, fm = (W.f_of_t(U, S, V, M, PU, PS, PV, t) for t in (h, 0.0, -h))
    fd1 = (fp - fm) / (2 * h)
    fd2 = (fp - 2 * f0 + fm) / (h * h)
    assert abs(f1 - fd1) <= 1e-7 * max(1.0, abs(f1)), (f1, fd1)
    assert abs(f2 - fd2) <= 1e-4 * max(1.0, abs(f2)), (f2, fd2)
    assert abs(f0 - 0.5 * np.sum((M - (U * S) @ V.T) ** 2)) < 1e-14


def test_cayley_curve_stays_orthonormal_and_starts_at_x():
    rng = np.random.default_rng(3)
    U, S, V = _previous(rng, 15, 6)
    M = rng.standard_normal((15, 6))
    PU, PS, PV = W.projected_gradients(U, S, V, M)
    assert np.allclose(PU, -PU.T) and np.allclose(PV, -PV.T)     # skew: tangent directions
    for t in (0.0, 0.3, -1.7, 5.0):
        Ut, St, Vt = W.curve(U, S, V, PU, PS, PV, t)
        assert np.allclose(Ut.T @ Ut, np.eye(6), atol=1e-12)
        assert np.allclose(Vt.T @ Vt, np.eye(6), atol=1e-12)
    Ut, St, Vt = W.curve(U, S, V, PU, PS, PV, 0.0)
    assert np.allclose(Ut, U) and np.allclose(Vt, V) and np.allclose(St, S)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_step_descends_and_shrinkage_is_within_the_bound(seed):
    rng = np.random.default_rng(seed)
    m, n = 18, 11
    M0 = rng.standard_normal((m, 3)) @ rng.standard_normal((3, n)) + 0.1 * rng.standard_normal((m, n))
    prev = W.svd_full(M0)
    M1 = M0 + 1e-3 * rng.standard_normal((m, n))
    dec, info = W.svdws(prev, M1, eps_svd=1e-2)
    assert info.warm and info.ft < info.f0
    approx = (dec.U * dec.S) @ dec.V.T
    for eps in (0.05, 0.3, 1.0):
        err = np.linalg.norm(W.shrink(dec, eps) - O.svt(M1, eps)[0])
        assert err <= np.linalg.norm(approx - M1) + 1e-12          # pseudocontraction of S_eps
    assert np.linalg.norm(approx - M1) <= np.linalg.norm(M0 - M1)  # the step does not move away


def test_switches_to_full_svd_beyond_threshold():
    rng = np.random.default_rng(7)
    M0 = rng.standard_normal((9, 6))
    prev = W.svd_full(M0)
    dec, info = W.svdws(prev, M0 + 0.5 * rng.standard_normal((9, 6)), eps_svd=1e-3)
    assert not info.warm
    U, S, Vt = np.linalg.svd(dec.M, full_matrices=False)
    assert np.allclose(dec.S, S)


def _inner_case():
    rng = np.random.default_rng(8)
    m, n, p = 30, 24, 3
    I = rng.uniform(0, 1, (m, n))
    J = rng.standard_normal((m * n, p))
    return I, O.Annihilator(J), 1.0 / np.sqrt(max(m, n))


def test_inner_loop_with_svdws_reaches_the_same_optimum():
    """The LADMAP inner loop with the warm-started decomposition in place of
    the full SVD (switch at eps_svd = 1e-3 relative) reaches the exact
    loop's objective to 1e-4.  (Consecutive iterates change by 0.1-46 % here
    -- every increase of the penalty moves M -- so the warm step is taken in
    a minority of the iterations; with a looser switch the approximate
    shrinkage stalls the loop.)"""
    I, Jp, lam = _inner_case()
    prm = O.Params()
    Z = np.zeros_like(I)
    exact = O.ladmap_inner(I, Jp, lam, I, Z, Z, prm)
    op = W.SvdwsSvt(eps_svd=1e-3)
    ws = O.ladmap_inner(I, Jp, lam, I, Z, Z, prm, svt_op=op)
    assert op.steps > 0
    oe = O.objective(exact.A, exact.E, lam)
    ow = O.objective(ws.A, ws.E, lam)
    assert abs(ow - oe) <= 1e-4 * oe, (ow, oe, op.steps)


def test_fixed_schedule_svt():
    """The fixed schedule: every = 1 is the exact loop bit for bit; with
    every = 2 the odd iterations are one Cayley step from the previous full
    SVD (the step the pinned curve functions give), and the loop still
    reaches the exact objective to 1e-4 (76 instead of 57 iterations)."""
    I, Jp, lam = _inner_case()
    prm = O.Params()
    Z = np.zeros_like(I)
    exact = O.ladmap_inner(I, Jp, lam, I, Z, Z, prm)
    one = O.ladmap_inner(I, Jp, lam, I, Z, Z, prm, svt_op=W.SvdwsSvt(every=1))
    assert one.iters == exact.iters and np.array_equal(one.A, exact.A) and np.array_equal(one.E, exact.E)
    rng = np.random.default_rng(3)
    M0 = rng.standard_normal((9, 6))
    M1 = M0 + 1e-2 * rng.standard_normal((9, 6))
    op = W.SvdwsSvt(every=2)
    A0, _ = op(M0, 0.1, 0)
    assert np.allclose(A0, O.svt(M0, 0.1)[0], atol=1e-12)
    A1, _ = op(M1, 0.1, 1)
    prev = W.svd_full(M0)
    PU, PS, PV = W.projected_gradients(prev.U, prev.S, prev.V, M1)
    f1, f2 = W.derivatives(prev.U, prev.S, prev.V, M1, PU, PS, PV)
    Ut, St, Vt = W.curve(prev.U, prev.S, prev.V, PU, PS, PV, -f1 / f2)
    assert op.steps == 1 and np.allclose(A1, W.shrink(W.WarmSVD(Ut, St, Vt, M1), 0.1), atol=1e-12)
    two_op = W.SvdwsSvt(every=2)
    two = O.ladmap_inner(I, Jp, lam, I, Z, Z, prm, svt_op=two_op)
    oe = O.objective(exact.A, exact.E, lam)
    assert two_op.steps == two.iters // 2 and two.iters < prm.max_inner
    assert abs(O.objective(two.A, two.E, lam) - oe) <= 1e-4 * oe
