"""tilt_svdws_batch (SVD with warm start, Sec. 5 Alg. 2 with the
derivatives of Appendix A) against the FP64 oracle ``oracle.svdws`` on the
same FP32 inputs: one Cayley step per matrix from the decomposition of the
previous matrix, the Sherman-Morrison-Woodbury form on the device against
the oracle's direct m x m inverse.

Inputs: M0 = rank-3 + 5 % noise (the statistics of a low-rank patch), its
SVD (U, S, V) in FP64 rounded to FP32, and the next matrix M = M0 + delta
G ||M0|| / ||G|| with G Gaussian: the change between consecutive outer
iterations that Alg. 2 hands the warm step (delta from 1e-3 to 3e-2).
Tolerances (FP32 products against FP64): the step size t and f(t) agree
to 1e-3 relative (both are built from inner products of M - X, whose FP32
rounding of ~1e-7 ||M|| sits on a difference of size delta ||M||: 1.5e-4
was measured at delta = 1e-3); U(t), V(t) to 5e-6 and S(t), A to 5e-6
||.|| (measured <= 5e-7); U(t) keeps orthonormal columns to 2e-6 (the
Cayley factor is orthogonal; measured <= 4e-7)."""

import numpy as np
import pytest

from oracle import svdws as SW
from gpu_util import to_device

pytestmark = pytest.mark.gpu


def _case(m, n, delta, seed):
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((m, 3)) @ rng.standard_normal((3, n))
    M0 = L / np.linalg.norm(L) + 0.05 * rng.standard_normal((m, n)) / np.sqrt(m * n)
    G = rng.standard_normal((m, n))
    M = M0 + delta * G * np.linalg.norm(M0) / np.linalg.norm(G)
    d = SW.svd_full(M0)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return f32(d.U), f32(d.S), f32(d.V), f32(M)


def _run(ctx, device, U, S, V, M, eps=None):
    import torch

    count, m, n = M.shape
    dU, dS, dV, dM = (to_device(a, device) for a in (U, S, V, M))
    oU = torch.full_like(dU, float("nan"))
    oS = torch.full_like(dS, float("nan"))
    oV = torch.full_like(dV, float("nan"))
    oA = torch.full_like(dM, float("nan")) if eps is not None else None
    print(f"tilt_svdws_batch: {count} x {m}x{n}", flush=True)
    rc, t, f0, ft, st = ctx.svdws_batch(count, m, n, dU.data_ptr(), dS.data_ptr(), dV.data_ptr(), dM.data_ptr(),
                                        oU.data_ptr(), oS.data_ptr(), oV.data_ptr(),
                                        oA.data_ptr() if oA is not None else 0, eps)
    torch.cuda.synchronize()
    out = [oU.cpu().numpy(), oS.cpu().numpy(), oV.cpu().numpy(), oA.cpu().numpy() if oA is not None else None]
    return rc, t, f0, ft, st, out


def _oracle(U, S, V, M):
    f64 = lambda a: a.astype(np.float64)
    prev = SW.WarmSVD(f64(U), f64(S), f64(V), None)
    Mx = f64(M)
    PU, PS, PV = SW.projected_gradients(prev.U, prev.S, prev.V, Mx)
    f1, f2 = SW.derivatives(prev.U, prev.S, prev.V, Mx, PU, PS, PV)
    f0 = 0.5 * float(np.sum((Mx - (prev.U * prev.S) @ prev.V.T) ** 2))
    if not f2 > 0.0:
        return None, f0
    t = -f1 / f2
    Ut, St, Vt = SW.curve(prev.U, prev.S, prev.V, PU, PS, PV, t)
    ft = SW.f_of_t(prev.U, prev.S, prev.V, Mx, PU, PS, PV, t)
    return (SW.WarmSVD(Ut, St, Vt, Mx), t, ft), f0


@pytest.mark.parametrize("m,n", [(40, 24), (100, 100), (130, 57), (7, 1)])
def test_svdws_step_matches_oracle(ctx, device, m, n):
    deltas = [1e-3, 3e-3, 1e-2, 3e-2]
    cases = [_case(m, n, d, 900 + 7 * m + n + k) for k, d in enumerate(deltas)]
    U, S, V, M = (np.stack([c[i] for c in cases]) for i in range(4))
    eps = np.full(len(cases), 0.02, np.float32)
    rc, t, f0, ft, st, (oU, oS, oV, oA) = _run(ctx, device, U, S, V, M, eps)
    assert rc == 0
    for i in range(len(cases)):
        ref, f0_ref = _oracle(U[i], S[i], V[i], M[i])
        assert ref is not None, "these inputs have f''(0) > 0"
        dec, t_ref, ft_ref = ref
        assert st[i] == 0, (i, st[i])
        dt = abs(t[i] - t_ref) / abs(t_ref)
        dU = np.abs(oU[i] - dec.U).max()
        dV = np.abs(oV[i] - dec.V).max()
        dS = np.abs(oS[i] - dec.S).max() / np.abs(dec.S).max()
        Aref = SW.shrink(dec, float(eps[i]))
        dA = np.linalg.norm(oA[i] - Aref) / max(np.linalg.norm(Aref), 1e-30)
        orth = np.abs(oU[i].astype(np.float64).T @ oU[i] - np.eye(n)).max()
        print(f"  [{i}] delta {deltas[i]:.0e} t {t[i]:.6g}/{t_ref:.6g} (rel {dt:.1e}) f(t)/f(0) {ft[i] / f0[i]:.3g} "
              f"dU {dU:.1e} dV {dV:.1e} dS {dS:.1e} dA {dA:.1e} orth {orth:.1e}")
        assert dt <= 1e-3, (i, t[i], t_ref)
        assert abs(f0[i] - f0_ref) <= 1e-3 * f0_ref
        assert abs(ft[i] - ft_ref) <= 1e-3 * ft_ref + 1e-6 * f0_ref
        assert ft[i] < f0[i]                       # the step lowers the fit error
        assert dU <= 5e-6 and dV <= 5e-6 and dS <= 5e-6 and dA <= 5e-6, (i, dU, dV, dS, dA)
        assert orth <= 2e-6


def test_svdws_no_minimum_returns_inputs(ctx, device):
    """f''(0) <= 0 (next matrix unrelated to the previous one): no step,
    outputs are the inputs bit for bit, status 1 (Alg. 2's caller then
    computes a full SVD); the other matrices of the batch still step."""
    rng = np.random.default_rng(0)
    m, n = 12, 5
    M0 = rng.standard_normal((m, n))
    M1 = rng.standard_normal((m, n))
    d = SW.svd_full(M0)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    bad = (f32(d.U), f32(d.S), f32(d.V), f32(M1))
    good = _case(m, n, 1e-2, 5)
    U, S, V, M = (np.stack([bad[i], good[i]]) for i in range(4))
    ref, _ = _oracle(*bad)
    assert ref is None, "the oracle finds f''(0) <= 0 on this input"
    rc, t, f0, ft, st, (oU, oS, oV, _) = _run(ctx, device, U, S, V, M)
    assert rc == 0
    assert list(st) == [1, 0]
    assert t[0] == 0.0 and ft[0] == f0[0]
    assert np.array_equal(oU[0], U[0]) and np.array_equal(oS[0], S[0]) and np.array_equal(oV[0], V[0])
    assert np.all(np.isfinite(oU[1])) and ft[1] < f0[1]


def test_svdws_rejects_bad_shapes(tilt, ctx, device):
    import torch

    z = torch.zeros((64,), dtype=torch.float32, device=device)
    p = z.data_ptr()
    for m, n in ((4, 5), (10, 0), (5000, 10), (300, 257)):
        with pytest.raises(tilt.TiltError) as e:
            ctx.svdws_batch(1, m, n, p, p, p, p, p, p, p)
        assert e.value.code == tilt.tilt.TILT_ERR_ARG
    # an empty batch is a no-op
    rc, *_ = ctx.svdws_batch(0, 8, 4, p, p, p, p, p, p, p)
    assert rc == 0


# ---------------------------------------------------------------------------
# svt_mode 4: Alg. 2 as the SVT of the solver's inner loop, against the
# oracle's inner loop with the same switch (oracle.svdws.SvdwsSvt).
# ---------------------------------------------------------------------------


def _inner_inputs(tilt, m, n, p, count, device):
    import torch
    import tilt_synth as ts

    Is, Js = zip(*[ts.inner_problem(k, m, n, p) for k in range(count)])
    dI = to_device(np.stack(Is), device)
    dJ = to_device(np.stack(Js), device)
    return Is, Js, dI, dJ, torch.zeros_like(dI), torch.zeros_like(dI)


def _oracle_inner(O, I, J, tp, lam, op):
    mn = I.size
    Jm = J.reshape(J.shape[0], mn).T.astype(np.float64)
    I64 = I.astype(np.float64)
    Z = np.zeros_like(I64)
    from gpu_util import oracle_params
    return O.ladmap_inner(I64, O.Annihilator(Jm), lam, I64, Z, Z, oracle_params(O, tp), svt_op=op)


@pytest.mark.parametrize("m,n,p,fixed", [(40, 30, 3, True), (100, 100, 5, True), (64, 48, 5, False)])
def test_svdws_inner_loop_fixed_schedule_matches_oracle(tilt, ctx, device, m, n, p, fixed):
    """Full SVD in even iterations, the Cayley step in odd ones (svdws_every
    = 2): the device's decomposition comes from the warm-started Jacobi, the
    oracle's from LAPACK -- the step depends on them only through
    U Sigma V^T and the per-triplet P_Sigma, so both reach the same A.
    Same tolerances as the inner-loop parity tests (1e-4)."""
    import math

    import oracle as O

    count = 3
    Is, Js, dI, dJ, dA, dE = _inner_inputs(tilt, m, n, p, count, device)
    tp = tilt.default_params(svt_mode=4, svdws_every=2, fixed_iters=1 if fixed else 0,
                             max_inner=25 if fixed else 2000)
    print(f"svt_mode 4 inner loop {count} x {m}x{n} fixed={fixed}", flush=True)
    rc, res = ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), count, m, n, p, tp, dA.data_ptr(), dE.data_ptr())
    A = dA.cpu().numpy()
    lam = 1.0 / math.sqrt(max(m, n))
    for k in range(count):
        op = O.svdws.SvdwsSvt(every=2)
        ref = _oracle_inner(O, Is[k], Js[k], tp, lam, op)
        r = res[k]
        errA = np.linalg.norm(A[k] - ref.A) / np.linalg.norm(ref.A)
        obj = O.objective(ref.A, ref.E, lam)
        print(f"  [{k}] iters {r['inner_iters_total']}/{ref.iters} steps {r['counters']['svdws_steps']}/{op.steps} "
              f"A {errA:.1e} obj {abs(r['objective'] - obj) / obj:.1e}", flush=True)
        assert r["status"] >= 0
        assert errA <= 1e-4
        assert abs(r["objective"] - obj) <= 1e-4 * obj
        if fixed:
            assert r["inner_iters_total"] == 25 and r["counters"]["svdws_steps"] == op.steps == 12
        else:
            assert abs(r["inner_iters_total"] - ref.iters) <= max(3, 0.1 * ref.iters)
            assert r["counters"]["svdws_steps"] > 0


def test_svdws_inner_loop_threshold_rule(tilt, ctx, device):
    """Alg. 2's own switch (eps_svd = 1e-3): FP32 and FP64 may take it
    differently near the threshold, so the counts of Cayley steps are
    compared loosely; the objective must match the oracle's Alg. 2 loop and
    the exact loop to 1e-4 (the oracle pin of the method)."""
    import math

    import oracle as O

    m, n, p, count = 64, 48, 5, 3
    Is, Js, dI, dJ, dA, dE = _inner_inputs(tilt, m, n, p, count, device)
    tp = tilt.default_params(svt_mode=4, eps_svd=1e-3)
    rc, res = ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), count, m, n, p, tp, dA.data_ptr(), dE.data_ptr())
    lam = 1.0 / math.sqrt(max(m, n))
    for k in range(count):
        op = O.svdws.SvdwsSvt(eps_svd=1e-3)
        ref = _oracle_inner(O, Is[k], Js[k], tp, lam, op)
        exact = _oracle_inner(O, Is[k], Js[k], tp, lam, None)
        r = res[k]
        obj = O.objective(ref.A, ref.E, lam)
        obj_exact = O.objective(exact.A, exact.E, lam)
        print(f"  [{k}] iters {r['inner_iters_total']}/{ref.iters} (exact {exact.iters}) steps "
              f"{r['counters']['svdws_steps']}/{op.steps}", flush=True)
        assert r["status"] >= 0
        assert abs(r["objective"] - obj) <= 1e-4 * obj
        assert abs(r["objective"] - obj_exact) <= 1e-4 * obj_exact


def test_svdws_fused_solve_matches_oracle(tilt, ctx, device):
    """svt_mode 4 inside the fused kernel (whole TILT solves): a 100 x 100
    projective patch for 2 outer x 15 inner fixed iterations with the fixed
    schedule (full SVD in even inner iterations) against the oracle's Alg. 1
    with the same SVT, to the full-solve tolerance (1e-4 in tau and the
    objective); 2 x 7 Cayley steps unless a step falls back."""
    import oracle as O
    import tilt_synth as ts
    from gpu_util import oracle_params, solve_on_device

    p = ts.make_batch(1, [3])[0]
    tp = tilt.default_params(lam=p.lam, svt_mode=4, svdws_every=2, fixed_iters=1, max_outer=2, max_inner=15)
    print("svt_mode 4 fused solve 100x100", flush=True)
    _, res = solve_on_device(tilt, ctx, [p], device, tp)
    r = res[0]
    ops = []

    def factory():
        ops.append(O.svdws.SvdwsSvt(every=2))
        return ops[-1]

    ref = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, oracle_params(O, tp), lam=p.lam, svt_op_factory=factory)
    terr = O.tau_rel_err(r["tau"], ref.tau_px, p.m, p.n)
    steps = sum(o.steps for o in ops)
    print(f"  tau {terr:.1e} objective {abs(r['objective'] - ref.objective) / ref.objective:.1e} steps "
          f"{r['counters']['svdws_steps']}/{steps}", flush=True)
    assert r["status"] >= 0 and r["counters"]["svdws_steps"] == steps and steps >= 10
    assert terr <= 1e-4
    assert abs(r["objective"] - ref.objective) <= 1e-4 * ref.objective


def test_svdws_mode_outside_the_warm_layout_runs_the_cold_svt(tilt, ctx, device):
    """svt_mode 4 needs the warm-started Jacobi in LDS; on a shape whose
    rotation does not fit beside the rows (175 x 158) the SVT is the cold
    one: the inner loop equals svt_mode 0 bit for bit and takes no step."""
    m, n, p, count = 175, 158, 3, 2
    _, _, dI, dJ, dA0, dE0 = _inner_inputs(tilt, m, n, p, count, device)
    import torch

    dA4, dE4 = torch.zeros_like(dA0), torch.zeros_like(dE0)
    t0 = tilt.default_params(svt_mode=0, fixed_iters=1, max_inner=6)
    t4 = tilt.default_params(svt_mode=4, svdws_every=2, fixed_iters=1, max_inner=6)
    print(f"svt_mode 0 and 4 on {count} x {m}x{n}", flush=True)
    _, r0 = ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), count, m, n, p, t0, dA0.data_ptr(), dE0.data_ptr())
    _, r4 = ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), count, m, n, p, t4, dA4.data_ptr(), dE4.data_ptr())
    assert torch.equal(dA0, dA4) and torch.equal(dE0, dE4)
    assert all(r["counters"]["svdws_steps"] == 0 for r in r4)


def test_svdws_mode_served_equals_batched_over_pyramid_levels(tilt, device):
    """svt_mode 4 (fixed schedule) through the serving kernel, three pyramid
    levels per request (the decomposition is dropped at each level change):
    the same bits as the batched fused launch, and Cayley steps taken."""
    import tilt_synth as ts
    from gpu_util import solve_on_device
    from test_gpu_serving import _same, _serve

    ps = ts.make_batch(4, [20, 15, 7, 3])
    tp = tilt.default_params(svt_mode=4, svdws_every=2, pyramid_levels=3, max_outer=4, max_inner=40)
    print("svt_mode 4 served vs batched, 4 requests x 3 levels", flush=True)
    with tilt.Context(0) as c:
        served = _serve(tilt, c, device, ps, tp)
        _, batched = solve_on_device(tilt, c, ps, device, tp)
    for a, b in zip(served, batched):
        assert a["status"] == b["status"] and _same(a, b)
    assert sum(b["counters"]["svdws_steps"] for b in batched) > 0
