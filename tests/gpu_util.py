"""Helpers for the GPU tests: device copies of synthetic patches and calls
through the C interface.  Inputs come from ``tilt_synth``; expected values
come from ``oracle`` only."""

from __future__ import annotations

import numpy as np


def same_numerical_rank(O, A_dev, A_ref, rel=1e-3):
    """Numerical rank #{sigma_i > rel sigma_1} of the device result against
    the oracle's.  The count jumps at the cut, so it is compared as far as
    the two matrices determine it: by Weyl's inequality each singular value
    of A_dev lies within d = ||A_dev - A_ref||_2 of the matching one of
    A_ref (and the cut rel sigma_1 moves by at most rel d), so the counts
    may differ only by oracle singular values within (1 + rel) d of the
    cut, and only while d is below a quarter of the cut (so no singular
    value further than 25 % from the cut may fall on the other side).
    Returns (agree, rank_dev, rank_ref)."""
    a = np.asarray(A_dev, dtype=np.float64)
    b = np.asarray(A_ref, dtype=np.float64)
    r_dev, r_ref = O.numerical_rank(a, rel), O.numerical_rank(b, rel)
    if r_dev == r_ref:
        return True, r_dev, r_ref
    d = float(np.linalg.norm(a - b, 2))
    sv = np.linalg.svd(b, compute_uv=False)
    cut = rel * sv[0]
    lo, hi = min(r_dev, r_ref), max(r_dev, r_ref)
    agree = d <= 0.25 * cut and all(abs(sv[i] - cut) <= (1.0 + rel) * d for i in range(lo, hi))
    return agree, r_dev, r_ref


def to_device(arr, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)


def device_problems(T, patches, device, tau0s=None):
    """Upload images; returns (problems, keep-alive tensors)."""
    keep = []
    probs = []
    for i, p in enumerate(patches):
        img = to_device(p.image.astype(np.float32), device)
        keep.append(img)
        tau0 = p.tau0 if tau0s is None else tau0s[i]
        probs.append(T.make_problem(img.data_ptr(), p.height, p.width, p.width, p.m, p.n, p.model, tau0))
    return probs, keep


def solve_on_device(T, ctx, patches, device, params, plain=False):
    """Solve patches through tilt_solve_batch (or the plain variant).
    Returns (rc, results with numpy A/E)."""
    import torch

    probs, keep = device_problems(T, patches, device)
    As = [torch.zeros((p.m, p.n), dtype=torch.float32, device=device) for p in patches]
    Es = [torch.zeros((p.m, p.n), dtype=torch.float32, device=device) for p in patches]
    fn = ctx.solve_batch_plain if plain else ctx.solve_batch
    rc, res = fn(probs, params, [a.data_ptr() for a in As], [e.data_ptr() for e in Es])
    torch.cuda.synchronize()
    for r, a, e in zip(res, As, Es):
        r["A"] = a.cpu().numpy()
        r["E"] = e.cpu().numpy()
    del keep
    return rc, res


def oracle_params(O, tp, **kw):
    """Oracle parameters equal to the library's parameter struct."""
    return O.Params(lam=tp.lambda_, eps1=tp.eps1, eps2=tp.eps2, eps_outer=tp.eps_outer, mu0=tp.mu0,
                    rho0=tp.rho0, mu_max=tp.mu_max, max_inner=tp.max_inner, max_outer=tp.max_outer,
                    fixed_iters=bool(tp.fixed_iters), eps_obj=tp.eps_obj, **kw)
