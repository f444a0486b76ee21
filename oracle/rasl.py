"""RASL variant of the solve, in FP64.

TEST INFRASTRUCTURE.  Same rule as ``tilt_oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may
import or run it.

The paper states (Sec. 1, the paragraph on RASL) that TILT and RASL share one
model -- after the right transforms a data matrix splits into a low-rank and
a sparse part -- and differ only in the data matrix: one image window for
TILT, several images as the columns of the matrix for RASL.  This module
takes Alg. 1 with exactly that change:

* the data matrix D o tau is L x N with column k the window of image k
  warped by its own transform tau_k (L = m n pixels, the window's rows one
  after the other), each column normalised to unit norm;
* the Jacobian is block diagonal: column k depends on tau_k only, through
  J_k = d/dtau_k (D_k o tau_k / ||D_k o tau_k||) (L x p), so J_perp acts on
  every column separately, v_k - J_k (J_k^T J_k)^{-1} J_k^T v_k;
* Step 2 is the inner loop of Sec. 4.2 unchanged (``ladmap_inner``) with
  that projection;
* Step 3 is Delta tau_k = (J_k^T J_k)^{-1} J_k^T (a_k + e_k - d_k) per
  column, Step 4 tau_k <- tau_k + Delta tau_k.

Readings (the paper gives no RASL details): no extra constraints on the
transforms (the normalisation of each column is the only safeguard, p free
parameters per image); lambda = 1/sqrt(max(L, N)); every image carries its
own scaled coordinates (the window centre and s = max(m, n)/2 from its
initial transform); the outer loop stops when the norm of all Delta tau_k
together falls below eps_outer.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import tilt_oracle as T


class ColumnAnnihilator:
    """J_perp for a block-diagonal Jacobian: column k of V (L x N) is
    projected onto the orthogonal complement of range(J_k)."""

    def __init__(self, Js: List[np.ndarray]):
        self.Js = [np.asarray(J, dtype=np.float64) for J in Js]
        self.G = []
        for J in self.Js:
            G = J.T @ J
            if J.shape[1]:
                ev = np.linalg.eigvalsh(G)
                if not (ev[0] > 1e-14 * max(ev[-1], 1e-300)):
                    raise np.linalg.LinAlgError("J_k^T J_k is singular")
            self.G.append(G)

    def coeffs(self, V: np.ndarray) -> List[np.ndarray]:
        """(J_k^T J_k)^{-1} J_k^T v_k for every column k."""
        out = []
        for k, (J, G) in enumerate(zip(self.Js, self.G)):
            out.append(np.linalg.solve(G, J.T @ V[:, k]) if J.shape[1] else np.zeros(0))
        return out

    def __call__(self, V: np.ndarray) -> np.ndarray:
        out = np.array(V, dtype=np.float64, copy=True)
        for k, c in enumerate(self.coeffs(V)):
            if c.size:
                out[:, k] -= self.Js[k] @ c
        return out


@dataclasses.dataclass
class ImageFrame:
    """Scaled coordinates of image k: tau_k entries, window centre c, s."""

    tau: np.ndarray
    c: np.ndarray
    s: float


def frames_from_px(tau0_px, m, n, model) -> List[ImageFrame]:
    frames = []
    for H in tau0_px:
        Hn, c, s = T.normalise_transform(np.asarray(H, dtype=np.float64), m, n)
        if model == T.AFFINE:
            Hn[2, :] = [0.0, 0.0, 1.0]
        frames.append(ImageFrame(T.tau_from_matrix(Hn, model), np.asarray(c, dtype=np.float64), float(s)))
    return frames


def rasl_step1(images, frames: List[ImageFrame], m, n, model):
    """Step 1 for every image: the L x N data matrix (normalised columns)
    and the per-column Jacobians J_k (L x p)."""
    cols, Js = [], []
    for img, fr in zip(images, frames):
        Hn = T.matrix_from_tau(fr.tau, model)
        I, J, _ = T.step1(np.asarray(img, dtype=np.float64), Hn, fr.c, fr.s, m, n, model)
        cols.append(I.reshape(-1))
        Js.append(J)
    return np.stack(cols, axis=1), Js


@dataclasses.dataclass
class RaslResult:
    tau_px: np.ndarray        # (N, 3, 3) centred grid px -> image px
    A: np.ndarray             # L x N
    E: np.ndarray
    Y: np.ndarray
    outer_iters: int
    inner_iters: list
    objective: float
    status: int
    history: list


def rasl_solve(images, tau0_px, m, n, model, prm: Optional[T.Params] = None, lam=None) -> RaslResult:
    """Alg. 1 with the RASL data matrix (see the module notes)."""
    prm = prm or T.Params()
    if model not in (T.AFFINE, T.PROJECTIVE):
        raise ValueError("model must be 6 (affine) or 8 (projective)")
    N = len(images)
    L = m * n
    if lam is None:
        lam = prm.lam if prm.lam > 0 else 1.0 / math.sqrt(max(L, N))
    frames = frames_from_px(tau0_px, m, n, model)
    A = E = Y = None
    inner_counts, hist = [], []
    status = 0
    i = 0
    while i < prm.max_outer:
        D, Js = rasl_step1(images, frames, m, n, model)          # Step 1
        if A is None:
            A = D.copy()
            E = np.zeros_like(D)
            Y = np.zeros_like(D)
        Jp = ColumnAnnihilator(Js)
        res = T.ladmap_inner(D, Jp, lam, A, E, Y, prm)            # Step 2
        A, E, Y = res.A, res.E, res.Y
        inner_counts.append(res.iters)
        if res.iters >= prm.max_inner and not prm.fixed_iters:
            status = 1
        dt = Jp.coeffs(A + E - D)                                 # Step 3
        nrm2 = 0.0
        for fr, d in zip(frames, dt):                             # Step 4
            fr.tau = fr.tau + d
            nrm2 += float(d @ d)
        i += 1
        hist.append(dict(dtau_norm=math.sqrt(nrm2), inner=res.iters, mu=res.mu, cond1=res.cond1,
                         cond2=res.cond2))
        if not all(np.all(np.isfinite(fr.tau)) for fr in frames):
            status = -5
            break
        if not prm.fixed_iters and math.sqrt(nrm2) < prm.eps_outer:
            break
    taus = np.stack([T.denormalise_transform(T.matrix_from_tau(fr.tau, model), fr.c, fr.s) for fr in frames])
    return RaslResult(tau_px=taus, A=A, E=E, Y=Y, outer_iters=i, inner_iters=inner_counts,
                      objective=T.objective(A, E, lam), status=status, history=hist)
