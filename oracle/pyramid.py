"""Coarse-to-fine image pyramid around the TILT solve, in FP64.

TEST INFRASTRUCTURE.  Same rule as ``tilt_oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may
import or run it.

The paper runs TILT on single windows and does not describe a pyramid; the
serving workload (640x480 images, windows of 40..400 pixels) solves
coarse to fine.  The reading used by both this oracle and the device path:

* level l+1 is level l blurred with the separable binomial kernel
  [1 4 6 4 1]/16 (indices clamped at the borders) and sampled at every
  second pixel: pixel (i, j) of level l+1 is the blurred value at pixel
  (2i, 2j) of level l.  Level l+1 has ceil(H/2) x ceil(W/2) pixels;
* the window at level l has ceil(m / 2^l) x ceil(n / 2^l) samples;
* pixel and centred grid coordinates both halve from one level to the
  next, so a homography moves between levels by conjugation with
  S = diag(1/2, 1/2, 1):  H_{l+1} = S H_l S^{-1};
* the levels are solved from the coarsest to level 0, each by the whole
  of Alg. 1 started cold (A = D o tau, E = Y = 0) from the transform the
  coarser level returned; lambda is the caller's, or 1/sqrt(max(m_l, n_l))
  per level when not given.
"""

from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .tilt_oracle import Params, SolveResult, tilt_solve

BINOMIAL5 = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


def blur_decimate(img: np.ndarray) -> np.ndarray:
    """One pyramid step: binomial blur (clamped borders) at the even pixels."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    Ho, Wo = (H + 1) // 2, (W + 1) // 2
    taps = np.arange(-2, 3)
    rows = np.clip(2 * np.arange(Ho)[:, None] + taps[None, :], 0, H - 1)   # Ho x 5
    cols = np.clip(2 * np.arange(Wo)[:, None] + taps[None, :], 0, W - 1)   # Wo x 5
    vert = np.tensordot(img[rows], BINOMIAL5, axes=([1], [0]))             # Ho x W
    return np.tensordot(vert[:, cols], BINOMIAL5, axes=([2], [0]))         # Ho x Wo


def build_pyramid(img: np.ndarray, levels: int) -> List[np.ndarray]:
    out = [np.asarray(img, dtype=np.float64)]
    for _ in range(1, levels):
        out.append(blur_decimate(out[-1]))
    return out


def level_shape(m: int, n: int, level: int):
    f = 1 << level
    return (m + f - 1) // f, (n + f - 1) // f


def to_coarser(H: np.ndarray) -> np.ndarray:
    """H_{l+1} = S H_l S^{-1}."""
    S = np.diag([0.5, 0.5, 1.0])
    G = S @ np.asarray(H, dtype=np.float64) @ np.diag([2.0, 2.0, 1.0])
    return G / G[2, 2]


def to_finer(H: np.ndarray) -> np.ndarray:
    """H_l = S^{-1} H_{l+1} S."""
    G = np.diag([2.0, 2.0, 1.0]) @ np.asarray(H, dtype=np.float64) @ np.diag([0.5, 0.5, 1.0])
    return G / G[2, 2]


def tilt_solve_pyramid(image, tau0_px, m, n, model, prm: Optional[Params] = None, levels: int = 3,
                       lam: Optional[float] = None):
    """Solve coarse to fine; returns (level-0 result, list of per-level results,
    coarsest first)."""
    prm = prm or Params()
    if levels < 1:
        raise ValueError("levels must be >= 1")
    imgs = build_pyramid(image, levels)
    H = np.asarray(tau0_px, dtype=np.float64)
    for _ in range(levels - 1):
        H = to_coarser(H)
    per_level: List[SolveResult] = []
    res = None
    for lvl in range(levels - 1, -1, -1):
        ml, nl = level_shape(m, n, lvl)
        if ml < 2 or nl < 2:
            raise ValueError("window too small for this many levels")
        if lam is not None and lam > 0:
            lam_l = lam
        elif prm.lam > 0:
            lam_l = prm.lam
        else:
            lam_l = 1.0 / math.sqrt(max(ml, nl))
        res = tilt_solve(imgs[lvl], H, ml, nl, model, prm, lam=lam_l)
        per_level.append(res)
        if res.status < 0:
            break
        H = res.tau_px if lvl == 0 else to_finer(res.tau_px)
    return res, per_level
