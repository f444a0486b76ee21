"""Plain FP64 CPU oracle for TILT solved by LADMAP with variable warm start.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (the HIP library and its Python binding) never
imports it and shares no code with it.

Paper: X. Ren and Z. Lin, "Linearized Alternating Direction Method with
Adaptive Penalty and Warm Starts for Fast Solving Transform Invariant
Low-Rank Textures" (IJCV; arXiv 1205.5351).

What is computed, in the paper's order and notation:

* Alg. 1 (TILT via LADMAP+VWS), outer loop: Step 1 normalises D o tau and
  forms J = d/dzeta (D o zeta / ||D o zeta||_F); Step 2 solves the linearised
  convex problem (Eq. TILT_LADMAP) by LADMAP; Step 3 takes Delta tau from
  Eq. Delta_tau; Step 4 sets tau <- tau + Delta tau.
* Sec. 3.2 / Sec. 4.2 inner loop: A = S_{1/mu}(M) (Eq. A_1, S_operator),
  E = T_{lambda/mu}(N) (Eq. E_1), Y += mu J_perp(A + E - D o tau) (Eq. Y),
  mu = min(mu_max, rho mu) (Eq. mu) with rho from Eq. rho; stop on Cond1 and
  Cond2.  Y is kept in span(J_perp) (Sec. 4.2) and warm-started as
  Y_0 = J_perp Y_inf (Eq. warm_start_Y); A, E are warm-started from the
  previous inner loop (Eq. warm_start).
* J_perp v = v - J (J^T J)^{-1} J^T v (Eq. Jperpv).
* Extra constraints Q Delta tau = 0 (Sec. 4.3, Eq. add_constraints).  The
  oracle eliminates them through an orthonormal basis N_Q of null(Q) and the
  reduced Jacobian J~ = J N_Q; the W-formulation of Sec. 4.3 is provided as
  ``ladmap_inner_w`` for cross-checking on small cases (same optimum).

Readings where the paper is silent or inconsistent (all listed in the
design notes of the repository):

* sign of the Y update: +mu as in Eq. Y and Sec. 4.2/4.3 (Alg. 1 prints -mu);
* N_k of Sec. 4.3 starts from E_k (as in Sec. 3.2), not from A_{k+1};
* the dual bound is ||J_perp Y||_inf <= lambda (the printed lambda^{-1} is
  the reciprocal of the l1 weight's subgradient bound);
* Q: the image of the rectified centre (2 rows) and the area of the image of
  the rectified rectangle (1 row) are held fixed to first order;
* bilinear interpolation with pixel centres at integers; the gradient is the
  exact derivative of the interpolant, taken from the cell right of / below
  a pixel line for samples within 1e-9 px of it; outside the image the sample
  is clamped to the border and its gradient along the clamped axis is zero;
* tau is a homography in coordinates scaled by s = max(m, n)/2 about the
  image of the window centre; affine uses 6 entries, projective 8 (h33 = 1);
* mu_0 = 1.25 / ||D o tau||_2 at the start of every inner loop unless given;
* the outer loop stops when ||Delta tau||_2 < eps_outer or after max_outer
  iterations.

Every function that has a plain definition is that definition written out
(exact SVD from LAPACK for the shrinkage, a dense solve for the Gram system).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

AFFINE = 6
PROJECTIVE = 8
SNAP = 1e-9  # pixels: cell-edge convention of the bilinear gradient


# ---------------------------------------------------------------------------
# Parameters (defaults follow the readings above)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Params:
    lam: float = -1.0          # <= 0 -> 1/sqrt(max(m, n))
    eps1: float = 1e-5         # Cond1 threshold (Eq. Cond1)
    eps2: float = 1e-3         # Cond2 / rho threshold (Eq. Cond2, Eq. rho)
    eps_outer: float = 1e-5    # outer stop on ||Delta tau||_2
    mu0: float = -1.0          # <= 0 -> 1.25 / ||D o tau||_2
    rho0: float = 1.5          # rho_0 >= 1 (Eq. rho)
    mu_max: float = 1e10       # upper bound of mu (Eq. mu)
    max_inner: int = 2000
    max_outer: int = 50
    fixed_iters: bool = False  # run exactly max_outer x max_inner, no stop tests
    eps_obj: float = 0.0       # also stop when |f_i - f_{i-1}| < eps_obj f_{i-1} (0: off)


# ---------------------------------------------------------------------------
# Transform parametrisation
# ---------------------------------------------------------------------------


def grid_scale(m: int, n: int) -> float:
    return max(m, n) / 2.0


def normalise_transform(H_px: np.ndarray, m: int, n: int):
    """Pixel homography -> (H_norm, centre, s).

    The centre c is the image of the rectified grid centre under H_px; it is
    the origin of the normalised image coordinates for the whole solve.
    H_norm = T_img^{-1} H_px S_grid with S_grid = diag(s, s, 1) and
    T_img = [[s, 0, cx], [0, s, cy], [0, 0, 1]], scaled so that h33 = 1.
    """
    H = np.asarray(H_px, dtype=np.float64).reshape(3, 3)
    H = H / H[2, 2]
    s = grid_scale(m, n)
    c = np.array([H[0, 2], H[1, 2]])
    Timg_inv = np.array([[1.0 / s, 0.0, -c[0] / s], [0.0, 1.0 / s, -c[1] / s], [0.0, 0.0, 1.0]])
    Sg = np.diag([s, s, 1.0])
    Hn = Timg_inv @ H @ Sg
    Hn = Hn / Hn[2, 2]
    return Hn, c, s


def denormalise_transform(Hn: np.ndarray, c, s: float) -> np.ndarray:
    Timg = np.array([[s, 0.0, c[0]], [0.0, s, c[1]], [0.0, 0.0, 1.0]])
    Sg_inv = np.diag([1.0 / s, 1.0 / s, 1.0])
    H = Timg @ Hn @ Sg_inv
    return H / H[2, 2]


def tau_from_matrix(Hn: np.ndarray, model: int) -> np.ndarray:
    """tau = (h11, h12, h13, h21, h22, h23[, h31, h32])."""
    v = [Hn[0, 0], Hn[0, 1], Hn[0, 2], Hn[1, 0], Hn[1, 1], Hn[1, 2]]
    if model == PROJECTIVE:
        v += [Hn[2, 0], Hn[2, 1]]
    return np.array(v, dtype=np.float64)


def matrix_from_tau(tau: np.ndarray, model: int) -> np.ndarray:
    H = np.eye(3)
    H[0, :] = tau[0:3]
    H[1, :] = tau[3:6]
    if model == PROJECTIVE:
        H[2, 0], H[2, 1] = tau[6], tau[7]
    return H


def grid_coords(m: int, n: int, s: float):
    """Normalised rectified coordinates (ut, vt), each m x n."""
    j = np.arange(n, dtype=np.float64)
    i = np.arange(m, dtype=np.float64)
    ut = (j - (n - 1) / 2.0) / s
    vt = (i - (m - 1) / 2.0) / s
    UT, VT = np.meshgrid(ut, vt)
    return UT, VT


# ---------------------------------------------------------------------------
# Step 1: warp, gradient of the interpolant, Jacobian (Alg. 1, Step 1)
# ---------------------------------------------------------------------------


def bilinear_with_gradient(img: np.ndarray, x: np.ndarray, y: np.ndarray):
    """Bilinear sample of img at (x, y) and the exact partial derivatives of
    the interpolant.  Pixel centres at integer coordinates; outside the
    image the coordinate is clamped and the derivative along that axis is 0.
    """
    D = np.asarray(img, dtype=np.float64)
    Hh, Ww = D.shape
    if Hh < 2 or Ww < 2:
        raise ValueError("image must be at least 2x2")
    xc = np.clip(x, 0.0, Ww - 1.0)
    yc = np.clip(y, 0.0, Hh - 1.0)
    # a sample within SNAP pixels below a pixel line belongs to the next
    # cell, so coordinates that sit on the pixel grid up to rounding always
    # take the same one-sided gradient
    x0 = np.minimum(np.floor(xc + SNAP), Ww - 2).astype(np.int64)
    y0 = np.minimum(np.floor(yc + SNAP), Hh - 2).astype(np.int64)
    fx = xc - x0
    fy = yc - y0
    v00 = D[y0, x0]
    v01 = D[y0, x0 + 1]
    v10 = D[y0 + 1, x0]
    v11 = D[y0 + 1, x0 + 1]
    val = (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11)
    dx = (1 - fy) * (v01 - v00) + fy * (v11 - v10)
    dy = (1 - fx) * (v10 - v00) + fx * (v11 - v01)
    inside_x = (x >= 0.0) & (x <= Ww - 1.0)
    inside_y = (y >= 0.0) & (y <= Hh - 1.0)
    dx = np.where(inside_x, dx, 0.0)
    dy = np.where(inside_y, dy, 0.0)
    return val, dx, dy


def warp(img, Hn, c, s, m, n):
    """D o tau on the m x n grid plus the geometric terms of the Jacobian."""
    UT, VT = grid_coords(m, n, s)
    X = Hn[0, 0] * UT + Hn[0, 1] * VT + Hn[0, 2]
    Y = Hn[1, 0] * UT + Hn[1, 1] * VT + Hn[1, 2]
    Wh = Hn[2, 0] * UT + Hn[2, 1] * VT + Hn[2, 2]
    xt = X / Wh
    yt = Y / Wh
    x = s * xt + c[0]
    y = s * yt + c[1]
    val, dx, dy = bilinear_with_gradient(img, x, y)
    geo = dict(UT=UT, VT=VT, Wh=Wh, xt=xt, yt=yt)
    return val, dx, dy, geo


def coordinate_jacobian(geo, s, model):
    """dx/dtau and dy/dtau (image pixels per unit of tau), each (m, n, p)."""
    UT, VT, Wh, xt, yt = geo["UT"], geo["VT"], geo["Wh"], geo["xt"], geo["yt"]
    p = model
    z = np.zeros_like(UT)
    dxd = [s * UT / Wh, s * VT / Wh, s / Wh, z, z, z]
    dyd = [z, z, z, s * UT / Wh, s * VT / Wh, s / Wh]
    if p == PROJECTIVE:
        dxd += [-s * xt * UT / Wh, -s * xt * VT / Wh]
        dyd += [-s * yt * UT / Wh, -s * yt * VT / Wh]
    return np.stack(dxd, axis=-1), np.stack(dyd, axis=-1)


def raw_jacobian(dx, dy, geo, s, model):
    """d(D o tau)/dtau, arranged as an mn x p matrix (Sec. 4.1)."""
    gx, gy = coordinate_jacobian(geo, s, model)
    Jr = dx[..., None] * gx + dy[..., None] * gy
    m, n = dx.shape
    return Jr.reshape(m * n, model)


def step1(img, Hn, c, s, m, n, model):
    """Alg. 1, Step 1: normalised D o tau (m x n) and the Jacobian of the
    normalised warp, J = J_raw/||I|| - I (I^T J_raw)/||I||^3 (mn x p)."""
    val, dx, dy, geo = warp(img, Hn, c, s, m, n)
    Jr = raw_jacobian(dx, dy, geo, s, model)
    v = val.reshape(-1)
    nrm = float(np.linalg.norm(v))
    if not np.isfinite(nrm) or nrm == 0.0:
        raise FloatingPointError("D o tau has zero or non-finite norm")
    J = Jr / nrm - np.outer(v, v @ Jr) / nrm ** 3
    I = val / nrm
    return I, J, nrm


# ---------------------------------------------------------------------------
# Extra constraints on Delta tau (Sec. 4.3, Eq. add_constraints)
# ---------------------------------------------------------------------------


def corner_coords(m, n, s):
    a = (n - 1) / (2.0 * s)
    b = (m - 1) / (2.0 * s)
    return np.array([[-a, -b], [a, -b], [a, b], [-a, b]])  # TL, TR, BR, BL


def quad_area(Hn, m, n, s):
    """Signed shoelace area of the image of the rectified rectangle
    (normalised units)."""
    pts = []
    for ut, vt in corner_coords(m, n, s):
        w = Hn[2, 0] * ut + Hn[2, 1] * vt + Hn[2, 2]
        pts.append(((Hn[0, 0] * ut + Hn[0, 1] * vt + Hn[0, 2]) / w,
                    (Hn[1, 0] * ut + Hn[1, 1] * vt + Hn[1, 2]) / w))
    area = 0.0
    for k in range(4):
        x1, y1 = pts[k]
        x2, y2 = pts[(k + 1) % 4]
        area += x1 * y2 - x2 * y1
    return 0.5 * area


def area_gradient(Hn, m, n, s, model):
    """d(area)/dtau, written out from the shoelace formula."""
    p = model
    xs, ys, dxs, dys = [], [], [], []
    for ut, vt in corner_coords(m, n, s):
        X = Hn[0, 0] * ut + Hn[0, 1] * vt + Hn[0, 2]
        Y = Hn[1, 0] * ut + Hn[1, 1] * vt + Hn[1, 2]
        w = Hn[2, 0] * ut + Hn[2, 1] * vt + Hn[2, 2]
        xt, yt = X / w, Y / w
        dx = np.zeros(p)
        dy = np.zeros(p)
        dx[0:3] = [ut / w, vt / w, 1.0 / w]
        dy[3:6] = [ut / w, vt / w, 1.0 / w]
        if p == PROJECTIVE:
            dx[6:8] = [-xt * ut / w, -xt * vt / w]
            dy[6:8] = [-yt * ut / w, -yt * vt / w]
        xs.append(xt)
        ys.append(yt)
        dxs.append(dx)
        dys.append(dy)
    g = np.zeros(p)
    for k in range(4):
        k2 = (k + 1) % 4
        g += dxs[k] * ys[k2] + xs[k] * dys[k2] - dxs[k2] * ys[k] - xs[k2] * dys[k]
    return 0.5 * g


def constraint_matrix(Hn, m, n, s, model):
    """Q (3 x p): the image of the rectified centre (translation entries)
    and the area of the image of the rectified rectangle, held fixed to
    first order (reading of Sec. 4.3)."""
    Q = np.zeros((3, model))
    Q[0, 2] = 1.0
    Q[1, 5] = 1.0
    Q[2, :] = area_gradient(Hn, m, n, s, model)
    return Q


def null_basis(Q: np.ndarray) -> np.ndarray:
    """Orthonormal basis (p x p') of null(Q), from the SVD of Q."""
    if Q.shape[0] == 0:
        return np.eye(Q.shape[1])
    _, sv, Vt = np.linalg.svd(Q)
    rank = int(np.sum(sv > 1e-12 * max(1.0, sv[0])))
    return Vt[rank:].T.copy()


# ---------------------------------------------------------------------------
# Proximal maps (Eqs. A_1, S_operator, E_1)
# ---------------------------------------------------------------------------


def soft_threshold(x, eps):
    """T_eps(x) = sgn(x) max(|x| - eps, 0)."""
    return np.sign(x) * np.maximum(np.abs(x) - eps, 0.0)


def svt(W, eps):
    """S_eps(W) = U T_eps(Sigma) V^T with the SVD of W (LAPACK).

    Returns (S_eps(W), singular values of W)."""
    U, sv, Vt = np.linalg.svd(W, full_matrices=False)
    return (U * soft_threshold(sv, eps)) @ Vt, sv


# ---------------------------------------------------------------------------
# J_perp (Eq. Jperpv)
# ---------------------------------------------------------------------------


class Annihilator:
    """J_perp v = v - J ((J^T J)^{-1} (J^T v)) for an mn x p' Jacobian J,
    with the p' x p' Gram matrix formed once (Sec. 4.1)."""

    def __init__(self, J: np.ndarray):
        self.J = np.asarray(J, dtype=np.float64)
        p = self.J.shape[1]
        self.G = self.J.T @ self.J if p else np.zeros((0, 0))
        if p:
            ev = np.linalg.eigvalsh(self.G)
            if not (ev[0] > 1e-14 * max(ev[-1], 1e-300)):
                raise np.linalg.LinAlgError("J^T J is singular")

    def coeffs(self, v: np.ndarray) -> np.ndarray:
        """(J^T J)^{-1} J^T v."""
        if self.J.shape[1] == 0:
            return np.zeros(0)
        return np.linalg.solve(self.G, self.J.T @ v.reshape(-1))

    def __call__(self, v: np.ndarray) -> np.ndarray:
        shape = v.shape
        if self.J.shape[1] == 0:
            return v.copy()
        return (v.reshape(-1) - self.J @ self.coeffs(v)).reshape(shape)


# ---------------------------------------------------------------------------
# Step 2: the inner loop (Sec. 3.2 with the Sec. 4.2 form of the updates)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class InnerResult:
    A: np.ndarray
    E: np.ndarray
    Y: np.ndarray
    iters: int
    mu: float
    cond1: float
    cond2: float
    svt_count: int            # number of singular values of the last M above 1/mu
    sigma_last: np.ndarray    # singular values of the last M


def spectral_norm(X):
    return float(np.linalg.svd(X, compute_uv=False)[0])


def ladmap_inner(I, Jp: Annihilator, lam, A0, E0, Y0, prm: Params, mu0=None, trace=None,
                 svt_op=None) -> InnerResult:
    """LADMAP for min ||A||_* + lam ||E||_1 s.t. J_perp(A + E) = J_perp I.

    Updates (Sec. 4.2):
      M_k     = A_k - J_perp(A_k + E_k - I) - Y_k / mu_k
      A_{k+1} = S_{1/mu_k}(M_k)
      N_k     = E_k - J_perp(A_{k+1} + E_k - I) - Y_k / mu_k
      E_{k+1} = T_{lam/mu_k}(N_k)
      Y_{k+1} = Y_k + mu_k J_perp(A_{k+1} + E_{k+1} - I)
      mu_{k+1}= min(mu_max, rho mu_k), rho = rho0 if the Cond2 quantity < eps2

    ``trace`` (a list, optional) receives one (A_k, E_k, mu_k) tuple per
    iteration and the final (A, E, mu), so tests can check the penalty
    schedule against the iterates; it changes nothing in the iteration.
    ``svt_op`` (optional) replaces the exact SVT: called as svt_op(M, eps, k)
    with k the iteration index, it returns (A, singular values), e.g. the
    SVD with warm start of Sec. 5 (``svdws.SvdwsSvt``).
    """
    A = A0.copy()
    E = E0.copy()
    Y = Jp(Y0)                        # Eq. warm_start_Y
    R = Jp(A + E - I)                 # shared residual J_perp(A + E - I)
    c = float(np.linalg.norm(Jp(I)))  # ||J_perp (D o tau)||_F
    if mu0 is None:
        mu0 = prm.mu0 if prm.mu0 > 0 else 1.25 / spectral_norm(I)
    mu = float(mu0)
    k = 0
    cond1 = cond2 = float("inf")
    sv = np.zeros(0)
    svt_count = 0
    while k < prm.max_inner:
        if trace is not None:
            trace.append((A, E, mu))
        M = A - R - Y / mu
        A1, sv = svt(M, 1.0 / mu) if svt_op is None else svt_op(M, 1.0 / mu, k)
        svt_count = int(np.sum(sv > 1.0 / mu))
        N = E - Jp(A1 + E - I) - Y / mu
        E1 = soft_threshold(N, lam / mu)
        R = Jp(A1 + E1 - I)
        Y = Y + mu * R
        dA = float(np.linalg.norm(A1 - A))
        dE = float(np.linalg.norm(E1 - E))
        A, E = A1, E1
        k += 1
        cond1 = float(np.linalg.norm(R)) / c
        cond2 = mu * max(dA, dE) / c
        if not prm.fixed_iters and cond1 < prm.eps1 and cond2 < prm.eps2:
            break
        if cond2 < prm.eps2:
            mu = min(prm.mu_max, prm.rho0 * mu)
    if trace is not None:
        trace.append((A, E, mu))
    return InnerResult(A, E, Y, k, mu, cond1, cond2, svt_count, sv)


# ---------------------------------------------------------------------------
# Sec. 4.3 W-formulation (cross-check of the null-space elimination)
# ---------------------------------------------------------------------------


def ladmap_inner_w(I, J, Q, lam, A0, E0, Yt0, prm: Params, mu0=None):
    """LADMAP on min ||A||_* + lam||E||_1 s.t. W A + W E = W I with
    W^T W = Id - J (J^T J + Q^T Q)^{-1} J^T (Eq. WTW_property) and the
    Y~ = W^T Y iteration of Eq. newvars2 (N_k starts from E_k)."""
    K = J.T @ J + Q.T @ Q

    def WtW(v):
        return (v.reshape(-1) - J @ np.linalg.solve(K, J.T @ v.reshape(-1))).reshape(v.shape)

    A, E = A0.copy(), E0.copy()
    Yt = WtW(Yt0)                                   # Eq. Y_new_warmstart
    Ri = WtW(A + E - I)
    c = float(np.linalg.norm(WtW(I)))
    mu = float(mu0 if mu0 is not None else (prm.mu0 if prm.mu0 > 0 else 1.25 / spectral_norm(I)))
    k = 0
    while k < prm.max_inner:
        M = A - Yt / mu - Ri
        A1, _ = svt(M, 1.0 / mu)
        N = E - Yt / mu - WtW(A1 + E - I)
        E1 = soft_threshold(N, lam / mu)
        Ri = WtW(A1 + E1 - I)
        Yt = Yt + mu * Ri
        dA = float(np.linalg.norm(A1 - A))
        dE = float(np.linalg.norm(E1 - E))
        A, E = A1, E1
        k += 1
        c1 = float(np.linalg.norm(Ri)) / c
        c2 = mu * max(dA, dE) / c
        if not prm.fixed_iters and c1 < prm.eps1 and c2 < prm.eps2:
            break
        if c2 < prm.eps2:
            mu = min(prm.mu_max, prm.rho0 * mu)
    return A, E, Yt, k


# ---------------------------------------------------------------------------
# Step 3: Delta tau (Eq. Delta_tau with the constraints eliminated)
# ---------------------------------------------------------------------------


def delta_tau(Jp: Annihilator, NQ: np.ndarray, A, E, I):
    """Delta tau = N_Q (J~^T J~)^{-1} J~^T (A + E - I)."""
    return NQ @ Jp.coeffs(A + E - I)


# ---------------------------------------------------------------------------
# Alg. 1: the whole solve
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class SolveResult:
    tau_px: np.ndarray        # 3x3, centred grid px -> image px
    tau_norm: np.ndarray      # 3x3 normalised
    A: np.ndarray
    E: np.ndarray
    Y: np.ndarray
    outer_iters: int
    inner_iters: list
    objective: float
    svt_count: int
    status: int
    history: list


def objective(A, E, lam):
    """||A||_* + lam ||E||_1 (Eq. TILT_2)."""
    return float(np.sum(np.linalg.svd(A, compute_uv=False)) + lam * np.sum(np.abs(E)))


def numerical_rank(A, rel=1e-3):
    sv = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    if sv.size == 0 or sv[0] == 0:
        return 0
    return int(np.sum(sv > rel * sv[0]))


def tilt_solve(image, tau0_px, m, n, model, prm: Optional[Params] = None, lam=None,
               svt_op_factory=None) -> SolveResult:
    """Alg. 1 (TILT via LADMAP+VWS) on one window, in FP64.
    ``svt_op_factory`` (optional): called once per outer iteration, it gives
    the ``svt_op`` of that iteration's inner loop (see ``ladmap_inner``)."""
    prm = prm or Params()
    if model not in (AFFINE, PROJECTIVE):
        raise ValueError("model must be 6 (affine) or 8 (projective)")
    if lam is None:
        lam = prm.lam if prm.lam > 0 else 1.0 / math.sqrt(max(m, n))
    Hn, c, s = normalise_transform(tau0_px, m, n)
    if model == AFFINE:
        Hn[2, :] = [0.0, 0.0, 1.0]
    tau = tau_from_matrix(Hn, model)
    img = np.asarray(image, dtype=np.float64)

    A = E = Y = None
    inner_counts = []
    hist = []
    status = 0
    svt_count = 0
    i = 0
    while i < prm.max_outer:
        Hn = matrix_from_tau(tau, model)
        I, J, _ = step1(img, Hn, c, s, m, n, model)          # Step 1
        if A is None:                                        # initialise
            A = I.copy()
            E = np.zeros_like(I)
            Y = np.zeros_like(I)
        Q = constraint_matrix(Hn, m, n, s, model)
        NQ = null_basis(Q)
        Jt = J @ NQ
        Jp = Annihilator(Jt)
        res = ladmap_inner(I, Jp, lam, A, E, Y, prm,          # Step 2
                           svt_op=svt_op_factory() if svt_op_factory else None)
        A, E, Y = res.A, res.E, res.Y
        svt_count = res.svt_count
        inner_counts.append(res.iters)
        if res.iters >= prm.max_inner and not prm.fixed_iters:
            status = 1
        dtau = delta_tau(Jp, NQ, A, E, I)                    # Step 3
        tau = tau + dtau                                     # Step 4
        i += 1
        f = objective(A, E, lam) if prm.eps_obj > 0 else None
        hist.append(dict(dtau_norm=float(np.linalg.norm(dtau)), inner=res.iters,
                         mu=res.mu, cond1=res.cond1, cond2=res.cond2, objective=f))
        if not np.all(np.isfinite(tau)):
            status = -5
            break
        if not prm.fixed_iters and float(np.linalg.norm(dtau)) < prm.eps_outer:
            break
        # "while not converged" (Alg. 1): the objective of Eq. TILT_2 no
        # longer changes between outer iterations (reading R7)
        if (not prm.fixed_iters and prm.eps_obj > 0 and i > 1
                and abs(f - hist[-2]["objective"]) < prm.eps_obj * hist[-2]["objective"]):
            break
    Hn = matrix_from_tau(tau, model)
    H_px = denormalise_transform(Hn, c, s)
    return SolveResult(
        tau_px=H_px, tau_norm=Hn, A=A, E=E, Y=Y, outer_iters=i, inner_iters=inner_counts,
        objective=objective(A, E, lam), svt_count=svt_count, status=status, history=hist,
    )


def tau_rel_err(H_a, H_b, m, n):
    """||H_a - H_b||_F / ||H_b||_F with both in the normalised coordinates
    of H_b's window."""
    Hb, c, s = normalise_transform(H_b, m, n)
    Ha = np.asarray(H_a, dtype=np.float64)
    Ha = Ha / Ha[2, 2]
    Timg_inv = np.array([[1.0 / s, 0.0, -c[0] / s], [0.0, 1.0 / s, -c[1] / s], [0.0, 0.0, 1.0]])
    Han = Timg_inv @ Ha @ np.diag([s, s, 1.0])
    Han = Han / Han[2, 2]
    return float(np.linalg.norm(Han - Hb) / np.linalg.norm(Hb))
