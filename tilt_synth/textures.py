"""Seeded low-rank textures, warped images and windows.

Every random quantity is drawn from a per-patch PCG64 stream
``Generator(PCG64(SeedSequence([MASTER_SEED + config_index, patch_index])))``
so any single patch of any workload can be regenerated on its own.

Texture model (rank r, separable, defined on the whole plane, in texture
pixel coordinates (u, v) centred on the window):

    T(u, v) = sum_i a_i(u) b_i(v),
    a_i(u)  = (1 + cos(2 pi f_i u / n + phi_i)) / 2,
    b_i(v)  = (1 + cos(2 pi g_i v / m + psi_i)) / 2,

with f_i, g_i uniform in [1, L/8] cycles per window side (pairwise at least
0.5 apart) and uniform phases.  T is divided by its maximum over the m x n
window grid only (a min-max rescale would add a constant, i.e. a rank-one
term).  The image is D(x) = T(G^{-1}(x)), evaluated analytically at every
pixel (no interpolation error), after which a fraction of the pixels, chosen
without replacement, is replaced by uniform (0, 1) values: the
random-corruption model of the paper's robustness experiment (Sec. 6.2,
"Robustness under Corruption"), in grey levels.

Coordinates (shared convention of the solver's interface):
  * image pixel centres sit at integer (x = column, y = row);
  * the rectified grid has rows i = 0..m-1, columns j = 0..n-1 and centred
    coordinates u = j - (n-1)/2, v = i - (m-1)/2;
  * a transform is a 3x3 homography H_px with (x, y, 1) ~ H_px (u, v, 1).

Ground truth: G_norm = [[g * R(theta) [[1, t], [0, 1]], 0], [h7, h8, 1]] in
coordinates scaled by s = max(m, n)/2 about the window centre (the affine
family A(theta, t) of the paper's range-of-convergence experiment, Sec. 6.2,
with a scale g and, for the projective model, a perspective row).
The initial transform tau0 is the axis-aligned window at the image centre.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MASTER_SEED = 120553510

AFFINE = 6
PROJECTIVE = 8


def patch_rng(config_index: int, patch_index: int) -> np.random.Generator:
    """Per-patch random stream (PCG64 seeded by [master + config, patch])."""
    ss = np.random.SeedSequence([MASTER_SEED + int(config_index), int(patch_index)])
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass
class Patch:
    """One rectification problem plus its ground truth."""

    image: np.ndarray          # (H, W) float32, row-major
    m: int                     # rectified rows
    n: int                     # rectified columns
    model: int                 # 6 = affine, 8 = projective
    tau0: np.ndarray           # (3, 3) float64, centred grid px -> image px
    lam: float                 # weight of the l1 term
    G_px: np.ndarray           # (3, 3) float64 ground truth, texture px -> image px
    rank: int
    corruption: float
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def height(self) -> int:
        return int(self.image.shape[0])

    @property
    def width(self) -> int:
        return int(self.image.shape[1])


def _freqs(rng: np.random.Generator, r: int, L: int) -> np.ndarray:
    """r frequencies uniform in [1, hi] cycles, pairwise at least 0.5 apart."""
    hi = max(1.0 + 0.5 * r + 0.5, L / 8.0)
    for _ in range(10000):
        f = rng.uniform(1.0, hi, size=r)
        fs = np.sort(f)
        if r == 1 or np.min(np.diff(fs)) >= 0.5:
            return f
    # Where r separated values barely fit (small windows of high rank) the
    # rejection rarely succeeds; draw from the same law directly: r uniform
    # points in the interval shortened by the r - 1 gaps, sorted, spread by
    # 0.5, in random order.
    span = (hi - 1.0) - 0.5 * (r - 1)
    f = np.sort(rng.uniform(0.0, span, size=r)) + 1.0 + 0.5 * np.arange(r)
    return rng.permutation(f)


def _texture_params(rng: np.random.Generator, r: int, m: int, n: int):
    f = _freqs(rng, r, n)
    g = _freqs(rng, r, m)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=r)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=r)
    return f, g, phi, psi


def _texture(u: np.ndarray, v: np.ndarray, m: int, n: int, params) -> np.ndarray:
    f, g, phi, psi = params
    out = np.zeros(np.broadcast(u, v).shape, dtype=np.float64)
    for i in range(len(f)):
        a = 0.5 * (1.0 + np.cos(2.0 * math.pi * f[i] * u / n + phi[i]))
        b = 0.5 * (1.0 + np.cos(2.0 * math.pi * g[i] * v / m + psi[i]))
        out += a * b
    return out


def _gt_norm(rng, model: int, theta_deg: float, skew: float, scale_rng, persp_px: float, s: float):
    theta = math.radians(rng.uniform(-theta_deg, theta_deg))
    t = rng.uniform(-skew, skew)
    g = rng.uniform(*scale_rng)
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    K = np.array([[1.0, t], [0.0, 1.0]])
    G = np.eye(3)
    G[:2, :2] = g * (R @ K)
    if model == PROJECTIVE:
        G[2, 0] = rng.uniform(-persp_px, persp_px) * s
        G[2, 1] = rng.uniform(-persp_px, persp_px) * s
    return G, dict(theta=theta, skew=t, scale=g)


def make_patch(
    rng: np.random.Generator,
    *,
    m: int,
    n: int,
    height: int,
    width: int,
    rank: int,
    model: int,
    corruption: float,
    lam: Optional[float] = None,
    theta_deg: float = 20.0,
    skew: float = 0.2,
    scale_rng=(0.9, 1.1),
    persp_px: float = 1e-3,
    center=None,
) -> Patch:
    """Draw one patch: texture, ground truth, warped + corrupted image."""
    s = max(m, n) / 2.0
    if center is None:
        cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    else:
        cx, cy = float(center[0]), float(center[1])
    params = _texture_params(rng, rank, m, n)
    G, meta = _gt_norm(rng, model, theta_deg, skew, scale_rng, persp_px, s)

    # normalisation over the window grid (rectified texture frame)
    jj, ii = np.meshgrid(np.arange(n), np.arange(m))
    u = jj - (n - 1) / 2.0
    v = ii - (m - 1) / 2.0
    tmax = float(np.max(_texture(u, v, m, n, params)))

    # image D(x) = T(G^{-1}(x)) at every pixel
    xs, ys = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    xt = (xs - cx) / s
    yt = (ys - cy) / s
    Gi = np.linalg.inv(G)
    X = Gi[0, 0] * xt + Gi[0, 1] * yt + Gi[0, 2]
    Y = Gi[1, 0] * xt + Gi[1, 1] * yt + Gi[1, 2]
    W = Gi[2, 0] * xt + Gi[2, 1] * yt + Gi[2, 2]
    img = _texture(s * X / W, s * Y / W, m, n, params) / tmax

    npx = height * width
    k = int(round(corruption * npx))
    if k > 0:
        idx = rng.choice(npx, size=k, replace=False)
        flat = img.reshape(-1)
        flat[idx] = rng.uniform(0.0, 1.0, size=k)

    tau0 = np.array([[1.0, 0.0, cx], [0.0, 1.0, cy], [0.0, 0.0, 1.0]])
    Timg = np.array([[s, 0.0, cx], [0.0, s, cy], [0.0, 0.0, 1.0]])
    Sg_inv = np.diag([1.0 / s, 1.0 / s, 1.0])
    G_px = Timg @ G @ Sg_inv
    if lam is None:
        lam = 1.0 / math.sqrt(max(m, n))
    meta.update(G_norm=G, texture=params, center=(cx, cy))
    return Patch(
        image=np.ascontiguousarray(img, dtype=np.float32),
        m=int(m), n=int(n), model=int(model), tau0=tau0, lam=float(lam),
        G_px=G_px, rank=int(rank), corruption=float(corruption), meta=meta,
    )


# ---------------------------------------------------------------------------
# Workloads.  Index k matches the k-th workload description:
#   0  single 50x50 affine patch in a 200x200 image (oracle-sized)
#   1  256 projective 100x100 patches in 400x400 images
#   2  1024 uneven patches, sides 32..256, 50/50 affine/projective
#   3  512 projective 128x128 patches in 256x256 images
#   4  serving requests on 640x480 images, lognormal sides in [40, 400]
# ---------------------------------------------------------------------------

_CONFIGS = {
    0: "single-50x50-affine",
    1: "batch-256x100x100-projective",
    2: "uneven-1024-32to256-mixed",
    3: "batch-512x128x128-projective",
    4: "serving-640x480-lognormal",
}


def config_names():
    return dict(_CONFIGS)


def _config_patch(config_index: int, i: int) -> Patch:
    rng = patch_rng(config_index, i)
    if config_index == 0:
        return make_patch(rng, m=50, n=50, height=200, width=200, rank=3,
                          model=AFFINE, corruption=0.10, lam=1.0 / math.sqrt(50))
    if config_index == 1:
        r = int(rng.integers(2, 6))
        return make_patch(rng, m=100, n=100, height=400, width=400, rank=r,
                          model=PROJECTIVE, corruption=0.20, lam=0.1)
    if config_index == 2:
        m = int(rng.integers(32, 257))
        n = int(rng.integers(32, 257))
        r = int(rng.integers(1, 9))
        model = AFFINE if rng.uniform() < 0.5 else PROJECTIVE
        corr = float(rng.uniform(0.05, 0.30))
        side = 2 * max(m, n)
        return make_patch(rng, m=m, n=n, height=side, width=side, rank=r,
                          model=model, corruption=corr)
    if config_index == 3:
        return make_patch(rng, m=128, n=128, height=256, width=256, rank=4,
                          model=PROJECTIVE, corruption=0.15)
    if config_index == 4:
        m = int(np.clip(round(math.exp(rng.normal(math.log(100.0), 0.5))), 40, 400))
        n = int(np.clip(round(math.exp(rng.normal(math.log(100.0), 0.5))), 40, 400))
        m = min(m, 400)
        n = min(n, 400)
        r = int(rng.integers(1, 7))
        model = AFFINE if rng.uniform() < 0.5 else PROJECTIVE
        corr = float(rng.uniform(0.0, 0.30))
        H, W = 480, 640
        # centre drawn so that the axis-aligned window fits in the image
        cx = rng.uniform((n - 1) / 2.0, W - 1 - (n - 1) / 2.0)
        cy = rng.uniform((m - 1) / 2.0, H - 1 - (m - 1) / 2.0)
        return make_patch(rng, m=m, n=n, height=H, width=W, rank=r, model=model,
                          corruption=corr, center=(cx, cy))
    raise ValueError(f"unknown workload index {config_index}")


def make_config(config_index: int, count: Optional[int] = None, start: int = 0) -> List[Patch]:
    """Patches ``start .. start+count-1`` of workload ``config_index``."""
    default = {0: 1, 1: 256, 2: 1024, 3: 512, 4: 256}[config_index]
    if count is None:
        count = default - start
    return [_config_patch(config_index, start + i) for i in range(count)]


def make_batch(config_index: int, indices) -> List[Patch]:
    return [_config_patch(config_index, int(i)) for i in indices]


def inner_problem(index: int, m: int, n: int, p: int = 5):
    """Inputs of the inner-loop-only workload (the setting of Table 1, whose
    distributions the paper does not state): I ~ U(0, 1) entries (m x n) and
    J with N(0, 1) entries (p planes of m x n), float32, seeded by the
    workload index 5 and `index`."""
    rng = patch_rng(5, index * 100003 + m * 1009 + n * 13 + p)
    I = rng.uniform(0.0, 1.0, (m, n)).astype(np.float32)
    J = rng.standard_normal((p, m, n)).astype(np.float32)
    return I, J


def checkerboard_patch(theta: float, skew: float, m: int = 60, n: int = 60, size: int = 200,
                       period: float = 10.0, edge: float = 0.3) -> Patch:
    """Soft-edged checkerboard window deformed by the affine
    A(theta, t) = R(theta) [[1, t], [0, 1]] about the image centre (the
    deformation family of the range-of-convergence experiment, Sec. 6.2).
    Texture T(u, v) = (1 + q(u) q(v)) / 2 with q(x) = tanh(sin(pi x / period)
    / edge): exactly rank two, squares of `period` pixels, edges about one
    pixel wide.  No corruption; tau0 is the axis-aligned window at the image
    centre."""
    def q(x):
        return np.tanh(np.sin(math.pi * x / period) / edge)

    s = max(m, n) / 2.0
    cx = cy = (size - 1) / 2.0
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    K = np.array([[1.0, skew], [0.0, 1.0]])
    G = np.eye(3)
    G[:2, :2] = R @ K
    Gi = np.linalg.inv(G)
    xs, ys = np.meshgrid(np.arange(size, dtype=np.float64), np.arange(size, dtype=np.float64))
    xt, yt = (xs - cx) / s, (ys - cy) / s
    U = s * (Gi[0, 0] * xt + Gi[0, 1] * yt)
    V = s * (Gi[1, 0] * xt + Gi[1, 1] * yt)
    img = 0.5 * (1.0 + q(U) * q(V))
    tau0 = np.array([[1.0, 0.0, cx], [0.0, 1.0, cy], [0.0, 0.0, 1.0]])
    Timg = np.array([[s, 0.0, cx], [0.0, s, cy], [0.0, 0.0, 1.0]])
    G_px = Timg @ G @ np.diag([1.0 / s, 1.0 / s, 1.0])
    return Patch(image=np.ascontiguousarray(img, dtype=np.float32), m=m, n=n, model=AFFINE, tau0=tau0,
                 lam=1.0 / math.sqrt(max(m, n)), G_px=G_px, rank=2, corruption=0.0,
                 meta=dict(G_norm=G, theta=theta, skew=skew, center=(cx, cy)))


def convergence_grid():
    """(theta, t) of the range-of-convergence sweep: theta in [0, pi/6] in
    steps of pi/60, t in [0, 1] in steps of 0.05 (11 x 21 cases)."""
    return [(k * math.pi / 60.0, j * 0.05) for k in range(11) for j in range(21)]


# ---------------------------------------------------------------------------
# RASL sets: several images of one scene, each moved by its own small
# planted transform; the data matrix holds one window per column.
# ---------------------------------------------------------------------------

RASL_SEED_OFFSET = 1000


@dataclasses.dataclass
class RaslSet:
    """N images of one texture, image k = T(G_k^{-1}(x)) plus corruption."""

    images: np.ndarray        # (N, H, W) float32
    m: int
    n: int
    model: int
    tau0: np.ndarray          # (N, 3, 3): centred grid px -> image px (all the same window)
    lam: float
    G_px: np.ndarray          # (N, 3, 3): planted transform, texture px -> image px
    corruption: float

    @property
    def count(self) -> int:
        return int(self.images.shape[0])

    @property
    def height(self) -> int:
        return int(self.images.shape[1])

    @property
    def width(self) -> int:
        return int(self.images.shape[2])


def rasl_set(index: int, count: int = 16, m: int = 20, n: int = 24, height: int = 48, width: int = 56,
             rank: int = 2, model: int = AFFINE, corruption: float = 0.05, shift_px: float = 1.5,
             theta_deg: float = 2.0, scale_rng=(0.98, 1.02), lam: Optional[float] = None) -> RaslSet:
    """Draw one RASL set.  The texture is the separable low-rank model above
    (its parameters drawn for an m x n window); image k is that texture seen
    through G_k = translation by U(-shift_px, shift_px) per axis after a
    rotation U(-theta_deg, theta_deg) and a scale U(scale_rng), all about the
    image centre.  tau0 is the axis-aligned window at the image centre for
    every image; lambda defaults to 1/sqrt(max(m n, N))."""
    rng = patch_rng(RASL_SEED_OFFSET + int(index), 0)
    s = max(m, n) / 2.0
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    params = _texture_params(rng, rank, m, n)
    jj, ii = np.meshgrid(np.arange(n), np.arange(m))
    tmax = float(np.max(_texture(jj - (n - 1) / 2.0, ii - (m - 1) / 2.0, m, n, params)))
    xs, ys = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    imgs = np.zeros((count, height, width), np.float32)
    G_all = np.zeros((count, 3, 3))
    for k in range(count):
        th = math.radians(rng.uniform(-theta_deg, theta_deg))
        g = rng.uniform(*scale_rng)
        dx, dy = rng.uniform(-shift_px, shift_px, size=2)
        G = np.array([[g * math.cos(th), -g * math.sin(th), cx + dx],
                      [g * math.sin(th), g * math.cos(th), cy + dy],
                      [0.0, 0.0, 1.0]])
        Gi = np.linalg.inv(G)
        u = Gi[0, 0] * xs + Gi[0, 1] * ys + Gi[0, 2]
        v = Gi[1, 0] * xs + Gi[1, 1] * ys + Gi[1, 2]
        img = _texture(u, v, m, n, params) / tmax
        npx = height * width
        c = int(round(corruption * npx))
        if c > 0:
            idx = rng.choice(npx, size=c, replace=False)
            flat = img.reshape(-1)
            flat[idx] = rng.uniform(0.0, 1.0, size=c)
        imgs[k] = img
        G_all[k] = G
    tau0 = np.tile(np.array([[1.0, 0.0, cx], [0.0, 1.0, cy], [0.0, 0.0, 1.0]]), (count, 1, 1))
    if lam is None:
        lam = 1.0 / math.sqrt(max(m * n, count))
    return RaslSet(images=imgs, m=int(m), n=int(n), model=int(model), tau0=tau0, lam=float(lam),
                   G_px=G_all, corruption=float(corruption))
