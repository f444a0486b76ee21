"""ctypes binding of ``libtilt.so`` (the C interface in ``include/tilt.h``).

Argument marshalling only: every step of the solve runs in the HIP library.
Device buffers are passed as raw pointers, typically from PyTorch tensors on
``cuda:N`` (PyTorch is used for device memory and streams only).  If the
library is missing, importing this module raises: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TILT_LIB", os.path.join(_PKG_DIR, "libtilt.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"HIP library not found at {LIB_PATH}; build it with "
        "`python paper_1205_5351_amd/build.py` (or __graft_entry__.build())"
    )

try:
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading
    # it first makes libtilt.so bind to that same runtime, so device memory
    # and streams from torch are valid in the library.
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for host-only use
    torch = None

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------------------
# Status codes and models (mirror of the header)
# ---------------------------------------------------------------------------
TILT_OK = 0
TILT_WARN_MAXITER = 1
TILT_PENDING = 2
TILT_ERR_ARG = -1
TILT_ERR_NOMEM = -2
TILT_ERR_DEVICE = -3
TILT_ERR_SINGULAR = -4
TILT_ERR_NONFINITE = -5
TILT_ERR_TOO_LARGE = -6
TILT_ERR_NOT_FOUND = -7
TILT_SVT_NOALLOC_BYTES = 64 << 20  # fixed working array of tilt_svt_batch_noalloc, per GPU

AFFINE = 6
PROJECTIVE = 8


class TiltError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        detail = last_error() if code == TILT_ERR_DEVICE else ""
        super().__init__(f"{what}: {status_string(code)} ({code}){' ' + detail if detail else ''}")


class Params(C.Structure):
    _fields_ = [
        ("lambda_", C.c_double),
        ("eps1", C.c_double),
        ("eps2", C.c_double),
        ("eps_outer", C.c_double),
        ("mu0", C.c_double),
        ("rho0", C.c_double),
        ("mu_max", C.c_double),
        ("max_inner", C.c_int),
        ("max_outer", C.c_int),
        ("fixed_iters", C.c_int),
        ("svt_mode", C.c_int),
        ("jacobi_tol", C.c_float),
        ("max_sweeps", C.c_int),
        ("pyramid_levels", C.c_int),
        ("graph_inner", C.c_int),
        ("eps_obj", C.c_double),
        ("eps_svd", C.c_double),
        ("svdws_every", C.c_int),
        ("reserved_params", C.c_int),
    ]


class Problem(C.Structure):
    _fields_ = [
        ("image", C.c_void_p),
        ("height", C.c_int),
        ("width", C.c_int),
        ("row_stride", C.c_longlong),
        ("m", C.c_int),
        ("n", C.c_int),
        ("model", C.c_int),
        ("init", C.c_int),
        ("tau0", C.c_double * 9),
        ("quad", C.c_double * 8),
    ]


class Counters(C.Structure):
    _fields_ = [
        ("inner_iters", C.c_longlong),
        ("svt_calls", C.c_longlong),
        ("jacobi_sweeps", C.c_longlong),
        ("jacobi_pairs", C.c_longlong),
        ("jacobi_rotations", C.c_longlong),
        ("recon_rows", C.c_longlong),
        ("svdws_steps", C.c_longlong),
    ]


class Result(C.Structure):
    _fields_ = [
        ("tau", C.c_double * 9),
        ("A", C.c_void_p),
        ("E", C.c_void_p),
        ("outer_iters", C.c_int),
        ("inner_iters_total", C.c_int),
        ("svt_rank", C.c_int),
        ("status", C.c_int),
        ("rank", C.c_int),
        ("reserved", C.c_int),
        ("objective", C.c_double),
        ("mu", C.c_double),
        ("cond1", C.c_double),
        ("cond2", C.c_double),
        ("dtau_norm", C.c_double),
        ("solve_ms", C.c_double),
        ("done_ms", C.c_double),
        ("counters", Counters),
    ]


class RaslProblem(C.Structure):
    _fields_ = [
        ("images", C.c_void_p),
        ("image_stride", C.c_longlong),
        ("height", C.c_int),
        ("width", C.c_int),
        ("row_stride", C.c_longlong),
        ("count", C.c_int),
        ("m", C.c_int),
        ("n", C.c_int),
        ("model", C.c_int),
        ("tau0", C.POINTER(C.c_double)),
    ]


class RaslResult(C.Structure):
    _fields_ = [
        ("tau", C.POINTER(C.c_double)),
        ("A", C.c_void_p),
        ("E", C.c_void_p),
        ("objective", C.c_double),
        ("outer_iters", C.c_int),
        ("inner_iters_total", C.c_int),
        ("svt_rank", C.c_int),
        ("status", C.c_int),
        ("solve_ms", C.c_double),
        ("counters", Counters),
    ]


_lib.tilt_default_params.argtypes = [C.POINTER(Params)]
_lib.tilt_default_params.restype = None
_lib.tilt_status_string.argtypes = [C.c_int]
_lib.tilt_status_string.restype = C.c_char_p
_lib.tilt_version.argtypes = []
_lib.tilt_version.restype = C.c_char_p
_lib.tilt_last_error.argtypes = []
_lib.tilt_last_error.restype = C.c_char_p
_lib.tilt_tau_from_quad.argtypes = [C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]
_lib.tilt_tau_from_quad.restype = C.c_int
_lib.tilt_solve.argtypes = [C.POINTER(Problem), C.POINTER(Params), C.POINTER(Result)]
_lib.tilt_solve.restype = C.c_int
_lib.tilt_ctx_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_size_t]
_lib.tilt_ctx_create.restype = C.c_int
_lib.tilt_ctx_destroy.argtypes = [C.c_void_p]
_lib.tilt_ctx_destroy.restype = C.c_int
_lib.tilt_ctx_last_kernel_ms.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
_lib.tilt_ctx_last_kernel_ms.restype = C.c_int
_lib.tilt_ctx_progress.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
_lib.tilt_ctx_progress.restype = C.c_int
_lib.tilt_workspace_bytes.argtypes = [C.POINTER(Problem)]
_lib.tilt_workspace_bytes.restype = C.c_size_t
_lib.tilt_solve_batch.argtypes = [C.c_void_p, C.POINTER(Problem), C.c_int, C.POINTER(Params),
                                  C.POINTER(Result), C.c_void_p]
_lib.tilt_solve_batch.restype = C.c_int
_lib.tilt_solve_batch_plain.argtypes = _lib.tilt_solve_batch.argtypes
_lib.tilt_solve_batch_plain.restype = C.c_int
_lib.tilt_svt_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                C.POINTER(C.c_float), C.POINTER(Params), C.POINTER(C.c_int),
                                C.POINTER(Counters), C.c_void_p]
_lib.tilt_svt_batch.restype = C.c_int
_lib.tilt_svt_batch_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                        C.POINTER(C.c_float), C.POINTER(Params), C.POINTER(C.c_int),
                                        C.POINTER(Counters), C.c_void_p]
_lib.tilt_svt_batch_noalloc.restype = C.c_int
_lib.tilt_svdws_batch.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int] + [C.c_void_p] * 8 + [
    C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
    C.POINTER(C.c_int), C.c_void_p]
_lib.tilt_svdws_batch.restype = C.c_int
_lib.tilt_warp_jacobian.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(C.c_double), C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
_lib.tilt_warp_jacobian.restype = C.c_int
_lib.tilt_submit.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Params), C.c_void_p, C.c_void_p,
                             C.POINTER(C.c_ulonglong)]
_lib.tilt_submit.restype = C.c_int
_lib.tilt_poll.argtypes = [C.c_void_p, C.c_ulonglong, C.POINTER(Result)]
_lib.tilt_poll.restype = C.c_int
_lib.tilt_serve_stop.argtypes = [C.c_void_p]
_lib.tilt_serve_stop.restype = C.c_int
_lib.tilt_pyramid.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_longlong, C.c_void_p, C.c_int,
                              C.c_void_p]
_lib.tilt_pyramid.restype = C.c_int
_lib.tilt_inner_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                  C.POINTER(Params), C.c_void_p, C.c_void_p, C.POINTER(Result), C.c_void_p]
_lib.tilt_inner_batch.restype = C.c_int
_lib.tilt_svt_layouts.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int]
_lib.tilt_svt_layouts.restype = C.c_int
_lib.tilt_tune_set.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
_lib.tilt_tune_set.restype = C.c_int
_lib.tilt_svt_layout.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int)]
_lib.tilt_svt_layout.restype = C.c_int
_lib.tilt_peak_probe.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_void_p]
_lib.tilt_peak_probe.restype = C.c_int
_lib.tilt_tune_clear.argtypes = []
_lib.tilt_tune_clear.restype = C.c_int
_lib.tilt_rasl_solve_batch.argtypes = [C.c_void_p, C.POINTER(RaslProblem), C.c_int, C.POINTER(Params),
                                       C.POINTER(RaslResult), C.c_void_p]
_lib.tilt_rasl_solve_batch.restype = C.c_int

EXPORTS = [
    "tilt_default_params", "tilt_status_string", "tilt_version", "tilt_tau_from_quad", "tilt_solve",
    "tilt_ctx_create", "tilt_ctx_destroy", "tilt_workspace_bytes", "tilt_solve_batch",
    "tilt_solve_batch_plain", "tilt_svt_batch", "tilt_svt_batch_noalloc", "tilt_svdws_batch", "tilt_warp_jacobian", "tilt_last_error",
    "tilt_ctx_last_kernel_ms", "tilt_ctx_progress", "tilt_submit", "tilt_poll", "tilt_serve_stop", "tilt_pyramid",
    "tilt_inner_batch", "tilt_svt_layouts", "tilt_svt_layout", "tilt_tune_set", "tilt_tune_clear",
    "tilt_rasl_solve_batch", "tilt_peak_probe",
]


def library():
    return _lib


def svt_layouts(m: int, n: int):
    """Valid (rows per block, lanes per pair) layouts of the LDS Jacobi for m x n."""
    bs = (C.c_int * 8)()
    lpp = (C.c_int * 8)()
    k = _lib.tilt_svt_layouts(int(m), int(n), bs, lpp, 8)
    return [(bs[i], lpp[i]) for i in range(min(k, 8))]


PEAK_HBM_COPY, PEAK_LDS_READ, PEAK_FP32_FMA, PEAK_FP32_MFMA = 0, 1, 2, 3


def peak_probe(kind: int, src_ptr: int, dst_ptr: int, nbytes: int, iters: int = 1, stream=None):
    """Run one machine-peak probe kernel; returns (ms, work) with work in
    bytes (kinds 0, 1) or flops (kinds 2, 3)."""
    ms = C.c_double()
    work = C.c_double()
    rc = _lib.tilt_peak_probe(int(kind), C.c_void_p(src_ptr or None), C.c_void_p(dst_ptr), C.c_size_t(nbytes),
                              int(iters), C.byref(ms), C.byref(work), C.c_void_p(_stream_ptr(stream)))
    if rc != TILT_OK:
        raise TiltError(rc, "tilt_peak_probe")
    return ms.value, work.value


def svt_layout(m: int, n: int):
    """Layout the SVT of an m x n window runs with now: (rows per block,
    lanes per pair, float4 chunks per lane, single floats per lane, tiled)."""
    out = (C.c_int * 5)()
    rc = _lib.tilt_svt_layout(int(m), int(n), out)
    if rc != TILT_OK:
        raise TiltError(rc, "tilt_svt_layout")
    return tuple(out[i] for i in range(5))


def tune_set(m: int, n: int, bs: int, lpp: int):
    rc = _lib.tilt_tune_set(int(m), int(n), int(bs), int(lpp))
    if rc != TILT_OK:
        raise TiltError(rc, "tilt_tune_set")


def tune_clear():
    _lib.tilt_tune_clear()


def load_tuning(path: str) -> int:
    """Apply a table written by autotune.py; returns the number of entries."""
    import json

    with open(path) as f:
        table = json.load(f)
    for e in table["entries"]:
        tune_set(e["m"], e["n"], e["bs"], e["lpp"])
    return len(table["entries"])


def status_string(code: int) -> str:
    return _lib.tilt_status_string(int(code)).decode()


def version() -> str:
    return _lib.tilt_version().decode()


def last_error() -> str:
    return _lib.tilt_last_error().decode()


def default_params(**overrides) -> Params:
    p = Params()
    _lib.tilt_default_params(C.byref(p))
    for k, v in overrides.items():
        key = "lambda_" if k in ("lam", "lambda") else k
        if not hasattr(p, key):
            raise KeyError(k)
        setattr(p, key, v)
    return p


def tau_from_quad(quad: Sequence[float], m: int, n: int, model: int) -> np.ndarray:
    q = (C.c_double * 8)(*[float(x) for x in quad])
    out = (C.c_double * 9)()
    rc = _lib.tilt_tau_from_quad(q, int(m), int(n), int(model), out)
    if rc != TILT_OK:
        raise TiltError(rc, "tilt_tau_from_quad")
    return np.array(list(out)).reshape(3, 3)


def make_problem(image_ptr: int, height: int, width: int, row_stride: int, m: int, n: int, model: int,
                 tau0=None, quad=None) -> Problem:
    """One window: start from the pixel homography tau0, or (quad given,
    tau0 None) from the map of the grid onto quad = TL, TR, BR, BL (x, y)."""
    if (tau0 is None) == (quad is None):
        raise ValueError("give exactly one of tau0 and quad")
    pr = Problem()
    pr.image = C.c_void_p(int(image_ptr))
    pr.height = int(height)
    pr.width = int(width)
    pr.row_stride = int(row_stride)
    pr.m = int(m)
    pr.n = int(n)
    pr.model = int(model)
    if quad is not None:
        pr.init = 1
        q = np.asarray(quad, dtype=np.float64).reshape(8)
        for k in range(8):
            pr.quad[k] = float(q[k])
    else:
        pr.init = 0
        t = np.asarray(tau0, dtype=np.float64).reshape(9)
        for k in range(9):
            pr.tau0[k] = float(t[k])
    return pr


def workspace_bytes(m: int, n: int, model: int = PROJECTIVE) -> int:
    pr = make_problem(1, 2, 2, 2, m, n, model, np.eye(3))
    return int(_lib.tilt_workspace_bytes(C.byref(pr)))


def result_dict(r: Result) -> dict:
    c = r.counters
    return dict(
        tau=np.array(list(r.tau)).reshape(3, 3),
        outer_iters=r.outer_iters,
        inner_iters_total=r.inner_iters_total,
        svt_rank=r.svt_rank,
        rank=r.rank,
        status=r.status,
        objective=r.objective,
        mu=r.mu,
        cond1=r.cond1,
        cond2=r.cond2,
        dtau_norm=r.dtau_norm,
        solve_ms=r.solve_ms,
        done_ms=r.done_ms,
        counters=dict(inner_iters=c.inner_iters, svt_calls=c.svt_calls, jacobi_sweeps=c.jacobi_sweeps,
                      jacobi_pairs=c.jacobi_pairs, jacobi_rotations=c.jacobi_rotations,
                      recon_rows=c.recon_rows, svdws_steps=c.svdws_steps),
    )


def solve(image: np.ndarray, tau0, m: int, n: int, model: int, params: Optional[Params] = None,
          want_AE: bool = True) -> dict:
    """Plain single-patch path (``tilt_solve``): host arrays in and out."""
    img = np.ascontiguousarray(image, dtype=np.float32)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    prm = params if params is not None else default_params()
    pr = make_problem(img.ctypes.data, img.shape[0], img.shape[1], img.shape[1], m, n, model, tau0)
    res = Result()
    A = E = None
    if want_AE:
        A = np.zeros((m, n), np.float32)
        E = np.zeros((m, n), np.float32)
        res.A = C.c_void_p(A.ctypes.data)
        res.E = C.c_void_p(E.ctypes.data)
    rc = _lib.tilt_solve(C.byref(pr), C.byref(prm), C.byref(res))
    if rc < 0 and rc not in (TILT_ERR_SINGULAR, TILT_ERR_NONFINITE):
        raise TiltError(rc, "tilt_solve")
    out = result_dict(res)
    out["A"] = A
    out["E"] = E
    out["rc"] = rc
    return out


def svt_batch_noalloc(M_ptr: int, A_ptr: int, sigma_ptr: int, count: int, m: int, n: int, eps,
                      params: Optional[Params] = None, stream=None):
    """tilt_svt_batch_noalloc: the SVT of `count` m x n matrices (DEVICE
    pointers) on the current device, working memory from the library's fixed
    array (no device allocation).  Returns (ranks, counters)."""
    prm = params if params is not None else default_params()
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (count,)))
    earr = (C.c_float * count)(*e.tolist())
    ranks = (C.c_int * count)()
    cnt = Counters()
    rc = _lib.tilt_svt_batch_noalloc(C.c_void_p(int(M_ptr)), C.c_void_p(int(A_ptr)),
                                     C.c_void_p(int(sigma_ptr)) if sigma_ptr else None, int(count), int(m), int(n),
                                     earr, C.byref(prm), ranks, C.byref(cnt), C.c_void_p(_stream_ptr(stream)))
    if rc != TILT_OK:
        raise TiltError(rc, "tilt_svt_batch_noalloc")
    return list(ranks), dict(svt_calls=cnt.svt_calls, jacobi_sweeps=cnt.jacobi_sweeps,
                             jacobi_pairs=cnt.jacobi_pairs, jacobi_rotations=cnt.jacobi_rotations,
                             recon_rows=cnt.recon_rows)


def _stream_ptr(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Context:
    """Owns the device workspace of batched solves on one GPU."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = C.c_void_p()
        rc = _lib.tilt_ctx_create(C.byref(h), int(device), C.c_size_t(int(budget_bytes)))
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_ctx_create")
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            _lib.tilt_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _batch(self, fn, problems: List[Problem], params: Optional[Params], outs_A, outs_E, stream):
        n = len(problems)
        prm = params if params is not None else default_params()
        parr = (Problem * n)(*problems)
        rarr = (Result * n)()
        for i in range(n):
            rarr[i].A = C.c_void_p(int(outs_A[i])) if outs_A is not None and outs_A[i] else None
            rarr[i].E = C.c_void_p(int(outs_E[i])) if outs_E is not None and outs_E[i] else None
        rc = fn(self._h, parr, n, C.byref(prm), rarr, C.c_void_p(_stream_ptr(stream)))
        if rc < 0 and rc not in (TILT_ERR_SINGULAR, TILT_ERR_NONFINITE, TILT_ERR_TOO_LARGE, TILT_ERR_ARG):
            raise TiltError(rc, fn.__name__)
        return rc, [result_dict(rarr[i]) for i in range(n)]

    def last_kernel_ms(self) -> float:
        ms = C.c_double()
        _lib.tilt_ctx_last_kernel_ms(self._h, C.byref(ms))
        return ms.value

    def progress(self):
        """(finished, total) requests of the fused launch in flight, (0, 0) if none."""
        f, t = C.c_int(), C.c_int()
        rc = _lib.tilt_ctx_progress(self._h, C.byref(f), C.byref(t))
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_ctx_progress")
        return f.value, t.value

    def svdws_batch(self, count: int, m: int, n: int, U_ptr: int, S_ptr: int, V_ptr: int, M_ptr: int,
                    U_out: int, S_out: int, V_out: int, A_out: int = 0, eps=None, stream=None):
        """One warm-start Cayley step per matrix (tilt_svdws_batch), DEVICE
        pointers.  Returns (rc, t, f0, ft, status) with the per-matrix arrays
        as numpy arrays."""
        t = (C.c_double * count)()
        f0 = (C.c_double * count)()
        ft = (C.c_double * count)()
        st = (C.c_int * count)()
        earr = None
        if A_out:
            e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (count,)))
            earr = (C.c_float * count)(*e.tolist())
        ptrs = [C.c_void_p(int(x)) if x else None for x in (U_ptr, S_ptr, V_ptr, M_ptr, U_out, S_out, V_out, A_out)]
        rc = _lib.tilt_svdws_batch(self._h, int(count), int(m), int(n), *ptrs, earr, t, f0, ft, st,
                                   C.c_void_p(_stream_ptr(stream)))
        if rc < 0:
            raise TiltError(rc, "tilt_svdws_batch")
        return rc, np.array(list(t)), np.array(list(f0)), np.array(list(ft)), np.array(list(st))

    def solve_batch(self, problems, params=None, outs_A=None, outs_E=None, stream=None):
        """Fused persistent kernel over all problems (device images/outputs)."""
        return self._batch(_lib.tilt_solve_batch, problems, params, outs_A, outs_E, stream)

    def solve_batch_plain(self, problems, params=None, outs_A=None, outs_E=None, stream=None):
        """Step-by-step kernels, one patch after another (device images/outputs)."""
        return self._batch(_lib.tilt_solve_batch_plain, problems, params, outs_A, outs_E, stream)

    def svt_batch(self, M_ptr: int, A_ptr: int, sigma_ptr: int, count: int, m: int, n: int, eps,
                  params: Optional[Params] = None, stream=None):
        prm = params if params is not None else default_params()
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (count,)))
        earr = (C.c_float * count)(*e.tolist())
        ranks = (C.c_int * count)()
        cnt = Counters()
        rc = _lib.tilt_svt_batch(self._h, C.c_void_p(int(M_ptr)), C.c_void_p(int(A_ptr)),
                                 C.c_void_p(int(sigma_ptr)) if sigma_ptr else None, int(count), int(m), int(n),
                                 earr, C.byref(prm), ranks, C.byref(cnt), C.c_void_p(_stream_ptr(stream)))
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_svt_batch")
        return list(ranks), dict(svt_calls=cnt.svt_calls, jacobi_sweeps=cnt.jacobi_sweeps,
                                 jacobi_pairs=cnt.jacobi_pairs, jacobi_rotations=cnt.jacobi_rotations,
                                 recon_rows=cnt.recon_rows)

    # -- serving ---------------------------------------------------------
    def submit(self, problem: Problem, params: Optional[Params] = None, A_ptr: int = 0, E_ptr: int = 0) -> int:
        """Queue one problem (device image, device A/E or 0); returns its ticket."""
        prm = params if params is not None else default_params()
        t = C.c_ulonglong()
        rc = _lib.tilt_submit(self._h, C.byref(problem), C.byref(prm), C.c_void_p(int(A_ptr)) if A_ptr else None,
                              C.c_void_p(int(E_ptr)) if E_ptr else None, C.byref(t))
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_submit")
        return int(t.value)

    def poll(self, ticket: int):
        """None while pending, else (status, result dict)."""
        r = Result()
        rc = _lib.tilt_poll(self._h, C.c_ulonglong(int(ticket)), C.byref(r))
        if rc == TILT_PENDING:
            return None
        if rc in (TILT_ERR_NOT_FOUND, TILT_ERR_DEVICE, TILT_ERR_ARG):
            raise TiltError(rc, "tilt_poll")
        return rc, result_dict(r)

    def serve_stop(self):
        rc = _lib.tilt_serve_stop(self._h)
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_serve_stop")

    def inner_batch(self, I_ptr: int, J_ptr: int, count: int, m: int, n: int, p: int,
                    params: Optional[Params] = None, A_ptr: int = 0, E_ptr: int = 0, stream=None):
        """LADMAP inner loop alone on given I (count x m x n) and J (count x p x m x n)."""
        prm = params if params is not None else default_params()
        rarr = (Result * count)()
        rc = _lib.tilt_inner_batch(self._h, C.c_void_p(int(I_ptr)), C.c_void_p(int(J_ptr)), int(count), int(m),
                                   int(n), int(p), C.byref(prm), C.c_void_p(int(A_ptr)) if A_ptr else None,
                                   C.c_void_p(int(E_ptr)) if E_ptr else None, rarr,
                                   C.c_void_p(_stream_ptr(stream)))
        if rc < 0 and rc not in (TILT_ERR_SINGULAR, TILT_ERR_NONFINITE):
            raise TiltError(rc, "tilt_inner_batch")
        return rc, [result_dict(rarr[i]) for i in range(count)]

    def pyramid(self, image_ptr: int, height: int, width: int, row_stride: int, out_ptr: int, levels: int,
                stream=None):
        rc = _lib.tilt_pyramid(self._h, C.c_void_p(int(image_ptr)), int(height), int(width), int(row_stride),
                               C.c_void_p(int(out_ptr)), int(levels), C.c_void_p(_stream_ptr(stream)))
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_pyramid")

    def rasl_solve_batch(self, sets, params=None, outs_A=None, outs_E=None, stream=None):
        """RASL problems: `sets` is a list of dicts with the device pointer
        `images` (count images, image_stride floats apart), height, width,
        row_stride, count, m, n, model and tau0 (count x 3 x 3, host).
        Returns (worst status, per-problem dicts with tau (count x 3 x 3),
        objective, outer_iters, inner_iters_total, svt_rank, status,
        solve_ms)."""
        n = len(sets)
        prm = params if params is not None else default_params()
        parr = (RaslProblem * n)()
        rarr = (RaslResult * n)()
        keep = []
        for i, st in enumerate(sets):
            N = int(st["count"])
            t0 = np.ascontiguousarray(np.asarray(st["tau0"], np.float64).reshape(N * 9))
            tb = (C.c_double * (N * 9))(*t0.tolist())
            tout = (C.c_double * (N * 9))()
            keep += [tb, tout]
            parr[i] = RaslProblem(C.c_void_p(int(st["images"])), int(st["image_stride"]), int(st["height"]),
                                  int(st["width"]), int(st["row_stride"]), N, int(st["m"]), int(st["n"]),
                                  int(st["model"]), C.cast(tb, C.POINTER(C.c_double)))
            rarr[i].tau = C.cast(tout, C.POINTER(C.c_double))
            rarr[i].A = C.c_void_p(int(outs_A[i])) if outs_A is not None and outs_A[i] else None
            rarr[i].E = C.c_void_p(int(outs_E[i])) if outs_E is not None and outs_E[i] else None
        rc = _lib.tilt_rasl_solve_batch(self._h, parr, n, C.byref(prm), rarr, C.c_void_p(_stream_ptr(stream)))
        if rc < 0 and rc not in (TILT_ERR_SINGULAR, TILT_ERR_NONFINITE, TILT_ERR_TOO_LARGE, TILT_ERR_ARG):
            raise TiltError(rc, "tilt_rasl_solve_batch")
        out = []
        for i, st in enumerate(sets):
            N = int(st["count"])
            r = rarr[i]
            c = r.counters
            out.append(dict(tau=np.array([r.tau[k] for k in range(9 * N)]).reshape(N, 3, 3),
                            objective=r.objective, outer_iters=r.outer_iters,
                            inner_iters_total=r.inner_iters_total, svt_rank=r.svt_rank, status=r.status,
                            solve_ms=r.solve_ms,
                            counters=dict(inner_iters=c.inner_iters, svt_calls=c.svt_calls,
                                          jacobi_sweeps=c.jacobi_sweeps, jacobi_pairs=c.jacobi_pairs,
                                          jacobi_rotations=c.jacobi_rotations, recon_rows=c.recon_rows)))
        del keep
        return rc, out

    def warp_jacobian(self, problems: List[Problem], taus, I_ptr: int, J_ptr: int, stream=None):
        n = len(problems)
        parr = (Problem * n)(*problems)
        t = np.ascontiguousarray(np.asarray(taus, np.float64).reshape(n, 9))
        tarr = (C.c_double * (9 * n))(*t.reshape(-1).tolist())
        rc = _lib.tilt_warp_jacobian(self._h, parr, tarr, n, C.c_void_p(int(I_ptr)), C.c_void_p(int(J_ptr)),
                                     C.c_void_p(_stream_ptr(stream)))
        if rc != TILT_OK:
            raise TiltError(rc, "tilt_warp_jacobian")
