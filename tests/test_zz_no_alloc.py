"""tilt_svt_batch_noalloc against tilt_svt_batch: the same kernels on the
same inputs, so A, the singular values, the ranks and the work counters
must agree bit for bit -- on two calls in a row, the second with a smaller
batch and a different shape (the fixed array keeps the first call's
contents), and with a tiled shape (the working planes of the Jacobi beyond
LDS come from the array too).  Also the limit: a batch beyond the array is
refused with TILT_ERR_TOO_LARGE and nothing is launched."""

import math

import numpy as np
import pytest

import oracle as O
from gpu_util import to_device

pytestmark = pytest.mark.gpu


def _batch(m, n, count, seed):
    rng = np.random.default_rng(seed)
    Ms = []
    for i in range(count):
        L = rng.standard_normal((m, 3)) @ rng.standard_normal((3, n))
        Mi = L / np.linalg.norm(L) + 0.05 * rng.standard_normal((m, n)) / math.sqrt(m * n)
        Ms.append(Mi.astype(np.float32))
    eps = np.linspace(1e-3, 0.05, count).astype(np.float32)
    return np.stack(Ms), eps


def _run(fn, M, eps, device):
    import torch

    count, m, n = M.shape
    dM = to_device(M, device)
    dA = torch.full_like(dM, float("nan"))
    dS = torch.full((count, min(m, n)), float("nan"), dtype=torch.float32, device=device)
    print(f"{fn.__name__}: {count} x {m}x{n}", flush=True)
    ranks, cnt = fn(dM.data_ptr(), dA.data_ptr(), dS.data_ptr(), count, m, n, eps)
    torch.cuda.synchronize()
    return dA.cpu().numpy(), dS.cpu().numpy(), ranks, cnt


@pytest.mark.parametrize("shapes", [((40, 100, 130), (7, 64, 48)), ((3, 256, 227), (2, 200, 150))])
def test_noalloc_equals_svt_batch_twice(tilt, ctx, device, shapes):
    for k, (count, m, n) in enumerate(shapes):
        M, eps = _batch(m, n, count, 77 + k)
        A0, S0, r0, c0 = _run(ctx.svt_batch, M, eps, device)
        A1, S1, r1, c1 = _run(tilt.svt_batch_noalloc, M, eps, device)
        assert np.array_equal(A0, A1) and np.array_equal(S0, S1), (k, count, m, n)
        assert r0 == r1 and c0 == c1, (k, r0, r1, c0, c1)
        # and the shrinkage itself against the FP64 oracle (tolerance of
        # the SVT parity tests)
        for i in (0, count - 1):
            Aref, _ = O.svt(M[i].astype(np.float64), float(eps[i]))
            assert np.linalg.norm(A1[i] - Aref) <= 1e-5 * np.linalg.norm(Aref), (k, i)


def test_noalloc_refuses_batches_beyond_its_array(tilt, device):
    import torch

    m = n = 512                                   # 2 MiB of working planes per matrix
    count = tilt.tilt.TILT_SVT_NOALLOC_BYTES // (8 * m * n) + 1
    dM = torch.zeros((1,), dtype=torch.float32, device=device)
    with pytest.raises(tilt.TiltError) as e:
        tilt.svt_batch_noalloc(dM.data_ptr(), dM.data_ptr(), 0, count, m, n, 1e-3)
    assert e.value.code == tilt.tilt.TILT_ERR_TOO_LARGE
