"""Host-only checks of the C interface: the library loads, exports every
symbol the header declares, and its host-side helpers and argument
validation behave as documented (no GPU needed)."""

import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tilt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tilt_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(tilt):
    lib = tilt.tilt.library()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(tilt.EXPORTS)


def test_nm_exports(tilt):
    out = subprocess.run(["nm", "-D", "--defined-only", tilt.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (tilt_\w+)", out))
    assert set(header_functions()) <= exported


def test_default_params(tilt):
    p = tilt.default_params()
    assert p.eps1 == 1e-5 and p.eps2 == 1e-3 and p.rho0 == 1.5 and p.mu_max == 1e10
    assert p.max_inner == 2000 and p.max_outer == 50 and p.lambda_ < 0 and p.mu0 < 0
    assert abs(p.jacobi_tol - 1e-6) < 1e-12 and p.max_sweeps == 40 and p.pyramid_levels == 1 and p.graph_inner == 0
    assert p.eps_obj == 0.0 and p.eps_svd == 1e-3 and p.svdws_every == 0


def test_status_strings(tilt):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert tilt.status_string(code) != "unknown status"
    assert tilt.status_string(42) == "unknown status"


def _apply(H, u, v):
    x = H @ np.array([u, v, 1.0])
    return x[:2] / x[2]


@pytest.mark.parametrize("model", [6, 8])
def test_tau_from_quad_maps_corners(tilt, model):
    m, n = 40, 70
    if model == 6:
        tl = np.array([10.0, 20.0])
        e = np.array([60.0, 8.0])
        f = np.array([-5.0, 35.0])
        quad = [tl, tl + e, tl + e + f, tl + f]
    else:
        quad = [np.array(q) for q in ([10.0, 20.0], [82.0, 25.0], [90.0, 70.0], [5.0, 60.0])]
    H = tilt.tau_from_quad(np.concatenate(quad), m, n, model)
    a, b = (n - 1) / 2, (m - 1) / 2
    for (u, v), q in zip([(-a, -b), (a, -b), (a, b), (-a, b)], quad):
        np.testing.assert_allclose(_apply(H, u, v), q, atol=1e-9)
    assert H[2, 2] == 1.0


def test_tau_from_quad_rejects_bad_input(tilt):
    with pytest.raises(tilt.TiltError):
        tilt.tau_from_quad([0, 0, 10, 0, 12, 10, 0, 10], 10, 10, 6)  # not a parallelogram
    with pytest.raises(tilt.TiltError):
        tilt.tau_from_quad([0, 0, 0, 0, 0, 0, 0, 0], 10, 10, 8)      # degenerate
    with pytest.raises(tilt.TiltError):
        tilt.tau_from_quad([0, 0, 1, 0, 1, 1, 0, 1], 10, 10, 7)      # unknown model


def test_workspace_bytes(tilt):
    b = tilt.workspace_bytes(100, 100)
    assert b >= 14 * 100 * 100 * 4
    assert tilt.workspace_bytes(20, 2100) == 0      # rows longer than the SVT's 2048
    assert tilt.workspace_bytes(1, 10) == 0 or tilt.workspace_bytes(1, 10) > 0


def test_argument_validation_without_device(tilt):
    import ctypes as C

    lib = tilt.tilt.library()
    prm = tilt.default_params()
    img = np.zeros((10, 10), np.float32)
    pr = tilt.make_problem(0, 10, 10, 10, 5, 5, 6, np.eye(3))           # null image
    res = tilt.Result()
    assert lib.tilt_solve(C.byref(pr), C.byref(prm), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    pr = tilt.make_problem(img.ctypes.data, 10, 10, 10, 5, 5, 7, np.eye(3))  # bad model
    assert lib.tilt_solve(C.byref(pr), C.byref(prm), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    pr = tilt.make_problem(img.ctypes.data, 10, 10, 5, 5, 5, 6, np.eye(3))   # stride < width
    assert lib.tilt_solve(C.byref(pr), C.byref(prm), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    bad = tilt.default_params(rho0=0.5)
    pr = tilt.make_problem(img.ctypes.data, 10, 10, 10, 5, 5, 6, np.eye(3))
    assert lib.tilt_solve(C.byref(pr), C.byref(bad), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    bad = tilt.default_params(eps1=0.0)
    assert lib.tilt_solve(C.byref(pr), C.byref(bad), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    assert lib.tilt_ctx_destroy(None) == tilt.tilt.TILT_ERR_ARG
    rp = (tilt.tilt.RaslProblem * 1)()
    rr = (tilt.tilt.RaslResult * 1)()
    assert lib.tilt_rasl_solve_batch(None, rp, 1, C.byref(prm), rr, None) == tilt.tilt.TILT_ERR_ARG


def test_quad_initialisation_is_validated(tilt):
    import ctypes as C

    lib = tilt.tilt.library()
    prm = tilt.default_params()
    img = np.zeros((10, 10), np.float32)
    res = tilt.Result()
    pr = tilt.make_problem(img.ctypes.data, 10, 10, 10, 5, 5, 6, quad=[0, 0, 0, 0, 0, 0, 0, 0])  # degenerate
    assert lib.tilt_solve(C.byref(pr), C.byref(prm), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    pr = tilt.make_problem(img.ctypes.data, 10, 10, 10, 5, 5, 6, quad=[1, 1, 2, 1, 2, 3, 1, 3])
    pr.init = 2                                                                            # unknown mode
    assert lib.tilt_solve(C.byref(pr), C.byref(prm), C.byref(res)) == tilt.tilt.TILT_ERR_ARG
    with pytest.raises(ValueError):
        tilt.make_problem(img.ctypes.data, 10, 10, 10, 5, 5, 6, np.eye(3), quad=[1, 1, 2, 1, 2, 3, 1, 3])


def test_struct_layouts_match_the_header(tilt, tmp_path):
    """sizeof and field offsets of the ABI structs, compiled from
    include/tilt.h with the host C compiler, against the ctypes binding."""
    fields = {"tilt_problem": ["image", "row_stride", "m", "model", "init", "tau0", "quad"],
              "tilt_result": ["tau", "A", "E", "outer_iters", "svt_rank", "status", "rank", "objective", "mu",
                              "solve_ms", "done_ms", "counters"],
              "tilt_params": ["lambda", "eps1", "max_inner", "svt_mode", "jacobi_tol", "max_sweeps",
                              "pyramid_levels", "graph_inner", "eps_obj", "eps_svd", "svdws_every"],
              "tilt_counters": ["inner_iters", "recon_rows", "svdws_steps"]}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "tilt.h"', "int main(void) {"]
    for st, fs in fields.items():
        src.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            src.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    src.append("  return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    T = tilt.tilt
    py = {"tilt_problem": T.Problem, "tilt_result": T.Result, "tilt_params": T.Params, "tilt_counters": T.Counters}
    for st, cls in py.items():
        assert int(got[st]) == C_sizeof(cls), st
        for f in fields[st]:
            name = "lambda_" if f == "lambda" else f
            assert int(got[f"{st}.{f}"]) == getattr(cls, name).offset, (st, f)


def C_sizeof(cls):
    import ctypes

    return ctypes.sizeof(cls)


def test_missing_library_fails_loudly():
    code = "import paper_1205_5351_amd"
    env = dict(os.environ, TILT_LIB="/nonexistent/libtilt.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode != 0 and "HIP library not found" in r.stderr


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1205_5351_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "tilt_oracle" not in src, f


def _restore_tuning(tilt):
    tilt.tune_clear()
    if os.path.exists(tilt.TUNING_TABLE):
        tilt.load_tuning(tilt.TUNING_TABLE)


def test_svt_layout_single_float_tails(tilt):
    """Two-row blocks of 8 or 16 lanes hold a remainder of at most 2 floats
    per lane as single floats; other layouts, longer remainders and the
    tiled path use whole chunks."""
    from svt_layouts import TAIL_LAYOUTS

    m = 22
    try:
        for lpp, nch, tl, nr in TAIL_LAYOUTS:
            tilt.tune_set(m, nr, 2, lpp)
            assert tilt.svt_layout(m, nr) == (2, lpp, nch, tl, 0), (lpp, nr)
            assert tilt.svt_layout(nr, m) == (2, lpp, nch, tl, 0), (lpp, nr)  # rows are min(m, n)
        tilt.tune_set(m, 128, 2, 8)
        assert tilt.svt_layout(m, 128) == (2, 8, 4, 0, 0)            # whole chunks: no tail
        tilt.tune_set(m, 120, 2, 8)
        assert tilt.svt_layout(m, 120) == (2, 8, 4, 0, 0)            # remainder of 3 floats per lane
        tilt.tune_set(m, 99, 1, 8)
        assert tilt.svt_layout(m, 99) == (1, 8, 4, 0, 0)             # one-row blocks: whole chunks
        tilt.tune_set(m, 35, 2, 4)
        assert tilt.svt_layout(m, 35) == (2, 4, 3, 0, 0)             # 4-lane groups: whole chunks
    finally:
        _restore_tuning(tilt)
    bs, lpp, nch, tl, tiled = tilt.svt_layout(600, 600)              # beyond LDS: tiled, whole chunks
    assert tiled == 1 and tl == 0
    with pytest.raises(tilt.TiltError):
        tilt.svt_layout(20, 2100)                                   # rows longer than 2048 floats
    with pytest.raises(tilt.TiltError):
        tilt.svt_layout(0, 10)


def test_peak_probe_rejects_bad_arguments(tilt):
    """Argument checks of the machine-peak probe come before any device call."""
    with pytest.raises(tilt.TiltError):
        tilt.peak_probe(7, 0, 1, 1 << 20, 1)          # unknown kind
    with pytest.raises(tilt.TiltError):
        tilt.peak_probe(2, 0, 0, 1 << 20, 1)          # no destination
    with pytest.raises(tilt.TiltError):
        tilt.peak_probe(0, 0, 1, 1 << 20, 1)          # copy without a source
    with pytest.raises(tilt.TiltError):
        tilt.peak_probe(2, 0, 1, 1 << 20, 0)          # no iterations
