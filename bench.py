#!/usr/bin/env python3
"""Throughput of batched TILT solves (LADMAP with adaptive penalty and
variable warm start, cold one-sided Jacobi SVT every iteration) on one GPU.

One step = one whole-batch solve: every patch of the workload runs the full
outer loop (warp, Jacobian, constraints, inner LADMAP loop, Delta tau) to
convergence in the fused persistent kernel.  Inputs are resident in HBM
before the timed region.  Prints one JSON line on stdout; progress goes to
stderr.

Default workload: 256 projective 100x100 windows in 400x400 synthetic
images (rank 2-5 cosine textures, random projective warp, 20% corrupted
pixels, lambda = 1/sqrt(100)).
"""

from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rectified patches/s at τ rel err≤1e-4 vs plain GPU path; p50/p99 latency"
PEAK_FP32_VECTOR_TFLOPS = 157.3
# MI355X published peaks used for the machine-peak study (256 CUs at 2.4 GHz;
# LDS 256 bytes per clock per CU)
NOMINAL_PEAKS = {"hbm_copy": (8000.0, "GB/s"), "lds_read": (157.3, "TB/s"),
                 "fp32_fma": (157.3, "TFLOP/s"), "fp32_mfma": (157.3, "TFLOP/s")}
# probe kind, work unit scale, iterations (each probe launch lasts ~10-50 ms)
PEAK_PROBES = {"hbm_copy": (0, 1e9, 1), "lds_read": (1, 1e12, 20000), "fp32_fma": (2, 1e12, 100000),
               "fp32_mfma": (3, 1e12, 40000)}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tau_rel_err(Ha, Hb, tau0, m, n):
    """||Ha - Hb||_F / ||Hb||_F in the window's scaled coordinates."""
    import numpy as np

    s = max(m, n) / 2.0
    c = tau0[:2, 2] / tau0[2, 2]
    Ti = np.array([[1 / s, 0, -c[0] / s], [0, 1 / s, -c[1] / s], [0, 0, 1.0]])
    S = np.diag([s, s, 1.0])

    def nrm(H):
        X = Ti @ (H / H[2, 2]) @ S
        return X / X[2, 2]

    a, b = nrm(np.asarray(Ha)), nrm(np.asarray(Hb))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def measure_peak(T, torch, name, reps=5, nbytes=1 << 30):
    """Best rate of `reps` launches of one machine-peak probe kernel
    (tilt_peak_probe), in the unit of NOMINAL_PEAKS[name]."""
    kind, scale, iters = PEAK_PROBES[name]
    dev = torch.device("cuda:0")
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev) if kind == 0 else None
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    best = 0.0
    for _ in range(reps):
        ms, work = T.peak_probe(kind, src.data_ptr() if src is not None else 0, dst.data_ptr(), nbytes, iters)
        best = max(best, work / (ms * 1e-3) / scale)
    del src, dst
    return best


def peaks_main(args):
    """Machine peaks measured with the solver's compiler flags: HBM stream
    copy, LDS 16-byte reads consumed by one VALU operation per word, FP32
    vector FMA (no packed FP32 in this build) and FP32 MFMA 16x16x4; each
    against MI355X's published figure."""
    import torch

    import paper_1205_5351_amd as T

    measured = {}
    for name in PEAK_PROBES:
        nbytes = (2 << 30) if name == "hbm_copy" else (1 << 30)
        measured[name] = measure_peak(T, torch, name, nbytes=nbytes)
        log(f"{name}: {measured[name]:.1f} {NOMINAL_PEAKS[name][1]}")
    out = {
        "metric": "machine peaks measured by probe kernels (best of 5 launches)",
        "value": round(measured["fp32_fma"], 2), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": 5, "warmup": 0, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "peak-probes", "hbm_copy_bytes": 2 << 30, "grid": "8 workgroups of 256 per CU"},
        "peaks": {k: {"measured": round(v, 2), "nominal": NOMINAL_PEAKS[k][0], "unit": NOMINAL_PEAKS[k][1],
                      "frac_of_nominal": round(v / NOMINAL_PEAKS[k][0], 4)} for k, v in measured.items()},
    }
    print(json.dumps(out), flush=True)


def solve_flops(res, p, warm=False):
    """Algorithmic FP32 flops of one patch's solve, from its work counters.

    Jacobi: every examined pair costs one length-nr inner product (2 nr; the
    squared norms are updated in O(1) per rotation); every rotated pair
    costs a 2x2 rotation of two length-nr rows (6 nr).  Shrinkage:
    C = X B^T and A = (C W) B over the k kept rows, 4 nc nr k.  Updates:
    about (20 + 8 p') flops per entry per inner iteration.  Warm start: the
    product R M (2 nc^2 nr per SVT) and the rotation rows (6 nc per
    rotation); the Newton-Schulz steps are not counted.  Pyramid levels are
    counted at the level-0 shape (an upper bound)."""
    nr, nc = max(p.m, p.n), min(p.m, p.n)
    c = res["counters"]
    pp = p.model - 3
    f = (2.0 * nr * c["jacobi_pairs"] + 6.0 * nr * c["jacobi_rotations"] + 4.0 * nc * nr * c["recon_rows"]
         + (20.0 + 8.0 * pp) * nc * nr * c["inner_iters"])
    if warm:
        f += 2.0 * nc * nc * nr * c["inner_iters"] + 6.0 * nc * c["jacobi_rotations"]
    return f


KERNEL_SOURCES = ("tilt_kernels.hip", "tilt_svdws.inc", "tilt_rasl.inc")  # one translation unit
# committed rocprofv3 summaries of the fused kernel: (workload, svt_mode) -> file under profiles/
PROFILES = {("batch-256x100x100-projective", 0): "k_fused_batch256x100x100.md",
            ("batch-256x100x100-projective", 1): "k_fused_warm_batch256x100x100.md",
            ("uneven-1024-32to256-mixed", 1): "k_fused_uneven1024.md"}


def kernel_source_sha(sources=KERNEL_SOURCES) -> str:
    import hashlib

    h = hashlib.sha256()
    for name in sources:
        h.update(open(os.path.join(ROOT, "paper_1205_5351_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(profile: str, sources=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel from its committed rocprofv3 summary
    (profiles/<profile>), or None when the kernel source has changed since
    the counters were taken (or no summary exists)."""
    prof = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(prof):
        return None
    fields = {}
    for line in open(prof):
        line = line.strip().lstrip("- ")
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_sha(sources) or "traffic_bytes" not in fields:
        return None
    return int(fields["traffic_bytes"])


def _oracle_worker(args):
    cfg, idx, prm_kw = args
    import oracle as O
    import tilt_synth as ts

    prm_kw = dict(prm_kw)
    levels = prm_kw.pop("levels", 1)
    p = ts.make_batch(cfg, [idx])[0]
    t0 = time.perf_counter()
    if levels > 1:
        r, _ = O.pyramid.tilt_solve_pyramid(p.image, p.tau0, p.m, p.n, p.model, O.Params(**prm_kw), levels=levels)
    else:
        r = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, O.Params(**prm_kw), lam=p.lam)
    return {"idx": idx, "seconds": time.perf_counter() - t0, "outer": r.outer_iters, "inner": sum(r.inner_iters),
            "tau": r.tau_px.tolist(), "objective": r.objective}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, indices, prm_kw, workers):
    """The FP64 oracle on host cores: one patch per task, one worker process
    per core, one BLAS thread each."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        out = pool.map(_oracle_worker, [(cfg, i, prm_kw) for i in indices])
    wall = time.perf_counter() - t0
    return wall, out


def cold_jacobi_work(res, p):
    """Section-8(d) work of the cold one-sided Jacobi of one patch's solve:
    6 S m n^2 flops and 8 S m n^2 LDS bytes per SVD of an m x n matrix
    (n = min side) after S sweeps, i.e. 6 and 8 x m n^2 per sweep summed
    over all the patch's sweeps (pyramid levels counted at the level-0
    shape, an upper bound)."""
    nr, nc = max(p.m, p.n), min(p.m, p.n)
    sweeps = res["counters"]["jacobi_sweeps"]
    return 6.0 * nr * nc * nc * sweeps, 8.0 * nr * nc * nc * sweeps


class Progress:
    """Prints the finished-request count of a long fused launch every
    `period` seconds (read from the device by tilt_ctx_progress), so a
    watcher sees the batch advance."""

    def __init__(self, ctx, label, period=20.0):
        import threading

        self.ctx, self.label, self.period = ctx, label, period
        self.stop = threading.Event()
        self.t0 = time.perf_counter()
        self.th = threading.Thread(target=self.run, daemon=True)

    def run(self):
        while not self.stop.wait(self.period):
            try:
                done, total = self.ctx.progress()
            except Exception:  # noqa: BLE001 - progress is best effort
                return
            if total:
                log(f"{self.label}: {done}/{total} requests finished after {time.perf_counter() - self.t0:.0f} s")

    def __enter__(self):
        self.th.start()
        return self

    def __exit__(self, *exc):
        self.stop.set()
        self.th.join()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=1, help="workload index in tilt_synth (default 1)")
    ap.add_argument("--patches", type=int, default=None, help="number of patches (default: all)")
    ap.add_argument("--plain-sample", type=int, default=8, help="patches re-solved by the plain path")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="patches solved by the CPU oracle (default: one per host core)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--per-patch", default=None, metavar="FILE",
                    help="write one JSON line per patch of the last timed launch (shape, iterations, solve time, "
                         "SVT calls and sweeps) to FILE")
    ap.add_argument("--svt-mode", type=int, default=None, choices=(0, 1),
                    help="0: cold Jacobi SVT every iteration; 1: warm start (default: the workload's definition, "
                         "cold for workload 1, warm for workload 2)")
    ap.add_argument("--pyramid", type=int, default=1, help="pyramid levels (1 = none)")
    ap.add_argument("--serve", action="store_true",
                    help="serving mode: Poisson arrivals through tilt_submit/tilt_poll (workload 4 by default)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="arrival window per rate in serving mode")
    ap.add_argument("--serve-max-outer", type=int, default=20,
                    help="outer iterations per pyramid level in serving mode")
    ap.add_argument("--serve-max-inner", type=int, default=200,
                    help="inner iterations per outer iteration in serving mode (a latency bound)")
    ap.add_argument("--convergence", action="store_true",
                    help="range-of-convergence sweep (checkerboard, 11 x 21 affine deformations, one batch)")
    ap.add_argument("--components", action="store_true",
                    help="run the component kernels once each for profiling: a 1 GiB device copy (counter "
                         "calibration), warp + Jacobian and SVT on the default workload's windows, and a short "
                         "plain-path solve of one patch; prints their kernel times")
    ap.add_argument("--precision", action="store_true",
                    help="precision study on the 128x128 workload: cold, warm FP32, warm bfloat16 + FP32 "
                         "refinement, warm bfloat16; tau and objective errors against the FP64 oracle")
    ap.add_argument("--precision-modes", default="0,1,2,3",
                    help="SVT variants of the precision study (svt_mode values); the bfloat16 start alone (3) runs "
                         "every inner loop to max_inner, so its single launch is long")
    ap.add_argument("--inner", action="store_true",
                    help="inner-loop-only mode (random I and J, the setting of Table 1)")
    ap.add_argument("--svdws", action="store_true",
                    help="SVD with warm start (svt_mode 4) against the warm-started Jacobi (svt_mode 1) on the "
                         "inner loop alone: time, iterations, Cayley steps, objective")
    ap.add_argument("--eps-svd", type=float, default=1e-3, help="switch threshold of --svdws")
    ap.add_argument("--rasl", action="store_true",
                    help="RASL variant: a batch of image sets (one window per image as the columns of the data "
                         "matrix), one fused launch; sets/s, images/s, latency, roofline, CPU oracle on a sample")
    ap.add_argument("--rasl-sets", type=int, default=256)
    ap.add_argument("--rasl-max-outer", type=int, default=10)
    ap.add_argument("--peaks", action="store_true",
                    help="machine peaks from probe kernels built like the solver: HBM copy, LDS reads, FP32 FMA, "
                         "FP32 MFMA, each against MI355X's published figure")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the solve, copy a buffer of this many MiB on the device (a plain copy of "
                         "known size, used to calibrate HBM byte counters in profiles)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver has no multi-GPU path; "
              "patches would be sharded across GPUs by the caller.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1205_5351_amd as T
    import tilt_synth as ts

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.svt_mode is None:
        # the uneven workload is defined with warm starts; the others cold
        args.svt_mode = 1 if args.workload == 2 else 0
    if args.serve:
        return serve_main(args)
    if args.svdws:
        return svdws_main(args)
    if args.inner:
        return inner_main(args)
    if args.rasl:
        return rasl_main(args)
    if args.precision:
        return precision_main(args)
    if args.peaks:
        return peaks_main(args)
    if args.components:
        return components_main(args)
    if args.convergence:
        return convergence_main(args)
    dev = torch.device("cuda:0")
    names = ts.config_names()
    t_gen = time.perf_counter()
    patches = ts.make_config(args.workload, count=args.patches)
    log(f"generated {len(patches)} patches of '{names[args.workload]}' in {time.perf_counter() - t_gen:.1f}s")

    imgs = [torch.from_numpy(p.image).to(dev) for p in patches]
    probs = [T.make_problem(im.data_ptr(), p.height, p.width, p.width, p.m, p.n, p.model, p.tau0)
             for im, p in zip(imgs, patches)]
    outA = [torch.zeros((p.m, p.n), dtype=torch.float32, device=dev) for p in patches]
    outE = [torch.zeros((p.m, p.n), dtype=torch.float32, device=dev) for p in patches]
    lam = patches[0].lam if all(abs(p.lam - patches[0].lam) < 1e-15 for p in patches) else -1.0
    prm = T.default_params(lam=lam, svt_mode=args.svt_mode, pyramid_levels=args.pyramid)
    ctx = T.Context(0)
    stream = torch.cuda.current_stream()
    Ap = [a.data_ptr() for a in outA]
    Ep = [e.data_ptr() for e in outE]
    torch.cuda.synchronize()

    if args.copy_probe_mib > 0:
        nel = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst

    for w in range(args.warmup):
        with Progress(ctx, f"warmup {w}"):
            rc, res = ctx.solve_batch(probs, prm, Ap, Ep, stream)
        log(f"warmup {w}: rc={rc} kernel {ctx.last_kernel_ms():.1f} ms")

    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        with Progress(ctx, f"step {k}"):
            rc, res = ctx.solve_batch(probs, prm, Ap, Ep, stream)
        kernel_ms.append(ctx.last_kernel_ms())
        log(f"step {k}: rc={rc} kernel {kernel_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    statuses = [r["status"] for r in res]
    outer_all = [r["outer_iters"] for r in res]
    # rectified: the solve finished normally, every inner loop met Cond1 and
    # Cond2 (no TILT_WARN_MAXITER) and the outer loop stopped on its own
    # before max_outer
    rectified = [s == 0 and o < prm.max_outer for s, o in zip(statuses, outer_all)]
    n_ok = sum(rectified)

    # Agreement with the plain (step-by-step) GPU path on a spread sample
    # (on the uneven workload among windows of at most 96x96 pixels: the
    # plain path drives each Jacobi round of a tiled window from the host)
    cand = [i for i in range(len(patches)) if args.workload != 2 or patches[i].m * patches[i].n <= 96 * 96]
    S = min(args.plain_sample, len(cand))
    sample = sorted(set(cand[int(round(i * (len(cand) - 1) / max(S - 1, 1)))] for i in range(S))) if S > 0 else []
    errs, plain_s, bitwise = [], 0.0, 0
    agree = 1.0
    if sample:
        t_pl = time.perf_counter()
        rc_p, res_p = ctx.solve_batch_plain([probs[i] for i in sample], prm, None, None, stream)
        plain_s = (time.perf_counter() - t_pl) / len(sample)
        errs = [tau_rel_err(res[i]["tau"], rp["tau"], patches[i].tau0, patches[i].m, patches[i].n)
                for i, rp in zip(sample, res_p)]
        agree = sum(1 for e in errs if e <= 1e-4) / len(errs)
        bitwise = sum(1 for i, rp in zip(sample, res_p) if np.array_equal(res[i]["tau"], rp["tau"]))
        log(f"plain path on {len(sample)} patches: {plain_s:.2f} s/patch, max tau rel err {max(errs):.2e}, "
            f"bitwise equal {bitwise}/{len(sample)}")

    n_patches = len(patches)
    value = n_patches * agree * (n_ok / n_patches) / (wall / args.steps)
    solve_ms = np.array([r["solve_ms"] for r in res])
    done_ms = np.array([r["done_ms"] for r in res])

    flops = sum(solve_flops(r, p, warm=args.svt_mode == 1) for r, p in zip(res, patches))
    jac = [cold_jacobi_work(r, p) for r, p in zip(res, patches)]
    jac_flops = sum(f for f, _ in jac)
    jac_lds = sum(b for _, b in jac)
    mfma_flops = (sum(2.0 * min(p.m, p.n) ** 2 * max(p.m, p.n) * r["counters"]["svt_calls"]
                      for r, p in zip(res, patches)) if args.svt_mode == 1 else 0.0)
    # attainable FP32 vector rate of this build (no packed FP32), measured
    # after the timed region by a probe kernel of a few ms
    fma_peak = measure_peak(T, torch, "fp32_fma", reps=3, nbytes=8 << 20)
    k_ms = float(np.mean(kernel_ms))
    achieved = jac_flops / (k_ms * 1e-3) / 1e12
    achieved_counted = flops / (k_ms * 1e-3) / 1e12
    lds_tbs = jac_lds / (k_ms * 1e-3) / 1e12
    outer = np.array(outer_all)
    inner = np.array([r["inner_iters_total"] for r in res])
    # the slowest patches of the launch (they set its length when few are
    # left running)
    tail = []
    for i in np.argsort(-solve_ms)[:5]:
        r, p = res[int(i)], patches[int(i)]
        tail.append({"idx": int(i), "m": p.m, "n": p.n, "outer": int(r["outer_iters"]),
                     "inner": int(r["inner_iters_total"]), "solve_ms": round(float(solve_ms[i]), 1),
                     "ms_per_inner": round(float(solve_ms[i]) / max(int(r["inner_iters_total"]), 1), 3),
                     "sweeps_per_svd": round(r["counters"]["jacobi_sweeps"] / max(r["counters"]["svt_calls"], 1), 2)})
    if args.per_patch:
        with open(args.per_patch, "w") as f:
            for i, (r, p) in enumerate(zip(res, patches)):
                f.write(json.dumps({"idx": i, "m": p.m, "n": p.n, "model": p.model, "status": int(r["status"]),
                                    "outer": int(r["outer_iters"]), "inner": int(r["inner_iters_total"]),
                                    "solve_ms": round(float(solve_ms[i]), 2), "done_ms": round(float(done_ms[i]), 2),
                                    "svt_calls": int(r["counters"]["svt_calls"]),
                                    "sweeps": int(r["counters"]["jacobi_sweeps"])}) + "\n")
    sweeps = sum(r["counters"]["jacobi_sweeps"] for r in res) / max(sum(r["counters"]["svt_calls"] for r in res), 1)

    cpu = None
    oracle_check = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        n_cpu = args.cpu_sample if args.cpu_sample is not None else cores
        # spread over the batch; on the uneven workload only windows of at
        # most 96 x 96 pixels, so the FP64 oracle sample stays at tens of
        # CPU-seconds
        pool_idx = [i for i in range(len(patches))
                    if args.workload != 2 or patches[i].m * patches[i].n <= 96 * 96]
        step = max(1, len(pool_idx) // max(n_cpu, 1))
        idx = pool_idx[::step][:n_cpu]
        prm_kw = dict(eps1=prm.eps1, eps2=prm.eps2, eps_outer=prm.eps_outer, mu0=prm.mu0, rho0=prm.rho0,
                      mu_max=prm.mu_max, max_inner=prm.max_inner, max_outer=prm.max_outer,
                      levels=args.pyramid)
        workers = min(cores, len(idx))
        log(f"CPU oracle on {len(idx)} patches with {workers} worker processes ({cores} cores) ...")
        cwall, cout = cpu_baseline(args.workload, idx, prm_kw, workers)
        secs = np.array([c["seconds"] for c in cout])
        cpu = {
            "value": round(len(idx) / cwall, 4),
            "unit": "patches/s",
            "cores": workers,
            "kind": "oracle",
            "cpu_model": cpu_model(),
            "host_cores": cores,
            "patch_s_p50": round(float(np.percentile(secs, 50)), 3),
            "patch_s_p99": round(float(np.percentile(secs, 99)), 3),
            "outer_mean": round(float(np.mean([c["outer"] for c in cout])), 2),
            "inner_total_mean": round(float(np.mean([c["inner"] for c in cout])), 1),
            "inner_total_max": int(max(c["inner"] for c in cout)),
            "sample": (f"{len(idx)} of the {n_patches} patches (indices {idx}"
                       + ("; windows of at most 96x96 px" if args.workload == 2 else "")
                       + f"), FP64 NumPy oracle with the same parameters, one process per core and one BLAS "
                       f"thread each; {secs.sum():.1f} CPU-s in {cwall:.1f} s wall"),
        }
        log(f"CPU oracle: {cpu['value']} patches/s")
        # the oracle gate: tau of the device result against the oracle on
        # the sampled patches whose outer loops both converged
        errs_o, obj_o, nconv = [], [], 0
        for c in cout:
            i = c["idx"]
            if res[i]["outer_iters"] < prm.max_outer and c["outer"] < prm.max_outer:
                nconv += 1
                errs_o.append(tau_rel_err(res[i]["tau"], np.array(c["tau"]), patches[i].tau0, patches[i].m,
                                          patches[i].n))
                obj_o.append(abs(res[i]["objective"] - c["objective"]) / c["objective"])
        oracle_check = {"sample": len(cout), "both_converged": nconv,
                        "within_1e-4": (sum(1 for e in errs_o if e <= 1e-4) / nconv) if nconv else None,
                        "max_tau_rel_err": max(errs_o) if errs_o else None,
                        "max_objective_rel_err": max(obj_o) if obj_o else None}
        log(f"oracle check: {oracle_check}")

    p0 = patches[0]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": names[args.workload],
            "patches": n_patches,
            "m": p0.m if len({(p.m, p.n) for p in patches}) == 1 else "mixed",
            "n": p0.n if len({(p.m, p.n) for p in patches}) == 1 else "mixed",
            "model": "projective" if all(p.model == 8 for p in patches) else "mixed",
            "lambda": lam if lam > 0 else "1/sqrt(max(m,n))",
            "svt": ("cold one-sided Jacobi every inner iteration" if args.svt_mode == 0
                    else "one-sided Jacobi warm-started from the previous rotation"),
            "pyramid_levels": args.pyramid,
            "eps1": prm.eps1, "eps2": prm.eps2, "eps_outer": prm.eps_outer, "rho0": prm.rho0,
        },
        "latency_ms": {
            "patch_solve_p50": round(float(np.percentile(solve_ms, 50)), 2),
            "patch_solve_p99": round(float(np.percentile(solve_ms, 99)), 2),
            "batch_done_p50": round(float(np.percentile(done_ms, 50)), 2),
            "batch_done_p99": round(float(np.percentile(done_ms, 99)), 2),
            "plain_path_per_patch": round(1000 * plain_s, 1),
        },
        "plain_check": {"sample": len(sample), "within_1e-4": agree, "bitwise_equal": bitwise,
                        "max_tau_rel_err": max(errs) if errs else None},
        "oracle_check": oracle_check,
        "work": {"outer_mean": float(outer.mean()), "inner_total_mean": float(inner.mean()),
                 "inner_total_max": int(inner.max()), "jacobi_sweeps_per_svd": round(sweeps, 2),
                 "rectified": n_ok, "status_ok": sum(1 for s in statuses if s == 0),
                 "status_maxiter": sum(1 for s in statuses if s == 1),
                 "outer_at_max": int(np.sum(outer >= prm.max_outer)),
                 "errors": sum(1 for s in statuses if s < 0),
                 "slowest": tail},
        "roofline": {
            "kernel": "k_fused (whole solves; one workgroup per patch, idle workgroups help tiled windows)",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
            "traffic": profiled_traffic(PROFILES[(names[args.workload], args.svt_mode)])
                       if (names[args.workload], args.svt_mode) in PROFILES and args.pyramid == 1
                       and args.patches is None else None,
            "work_model": "cold one-sided Jacobi, 6 S m n^2 flops and 8 S m n^2 LDS bytes per SVD (S: measured "
                          "sweeps, n = min side)",
            "kernel_ms": round(k_ms, 2),
            "flops_per_launch": jac_flops,
            "peak_measured": round(fma_peak, 2),
            "frac_of_measured": round(achieved / fma_peak, 4),
            "lds": {"achieved": round(lds_tbs, 3), "peak": NOMINAL_PEAKS["lds_read"][0], "unit": "TB/s",
                    "frac": round(lds_tbs / NOMINAL_PEAKS["lds_read"][0], 4), "bytes_per_launch": jac_lds},
            "mfma": ({"achieved": round(mfma_flops / (k_ms * 1e-3) / 1e12, 4), "peak": PEAK_FP32_VECTOR_TFLOPS,
                      "unit": "TFLOP/s", "frac": round(mfma_flops / (k_ms * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 6),
                      "flops_per_launch": mfma_flops, "what": "warm-start products R M, 2 n^2 m per SVD"}
                     if args.svt_mode == 1 else None),
            "counted": {"achieved": round(achieved_counted, 3), "flops_per_launch": flops,
                        "what": "flops from the work counters: 2 m per examined pair, 6 m per rotation, "
                                "shrinkage and updates"},
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def rectification_error(G_norm, tau_norm):
    """How far G^{-1} tau is from an axis-aligned scaling, allowing the
    axis swap a checkerboard is symmetric under: min over the two
    assignments of (largest off-assignment entry / smallest assigned entry)."""
    import numpy as np

    M = np.linalg.inv(G_norm) @ tau_norm
    M = M / M[2, 2]
    a = np.abs(M[:2, :2])
    diag = max(a[0, 1], a[1, 0]) / max(min(a[0, 0], a[1, 1]), 1e-300)
    swap = max(a[0, 0], a[1, 1]) / max(min(a[0, 1], a[1, 0]), 1e-300)
    return float(min(diag, swap))


def convergence_main(args):
    """Range of convergence: the checkerboard deformed by every (theta, t)
    of the grid, all solved in one batch; success = the returned transform
    undoes the deformation up to an axis-aligned scaling (error < 2e-2).
    The FP64 oracle re-solves a spread sample on the host."""
    import multiprocessing as mp

    import numpy as np
    import torch

    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    grid = ts.convergence_grid()
    patches = [ts.checkerboard_patch(th, t) for th, t in grid]
    imgs = [torch.from_numpy(p.image).to(dev) for p in patches]
    probs = [T.make_problem(im.data_ptr(), p.height, p.width, p.width, p.m, p.n, p.model, p.tau0)
             for im, p in zip(imgs, patches)]
    prm = T.default_params(max_outer=50, svt_mode=args.svt_mode)
    ctx = T.Context(0)
    ctx.solve_batch(probs[:4], prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, res = ctx.solve_batch(probs, prm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    errs = []
    for p, r in zip(patches, res):
        H = r["tau"]
        s = max(p.m, p.n) / 2.0
        c = p.meta["center"]
        Ti = np.array([[1 / s, 0, -c[0] / s], [0, 1 / s, -c[1] / s], [0, 0, 1.0]])
        Hn = Ti @ H @ np.diag([s, s, 1.0])
        errs.append(rectification_error(p.meta["G_norm"], Hn / Hn[2, 2]))
    ok = [e < 2e-2 for e in errs]
    rows = []
    for k in range(11):
        rows.append("".join("#" if ok[k * 21 + j] else "." for j in range(21)))
    log("success map (rows: theta = 0..30 deg in 3 deg steps; columns: t = 0..1 in 0.05 steps)")
    for k, row in enumerate(rows):
        log(f"  {3 * k:2d} deg  {row}")
    agree = None
    if not args.no_cpu:
        sample = list(range(0, len(grid), 23))[:10]
        ctxp = mp.get_context("spawn")
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        with ctxp.Pool(len(sample)) as pool:
            ref_errs = pool.map(_convergence_oracle_worker, [grid[i] for i in sample])
        agree = sum(1 for i, e in zip(sample, ref_errs) if (e < 2e-2) == ok[i]) / len(sample)
        log(f"oracle agreement on {len(sample)} sampled cases: {agree}")
    out = {
        "metric": "range of convergence: fraction of (theta, t) cases rectified",
        "value": round(sum(ok) / len(ok), 4),
        "unit": "fraction",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(1000 * wall, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic checkerboard",
        "config": {"workload": "convergence-sweep-11x21-checkerboard-60x60", "cases": len(grid),
                   "max_outer": 50, "patches_per_s": round(len(grid) / wall, 2)},
        "success_map": rows,
        "oracle_agreement": agree,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def _convergence_oracle_worker(theta_t):
    import oracle as O
    import tilt_synth as ts

    p = ts.checkerboard_patch(*theta_t)
    r = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, O.Params(max_outer=50))
    return rectification_error(p.meta["G_norm"], r.tau_norm)


def _precision_oracle_worker(idx):
    import oracle as O
    import tilt_synth as ts

    p = ts.make_batch(3, [idx])[0]
    r = O.tilt_solve(p.image, p.tau0, p.m, p.n, p.model, O.Params(), lam=p.lam)
    return r.tau_px, r.objective, r.outer_iters


def precision_main(args):
    """512 projective 128x128 windows (rank 4, 15 % corruption) with four
    SVT variants; per-patch tau and objective error against the FP64 oracle
    on a sample solved on the host in parallel."""
    import numpy as np
    import torch

    import oracle as O
    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    count = args.patches or 512
    patches = ts.make_config(3, count=count)
    imgs = [torch.from_numpy(p.image).to(dev) for p in patches]
    probs = [T.make_problem(im.data_ptr(), p.height, p.width, p.width, p.m, p.n, p.model, p.tau0)
             for im, p in zip(imgs, patches)]
    ctx = T.Context(0)
    sample = list(range(0, count, max(1, count // 12)))[:12]
    ref = None
    if not args.no_cpu:
        import multiprocessing as mp

        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(len(sample)) as pool:
            ref = pool.map(_precision_oracle_worker, sample)
        log(f"oracle on {len(sample)} patches: {time.perf_counter() - t0:.1f} s")
    modes = []
    names = {0: "cold FP32", 1: "warm FP32 (MFMA f32)", 2: "warm BF16 MFMA + FP32 refinement", 3: "warm BF16 MFMA"}
    for mode in sorted({int(x) for x in args.precision_modes.split(",")}):
        prm = T.default_params(lam=patches[0].lam, svt_mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = ctx.solve_batch(probs, prm)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        row = {"svt_mode": mode, "name": names[mode], "patches_per_s": round(count / wall, 3),
               "kernel_ms": round(ctx.last_kernel_ms(), 1),
               "sweeps_per_svd": round(sum(r["counters"]["jacobi_sweeps"] for r in res) /
                                       max(1, sum(r["counters"]["svt_calls"] for r in res)), 2)}
        if ref is not None:
            terr = [O.tau_rel_err(res[i]["tau"], rt[0], patches[i].m, patches[i].n) for i, rt in zip(sample, ref)]
            oerr = [abs(res[i]["objective"] - rt[1]) / rt[1] for i, rt in zip(sample, ref)]
            conv = [rt[2] < 50 and res[i]["outer_iters"] < 50 for i, rt in zip(sample, ref)]
            row.update(tau_err_max=float(np.max(terr)), tau_err_median=float(np.median(terr)),
                       tau_err_max_converged=float(max([e for e, c in zip(terr, conv) if c], default=0.0)),
                       objective_err_max=float(np.max(oerr)), per_patch_tau_err=[float(e) for e in terr])
        modes.append(row)
        log(f"{names[mode]}: {row['patches_per_s']} patches/s")
    out = {
        "metric": "precision study: patches/s and error vs FP64 oracle per SVT variant",
        "value": next((m for m in modes if m["svt_mode"] == 2), modes[-1])["patches_per_s"],
        "unit": "patches/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": next((m for m in modes if m["svt_mode"] == 2), modes[-1])["kernel_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": "batch-512x128x128-projective", "patches": count, "oracle_sample": sample},
        "modes": modes, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def components_main(args):
    """Component kernels on the 256 x 100x100 workload, for rocprofv3."""
    import numpy as np
    import torch

    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    ctx = T.Context(0)
    ps = ts.make_config(1)
    nel = (1 << 30) // 4
    src = torch.ones(nel, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    log("copy probe: 1024 MiB read + 1024 MiB written")
    imgs = [torch.from_numpy(p.image).to(dev) for p in ps]
    probs = [T.make_problem(im.data_ptr(), p.height, p.width, p.width, p.m, p.n, p.model, p.tau0)
             for im, p in zip(imgs, ps)]
    m, n, pm = ps[0].m, ps[0].n, ps[0].model
    dI = torch.zeros((len(ps), m, n), dtype=torch.float32, device=dev)
    dJ = torch.zeros((len(ps), pm, m, n), dtype=torch.float32, device=dev)
    taus = np.stack([p.tau0 for p in ps])
    out = {}
    for name, fn in (("warp_jacobian", lambda: ctx.warp_jacobian(probs, taus, dI.data_ptr(), dJ.data_ptr())),
                     ("svt", lambda: ctx.svt_batch(dI.data_ptr(), dA.data_ptr(), 0, len(ps), m, n,
                                                   np.full(len(ps), 0.02, np.float32)))):
        if name == "svt":
            dA = torch.zeros_like(dI)
        ts_ = []
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts_.append(1000 * (time.perf_counter() - t0))
        out[name + "_ms"] = round(min(ts_), 3)
        log(f"{name}: {min(ts_):.3f} ms per call ({len(ps)} windows)")
    for g in (0, 16):
        prm = T.default_params(lam=ps[0].lam, fixed_iters=1, max_outer=2, max_inner=50, graph_inner=g)
        t0 = time.perf_counter()
        ctx.solve_batch_plain(probs[:1], prm)
        torch.cuda.synchronize()
        key = "plain_2x50_ms" if g == 0 else f"plain_2x50_graph{g}_ms"
        out[key] = round(1000 * (time.perf_counter() - t0), 1)
        log(f"plain path, one patch, 2 x 50 iterations, graph_inner={g}: {out[key]} ms")
    print(json.dumps({"components": out}), flush=True)
    ctx.close()


# LADMAP column of Table 1 (MATLAB, one Xeon E5540 core): seconds per
# solve and iterations; context only (other machine, unstated inputs).
PAPER_TABLE1_LADMAP = {10: (7.49e-6, 20.4), 50: (0.00054, 21.2), 100: (0.00252, 22.2), 300: (0.10501, 21.9),
                       500: (0.6574, 22.0), 1000: (25.8139, 23.0)}


def inner_main(args):
    """Inner loop alone on random I ~ U(0,1) and J ~ N(0,1) (p = 5) at the
    sizes of Table 1 (10 x 10 to 1000 x 1000): batch throughput, mean
    per-solve latency and iterations, with the FP64 oracle on one problem
    per size (same inputs, up to 500 x 500) for the objective and iteration
    count.  Batches of 64 or more large problems run one workgroup per
    problem; a single large problem (the latency rows) takes the wide path,
    whose Jacobi rounds run on many workgroups."""
    import numpy as np
    import torch

    import oracle as O
    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    ctx = T.Context(0)
    prm = T.default_params(svt_mode=args.svt_mode)
    rows = []
    p = 5
    for size, count in ((10, 256), (50, 256), (100, 256), (300, 64), (300, 1), (500, 16), (500, 1), (1000, 1)):
        Is, Js = zip(*[ts.inner_problem(k, size, size, p) for k in range(count)])
        dI = torch.from_numpy(np.stack(Is)).to(dev)
        dJ = torch.from_numpy(np.stack(Js)).to(dev)
        dA = torch.zeros_like(dI)
        dE = torch.zeros_like(dI)
        ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), min(count, 8), size, size, p, prm)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), count, size, size, p, prm, dA.data_ptr(),
                                  dE.data_ptr())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = ctx.last_kernel_ms()
        iters = np.array([r["inner_iters_total"] for r in res])
        objs = np.array([r["objective"] for r in res])
        lat = np.array([r["solve_ms"] for r in res])
        row = {"size": size, "count": count, "path": "wide" if (size >= 300 and count * 8 <= 256) else "one workgroup per problem",
               "solves_per_s": round(count / (kms * 1e-3), 2),
               "kernel_ms": round(kms, 2), "latency_mean_ms": round(float(lat.mean()), 3),
               "iters_mean": round(float(iters.mean()), 2), "objective_mean": round(float(objs.mean()), 4),
               "gpu_iters_0": int(iters[0]),
               "paper_ladmap_s_per_solve": PAPER_TABLE1_LADMAP[size][0],
               "paper_ladmap_iters": PAPER_TABLE1_LADMAP[size][1]}
        if size <= 500 and count > 1:
            # oracle on problem 0
            lam = 1.0 / math.sqrt(size)
            Jm = np.asarray(Js[0], np.float64).reshape(p, size * size).T
            I64 = np.asarray(Is[0], np.float64)
            Z = np.zeros_like(I64)
            opr = O.Params(eps1=prm.eps1, eps2=prm.eps2, mu0=prm.mu0, rho0=prm.rho0, mu_max=prm.mu_max,
                           max_inner=prm.max_inner)
            t1 = time.perf_counter()
            ref = O.ladmap_inner(I64, O.Annihilator(Jm), lam, I64, Z, Z, opr)
            cpu_s = time.perf_counter() - t1
            ref_obj = O.objective(ref.A, ref.E, lam)
            row.update({"oracle_obj_rel_err": float(abs(res[0]["objective"] - ref_obj) / ref_obj),
                        "oracle_iters": ref.iters, "oracle_cpu_s": round(cpu_s, 3)})
        rows.append(row)
        log(f"inner {size}x{size}: {row}")
    head = next(r for r in rows if r["size"] == 100)
    out = {
        "metric": "LADMAP inner loop alone (Table 1 setting): solves/s",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": head["kernel_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (I ~ U(0,1), J ~ N(0,1), p = 5)",
        "config": {"workload": "inner-loop-only-table1", "value_at": "256 problems of 100x100",
                   "svt": "cold" if args.svt_mode == 0 else "warm", "eps1": prm.eps1, "eps2": prm.eps2},
        "sizes": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def svdws_main(args):
    """Alg. 2 (SVD with warm start, svt_mode 4) against the warm-started
    Jacobi (svt_mode 1) on the inner loop alone (random I ~ U(0,1), J ~
    N(0,1), p = 5, batches of 256): kernel time, iterations, the share of
    SVTs done by a Cayley step and the objective against svt_mode 1, for the
    eps_svd switch and for the fixed schedule svdws_every = 2; the FP64
    oracle runs problem 0 of each size with the exact SVT and with Alg. 2."""
    import numpy as np
    import torch

    import oracle as O
    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    ctx = T.Context(0)
    p, count = 5, 256
    modes = [("warm Jacobi (svt_mode 1)", dict(svt_mode=1)),
             (f"SVDWS, eps_svd {args.eps_svd:g}", dict(svt_mode=4, eps_svd=args.eps_svd)),
             ("SVDWS, every 2nd SVT", dict(svt_mode=4, svdws_every=2))]
    rows = []
    for size in (10, 50, 100):
        Is, Js = zip(*[ts.inner_problem(k, size, size, p) for k in range(count)])
        dI = torch.from_numpy(np.stack(Is)).to(dev)
        dJ = torch.from_numpy(np.stack(Js)).to(dev)
        base_obj = None
        for name, kw in modes:
            prm = T.default_params(**kw)
            ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), 8, size, size, p, prm)  # warm-up
            torch.cuda.synchronize()
            rc, res = ctx.inner_batch(dI.data_ptr(), dJ.data_ptr(), count, size, size, p, prm)
            kms = ctx.last_kernel_ms()
            iters = np.array([r["inner_iters_total"] for r in res])
            objs = np.array([r["objective"] for r in res])
            steps = np.array([r["counters"]["svdws_steps"] for r in res])
            svts = np.array([r["counters"]["svt_calls"] for r in res])
            if base_obj is None:
                base_obj = objs
            rel = np.abs(objs - base_obj) / base_obj
            row = {"size": size, "svt": name, "kernel_ms": round(kms, 2),
                   "solves_per_s": round(count / (kms * 1e-3), 1), "iters_mean": round(float(iters.mean()), 1),
                   "iters_max": int(iters.max()), "cayley_share": round(float(steps.sum() / max(svts.sum(), 1)), 3),
                   "obj_vs_mode1_mean": float(rel.mean()), "obj_vs_mode1_max": float(rel.max()),
                   "status_maxiter": int(sum(1 for r in res if r["status"] == 1))}
            rows.append(row)
            log(f"svdws {size}x{size}: {row}")
        # the oracle on problem 0: exact SVT and Alg. 2 with the same switch
        lam = 1.0 / math.sqrt(size)
        Jm = np.asarray(Js[0], np.float64).reshape(p, size * size).T
        I64 = np.asarray(Is[0], np.float64)
        Z = np.zeros_like(I64)
        opr = O.Params()
        ex = O.ladmap_inner(I64, O.Annihilator(Jm), lam, I64, Z, Z, opr)
        op = O.svdws.SvdwsSvt(eps_svd=args.eps_svd)
        ws = O.ladmap_inner(I64, O.Annihilator(Jm), lam, I64, Z, Z, opr, svt_op=op)
        oe, ow = O.objective(ex.A, ex.E, lam), O.objective(ws.A, ws.E, lam)
        rows.append({"size": size, "svt": "oracle (FP64), problem 0", "iters_exact": ex.iters,
                     "iters_svdws": ws.iters, "cayley_steps": op.steps, "obj_rel_diff": abs(ow - oe) / oe})
        log(f"svdws {size}x{size} oracle: {rows[-1]}")
    head = next(r for r in rows if r["size"] == 100 and r["svt"].startswith("SVDWS, eps"))
    out = {
        "metric": "LADMAP inner loop alone with the SVD with warm start: solves/s",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": head["kernel_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (I ~ U(0,1), J ~ N(0,1), p = 5)",
        "config": {"workload": "inner-loop-svdws", "value_at": "256 problems of 100x100", "eps_svd": args.eps_svd},
        "rows": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


RASL_SHAPE = dict(count=32, m=16, n=24, height=48, width=56)


def _rasl_oracle_worker(args):
    idx, prm_kw = args
    import oracle as O
    import tilt_synth as ts

    r = ts.rasl_set(idx, **RASL_SHAPE)
    t0 = time.perf_counter()
    res = O.rasl.rasl_solve(r.images, r.tau0, r.m, r.n, r.model, O.Params(**prm_kw), lam=r.lam)
    return time.perf_counter() - t0, res.tau_px


def rasl_main(args):
    """RASL variant: `--rasl-sets` independent image sets, each 32 images of
    48 x 56 with a 16 x 24 window (the data matrix is 384 x 32), affine,
    5 % corruption, planted shifts of up to 1.5 px; one fused launch
    (k_rasl, one workgroup per set).  Reports sets/s and images/s over the
    kernel time, per-set latency, the alignment error against the planted
    transforms, the roofline of k_rasl from its work counters, and the FP64
    oracle on a sample of sets (its tau compared with the device's)."""
    import numpy as np
    import torch

    import oracle as O
    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    ctx = T.Context(0)
    nsets = args.rasl_sets
    t_gen = time.perf_counter()
    sets = [ts.rasl_set(i, **RASL_SHAPE) for i in range(nsets)]
    log(f"generated {nsets} RASL sets in {time.perf_counter() - t_gen:.1f}s")
    imgs = [torch.from_numpy(r.images).to(dev) for r in sets]
    descs = [dict(images=im.data_ptr(), image_stride=r.height * r.width, height=r.height, width=r.width,
                  row_stride=r.width, count=r.count, m=r.m, n=r.n, model=r.model, tau0=r.tau0)
             for im, r in zip(imgs, sets)]
    As = [torch.zeros((r.count, r.m, r.n), dtype=torch.float32, device=dev) for r in sets]
    Es = [torch.zeros_like(a) for a in As]
    lam = sets[0].lam
    prm = T.default_params(lam=lam, max_outer=args.rasl_max_outer)
    if args.copy_probe_mib > 0:
        nel = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    for w in range(args.warmup):
        ctx.rasl_solve_batch(descs[:min(8, nsets)], prm)
    torch.cuda.synchronize()
    kms, walls, res = [], [], None
    for step in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = ctx.rasl_solve_batch(descs, prm, [a.data_ptr() for a in As], [e.data_ptr() for e in Es])
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kms.append(ctx.last_kernel_ms())
        log(f"step {step}: kernel {kms[-1]:.1f} ms, wall {1000 * walls[-1]:.1f} ms, status {rc}")
    kernel_ms = float(np.mean(kms))
    lat = np.array([r["solve_ms"] for r in res])
    # alignment: corner spread of G_k^-1 tau_k around its mean, per set
    spreads = []
    for r, out in zip(sets, res):
        Ms = [np.linalg.inv(r.G_px[k]) @ out["tau"][k] for k in range(r.count)]
        M0 = np.mean(Ms, axis=0)
        a, b = (r.n - 1) / 2.0, (r.m - 1) / 2.0
        cn = np.array([[-a, -b, 1], [a, -b, 1], [a, b, 1], [-a, b, 1]]).T
        ref = M0 @ cn
        ref = ref[:2] / ref[2]
        spreads.append(max(float(np.max(np.linalg.norm((M @ cn)[:2] / (M @ cn)[2] - ref, axis=0))) for M in Ms))
    nr, nc = RASL_SHAPE["m"] * RASL_SHAPE["n"], RASL_SHAPE["count"]
    flops = 0.0
    for out in res:
        c = out["counters"]
        flops += (2.0 * nr * c["jacobi_pairs"] + 6.0 * nr * c["jacobi_rotations"] + 4.0 * nc * nr * c["recon_rows"]
                  + (20.0 + 8.0 * sets[0].model) * nc * nr * c["inner_iters"])
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    fma_peak = measure_peak(T, torch, "fp32_fma", reps=3, nbytes=8 << 20)
    roofline = {"kernel": "k_rasl (whole RASL solves, one workgroup per set)", "bound": "alu",
                "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": (profiled_traffic("k_rasl_rasl256x32x16x24.md")
                            if nsets == 256 and args.rasl_max_outer == 10 else None),
                "kernel_ms": round(kernel_ms, 2), "flops_per_launch": flops,
                "peak_measured": round(fma_peak, 2), "frac_of_measured": round(achieved / fma_peak, 4)}
    cpu = None
    if not args.no_cpu:
        import multiprocessing as mp

        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        sample = list(range(min(args.cpu_sample, nsets)))
        log(f"cpu baseline: FP64 oracle on {len(sample)} sets, one process and one BLAS thread each")
        prm_kw = dict(lam=lam, eps1=prm.eps1, eps2=prm.eps2, eps_outer=prm.eps_outer, mu0=prm.mu0, rho0=prm.rho0,
                      mu_max=prm.mu_max, max_inner=prm.max_inner, max_outer=prm.max_outer)
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(len(sample)) as pool:
            outs = pool.map(_rasl_oracle_worker, [(i, prm_kw) for i in sample])
        wall = time.perf_counter() - t0
        cpu_s = sum(o[0] for o in outs)
        tau_err = max(O.tau_rel_err(res[i]["tau"][k], outs[j][1][k], RASL_SHAPE["m"], RASL_SHAPE["n"])
                      for j, i in enumerate(sample) for k in range(RASL_SHAPE["count"]))
        cpu = {"value": round(len(sample) / wall, 4), "unit": "sets/s", "cores": len(sample), "kind": "oracle",
               "sample": f"{len(sample)} of the {nsets} sets (indices {sample}), FP64 NumPy oracle with the same "
                         f"parameters, one process per set; {cpu_s:.1f} CPU-s in {wall:.1f} s wall",
               "max_tau_rel_err_vs_gpu": tau_err}
    out = {
        "metric": "RASL image sets aligned/s",
        "value": round(nsets / (kernel_ms * 1e-3), 3),
        "unit": "sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(kernel_ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (one low-rank texture per set seen through planted per-image transforms, 5 % corruption)",
        "config": {"workload": f"rasl-{nsets}x{RASL_SHAPE['count']}x{RASL_SHAPE['m']}x{RASL_SHAPE['n']}-affine",
                   "sets": nsets, **RASL_SHAPE, "model": "affine", "max_outer": prm.max_outer,
                   "lambda": lam, "images_per_s": round(nsets * RASL_SHAPE["count"] / (kernel_ms * 1e-3), 1)},
        "latency_ms": {"set_solve_p50": round(float(np.percentile(lat, 50)), 2),
                       "set_solve_p99": round(float(np.percentile(lat, 99)), 2)},
        "alignment_px": {"p50": round(float(np.median(spreads)), 4), "max": round(float(np.max(spreads)), 4)},
        "work": {"inner_mean": float(np.mean([r["inner_iters_total"] for r in res])),
                 "status_ok": int(sum(1 for r in res if r["status"] >= 0))},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def serve_main(args):
    """Serving workload: requests arrive as a Poisson process and go through
    tilt_submit / tilt_poll (continuous batching on one GPU).  First the
    saturation throughput (all requests submitted at once), then arrival
    rates of 0.25, 0.5, 0.75 and 0.9 times it; latency is arrival -> result
    seen by the polling host thread."""
    import numpy as np
    import torch

    import paper_1205_5351_amd as T
    import tilt_synth as ts

    dev = torch.device("cuda:0")
    names = ts.config_names()
    wl = args.workload if args.workload != 1 else 4
    patches = ts.make_config(wl, count=args.serve_requests)
    imgs = [torch.from_numpy(p.image).to(dev) for p in patches]
    probs = [T.make_problem(im.data_ptr(), p.height, p.width, p.width, p.m, p.n, p.model, p.tau0)
             for im, p in zip(imgs, patches)]
    outA = [torch.zeros((p.m, p.n), dtype=torch.float32, device=dev) for p in patches]
    outE = [torch.zeros((p.m, p.n), dtype=torch.float32, device=dev) for p in patches]
    levels = args.pyramid if args.pyramid > 1 else 3
    prm = T.default_params(svt_mode=args.svt_mode, pyramid_levels=levels, max_outer=args.serve_max_outer,
                           max_inner=args.serve_max_inner)
    ctx = T.Context(0)
    torch.cuda.synchronize()

    def run(arrivals):
        """arrivals: seconds after start for request k (k cycles over the set)."""
        pending = {}
        lat, solve_ms, statuses = [], [], []
        t0 = time.perf_counter()
        nxt = 0
        last_log = t0
        while nxt < len(arrivals) or pending:
            now = time.perf_counter() - t0
            while nxt < len(arrivals) and arrivals[nxt] <= now:
                k = nxt % len(probs)
                t = ctx.submit(probs[k], prm, outA[k].data_ptr(), outE[k].data_ptr())
                pending[t] = arrivals[nxt]
                nxt += 1
            for t in list(pending):
                out = ctx.poll(t)
                if out is not None:
                    done = time.perf_counter() - t0
                    lat.append(1000.0 * (done - pending.pop(t)))
                    solve_ms.append(out[1]["solve_ms"])
                    statuses.append(out[0])
            if time.perf_counter() - last_log > 20:
                log(f"  {len(lat)} done, {len(pending)} in flight")
                last_log = time.perf_counter()
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        return wall, np.array(lat), np.array(solve_ms), statuses

    n = len(probs)
    log(f"serving: {n} requests of '{names[wl]}', {levels} pyramid levels")
    run([0.0] * min(n, 16))  # warm-up
    wall, lat, sms, st = run([0.0] * n)
    sat = n / wall
    log(f"saturation: {sat:.2f} requests/s (all {n} submitted at once, {wall:.1f} s)")
    rng = np.random.default_rng(20250)
    rates = []
    for f in (0.25, 0.5, 0.75, 0.9):
        lam_arr = f * sat
        count = max(8, int(lam_arr * args.serve_seconds))
        arrivals = np.cumsum(rng.exponential(1.0 / lam_arr, size=count)).tolist()
        w, l, s_ms, stt = run(arrivals)
        rates.append({"load": f, "arrival_per_s": round(lam_arr, 3), "requests": count,
                      "patches_per_s": round(count / w, 3),
                      "latency_p50_ms": round(float(np.percentile(l, 50)), 1),
                      "latency_p99_ms": round(float(np.percentile(l, 99)), 1),
                      "solve_p50_ms": round(float(np.percentile(s_ms, 50)), 1),
                      "ok": int(sum(1 for x in stt if x >= 0))})
        log(f"load {f}: {rates[-1]}")
    headline = next(r for r in rates if r["load"] == 0.75)
    out = {
        "metric": METRIC,
        "value": round(sat, 3),
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": len(rates),
        "warmup": 1,
        "ms_per_step": round(1000.0 * wall / n, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": names[wl], "requests": n, "pyramid_levels": levels,
                   "max_outer_per_level": args.serve_max_outer,
                   "max_inner_per_outer": args.serve_max_inner,
                   "svt": "cold" if args.svt_mode == 0 else "warm",
                   "value_is": "saturation throughput (all requests in flight)"},
        "latency_ms": {"p50_at_0.75": headline["latency_p50_ms"], "p99_at_0.75": headline["latency_p99_ms"],
                       "saturation_p50": round(float(np.percentile(lat, 50)), 1),
                       "saturation_p99": round(float(np.percentile(lat, 99)), 1)},
        "rates": rates,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
