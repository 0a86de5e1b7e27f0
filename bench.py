#!/usr/bin/env python
"""Benchmark of the dense Pauli decomposition hot path on one MI355X.

Workload: the n = 14 dense matrix (16384 x 16384, complex128, real and
imaginary parts iid N(0, 1), seed 0) -- the headline configuration -- and its
complex64 cast.  A "step" is one full pauli_decompose call computing all
4^14 = 268,435,456 coefficients, input resident in HBM.  The primary value
is the float64 (complex128 -> complex128) path; the complex64 path is
reported beside it with its error against the float64 oracle.

Prints ONE JSON line:  metric, value (GCoeff/s), ms_per_step, the roofline
of the dominant kernel (HIP-event timing of that kernel alone, algorithmic
bytes = read A once + write c once), the oracle timed on this host's cores
on a bounded sample (cpu_baseline), and the sampled error against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, 8 TB/s


def _kernel_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_11644_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, n: int, dtype: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    rec = data.get("%s/n%d/%s" % (kernel, n, dtype))
    if not rec or rec.get("kernel_hash") != _kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def _time_calls(fn, steps: int, warmup: int, stream) -> float:
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps  # ms per call


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=14)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle sample time")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; the decomposition shards by X-pattern group "
              "with no communication, so more GPUs are not measured here (--gpus 1).", file=sys.stderr)
        return 2

    import torch

    sys.path.insert(0, ROOT)
    import paper_2403_11644_amd as ptd
    from paper_2403_11644_amd import _native, api
    import synth

    n = args.n
    N = 1 << n
    ncoef = float(N) * N
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    t_gen = time.time()
    A_host = synth.dense(n, seed=0)  # complex128, re then im, N(0, 1)
    A = torch.from_numpy(A_host).to(dev)
    A64 = A.to(torch.complex64)  # the cast is not part of the timed step
    gen_s = time.time() - t_gen
    out128 = torch.empty((N, N), dtype=torch.complex128, device=dev)
    out64 = torch.empty((N, N), dtype=torch.complex64, device=dev)

    ms128 = _time_calls(lambda: ptd.decompose(A, out=out128), args.steps, args.warmup, stream)
    ms64 = _time_calls(lambda: ptd.decompose(A64, out=out64), args.steps, args.warmup, stream)

    # per-kernel timing of the two passes (same launches as inside the call)
    L = _native.lib()
    kern = {}
    for dtname, Ain, out in (("c128", A, out128), ("c64", A64, out64)):
        code = api._dtype_code(Ain.dtype)
        for stage, kname in ((1, "k_tile_fwd"), (2, "k_high_fwd")):
            def fn(stage=stage, Ain=Ain, out=out, code=code):
                _native.check(L.ptd_debug_decompose_stage(n, code, 0, api._ptr(Ain), N, api._ptr(out), stage,
                                                          api._stream_handle(dev, None)), "stage")
            kern[(dtname, kname)] = _time_calls(fn, args.steps, 2, stream)
    # leave the outputs holding the full results again
    ptd.decompose(A, out=out128)
    ptd.decompose(A64, out=out64)
    torch.cuda.synchronize()

    # plain device copy of the same bytes (practical bandwidth ceiling)
    cpy = torch.empty_like(A)
    ms_copy = _time_calls(lambda: cpy.copy_(A), 5, 2, stream)
    copy_gbps = 2 * A.numel() * 16 / (ms_copy * 1e-3) / 1e9
    del cpy

    # error against the oracle on sampled strings, and the float64 Parseval residual
    from oracle import oracle as O

    xs, zs = synth.sample_strings(n, 2000, seed=5)
    want = O.coeffs(A_host, xs, zs)
    ix = torch.from_numpy(xs.astype(np.int64)).to(dev)
    iz = torch.from_numpy(zs.astype(np.int64)).to(dev)
    got128 = out128[ix, iz].cpu().numpy()
    got64 = out64[ix, iz].cpu().numpy().astype(np.complex128)

    def rel(g, w):
        return float(np.linalg.norm(g - w) / np.linalg.norm(w))

    err128, err64 = rel(got128, want), rel(got64, want)
    _, _, pars128 = ptd.parseval(A, out128)
    _, _, pars64 = ptd.parseval(A64, out64)

    # CPU baseline: the oracle on whole X-pattern rows of the same matrix
    cpu = None
    if not args.no_cpu_baseline:
        threads = O.default_threads()
        t0 = time.time()
        O.rows(A_host, np.arange(threads, dtype=np.uint32), nthreads=threads)
        t_cal = time.time() - t0
        rows = max(threads, int(args.cpu_seconds / max(t_cal, 1e-3)) * threads)
        rows = min(rows, N)
        xs_rows = np.random.default_rng(6).choice(N, rows, replace=False).astype(np.uint32)
        t0 = time.time()
        O.rows(A_host, xs_rows, nthreads=threads)
        t_cpu = time.time() - t0
        cpu = {"value": rows * N / t_cpu / 1e9, "unit": "GCoeff/s", "cores": threads, "kind": "oracle",
               "sample": "%d of %d X-pattern rows (all %d strings each) of the n=%d matrix, %.1f s; "
                         "full n=%d run extrapolates to %.0f s" % (rows, N, N, n, t_cpu, n, t_cpu * N / rows)}

    bytes128 = 32.0 * ncoef  # read A (16 B) + write c (16 B) per coefficient
    bytes64 = 16.0 * ncoef
    dom = max(("k_tile_fwd", "k_high_fwd"), key=lambda k: kern[("c128", k)])
    dom_ms = kern[("c128", dom)]
    # each pass of the two-pass schedule reads and writes 4^n complex values
    dom_bytes = 32.0 * ncoef
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    gcoef128 = ncoef / (ms128 * 1e-3) / 1e9
    gcoef64 = ncoef / (ms64 * 1e-3) / 1e9
    line = {
        "metric": "Pauli GCoeff/s + % HBM roofline, n=14 dense; complex64 vs FP64 at stated error",
        "value": round(gcoef128, 3),
        "unit": "GCoeff/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms128, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dense n=%d (%dx%d) complex128 A, re/im iid N(0,1) seed 0; all 4^%d "
                               "coefficients per step" % (n, N, N, n), "n": n, "parallelism": "none"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": _traffic(dom, n, "c128"),
                     "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": round(dom_ms, 4)},
        "path_hbm_frac": round(bytes128 / (ms128 * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "err_rel_sampled": err128,
        "parseval_residual": pars128,
        "complex64": {"value": round(gcoef64, 3), "unit": "GCoeff/s", "ms_per_step": round(ms64, 4),
                      "path_hbm_frac": round(bytes64 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                      "err_rel_sampled_vs_f64_oracle": err64, "parseval_residual": pars64,
                      "speedup_vs_f64": round(ms128 / ms64, 3)},
        "kernels_ms": {"%s/%s" % k: round(v, 4) for k, v in kern.items()},
        "copy_GBps": round(copy_gbps, 1),
        "cpu_baseline": cpu,
        "input_gen_s": round(gen_s, 1),
        "kernel_hash": _kernel_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
