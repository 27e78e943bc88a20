#!/usr/bin/env python
"""Benchmark of the parallel Riccati LQR solve on one MI355X.

A step is one full solve of the workload (segment sweeps, linking solve,
rebuild and forward simulation) on inputs already resident in HBM, launched
through the C ABI on torch's current stream. The three kernels of every timed
step are bracketed by HIP events (torch.cuda.Event on that same stream) to get
per-kernel durations for the roofline of the dominant kernel. The plain serial
Riccati GPU kernel is timed on the same inputs for comparison, and the CPU
oracle on a bounded sample of the same workload for the CPU baseline.

Prints progress to stderr and ONE JSON line to stdout.
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LQR solves/s & timesteps/s, parallel vs plain Riccati on GPU, at stated rel err"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 (vector and matrix), dense
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {1: "k_phase1", 2: "k_phase2", 3: "k_phase3", "serial": "k_serial"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic work (flops, 2 per multiply-add, no symmetry exploited).
# ---------------------------------------------------------------------------
def f_ric(n, m):
    """One plain Riccati stage: P[B|A|c], B'(.), Cholesky, gains, value update."""
    return 4 * n ** 3 + 6 * n * n * m + 4 * n * m * m + m ** 3 / 3.0


def f_dual(n, m):
    """Extra work of one parametric (dual-form) stage: B'Gamma, L^{-1}B'Gamma,
    Psi, psi and Gamma updates."""
    return 2 * n ** 3 + 6 * n * n * m + 2 * n * m * m


def f_roll(n, m):
    """One forward-simulation stage: K x, A x + B u."""
    return 2 * n * n + 4 * n * m


def f_link(n):
    """One linking step: I + Psi P (2n^3), LU solve with n+1 right-hand sides
    (2/3 n^3 + 2 n^3), P F (2n^3), Gamma (P F) (2n^3)."""
    return 8.67 * n ** 3


def seg_lengths(T, J):
    L, e = divmod(T, J)
    return [L + (1 if j < e else 0) for j in range(J)]


def kernel_flops(n, m, T, J):
    lens = seg_lengths(T, J)
    mid = sum(lens[:-1])
    return {
        1: mid * (f_ric(n, m) + f_dual(n, m)) + lens[-1] * f_ric(n, m),
        2: (J - 1) * f_link(n),
        3: mid * f_ric(n, m) + T * f_roll(n, m),
        "serial": T * (f_ric(n, m) + f_roll(n, m)),
    }


def kernel_bytes(n, m, T, J):
    """Algorithmic HBM bytes per launch (FP64): inputs each phase must read and
    outputs it must write, plus the segment summaries that cross phases."""
    w = 8
    stage_in = n * n + n * m + m * m + 2 * n + m          # A, B, R, c, r (+Q, q below)
    stage_in += n * n + n                                  # Q, q
    stage_out = m * n + m + n * n + n                      # K, k, P, p
    lens = seg_lengths(T, J)
    mid = sum(lens[:-1])
    summ = 3 * n * n + 2 * n
    return {
        1: w * (T * stage_in + lens[-1] * stage_out + (J - 1) * summ),
        2: w * ((J - 1) * (summ + n * n + n) + J * (n * n + 2 * n)),
        3: w * (mid * (stage_in + stage_out) + T * (n * n + n * m + n + 2 * n + m)),
        "serial": w * (T * (stage_in + stage_out) + T * (2 * n + m)),
    }


def source_digest():
    """Hash of the kernel sources; stored with hardware-counter summaries so a
    stale traffic figure is never reported for a changed kernel."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1809_06360_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def counted_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary for this kernel and workload, if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "%s__%s__traffic.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    dig = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not dig or not val or dig.group(1) != source_digest():
        return None
    return float(val.group(1))


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["small", "large"])
    ap.add_argument("--serial-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate budget of the oracle CPU-baseline sample (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of known size (for hardware-counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the batched instances and the segments of one instance would shard across GPUs, "
              "see DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1809_06360_amd as L
    from synthetic import WORKLOADS, make_instance

    if not os.path.exists(L.LIB_PATH):
        log("library not built; building")
        from paper_1809_06360_amd import build as hip_build
        hip_build.build()

    w = WORKLOADS[args.workload]
    (n, m, T), = w.dims
    J = w.segments
    dev = torch.device("cuda:0")
    log("workload %s on %s" % (w.name, torch.cuda.get_device_name(0)))
    prob_np = make_instance(w.cfg, 0, n, m, T)
    data = {k: torch.from_numpy(v).to(dev) for k, v in prob_np.items()}
    e = lambda *s: torch.empty(*s, dtype=torch.float64, device=dev)  # noqa: E731
    out = dict(K=e(T, m, n), k=e(T, m), P=e(T + 1, n, n), p=e(T + 1, n), x=e(T + 1, n), u=e(T, m),
               lam=e(T + 1, n), info=torch.zeros(1, dtype=torch.int32, device=dev))
    prob = L._problem(data, out, J)
    opts = L.options("fp64", "parallel")
    ws_bytes = L.lqr_workspace_size(ctypes.byref(prob), 1, opts)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream

    def step():
        L.lqr_solve(prob, opts, ws.data_ptr(), ws_bytes, sh)

    # correctness gate on the timed configuration
    step()
    torch.cuda.synchronize()
    info = int(out["info"].item())
    rel = None
    if args.cpu_seconds > 0:
        import oracle
        ref = oracle.solve(prob_np)
        rel = {k: float(np.linalg.norm(out[k].cpu().numpy() - ref[k]) / np.linalg.norm(ref[k]))
               for k in ("K", "k", "P", "p", "x", "u", "lam")}
        log("max rel err vs oracle %.2e (info %d)" % (max(rel.values()), info))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        ev[s][0].record(stream)
        for ph in (1, 2, 3):
            L.lqr_solve_phase(prob, opts, ph, ws.data_ptr(), ws_bytes, sh)
            ev[s][ph].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / K
    kern_ms = {ph: float(np.mean([ev[s][ph - 1].elapsed_time(ev[s][ph]) for s in range(K)]))
               for ph in (1, 2, 3)}
    log("timed %d steps: %.3f ms/step; kernels %s" % (K, ms_per_step,
                                                      {KERNEL_NAMES[p]: round(v, 4) for p, v in kern_ms.items()}))

    # plain serial Riccati kernel on the same inputs
    sopts = L.options("fp64", "serial")
    sprob = L._problem(data, out, 0)
    sws_bytes = L.lqr_workspace_size(ctypes.byref(sprob), 1, sopts)
    sws = torch.empty(max(sws_bytes, 256), dtype=torch.uint8, device=dev)
    L.lqr_solve(sprob, sopts, sws.data_ptr(), sws_bytes, sh)
    torch.cuda.synchronize()
    se0, se1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    se0.record(stream)
    for _ in range(args.serial_steps):
        L.lqr_solve(sprob, sopts, sws.data_ptr(), sws_bytes, sh)
    se1.record(stream)
    torch.cuda.synchronize()
    serial_ms = se0.elapsed_time(se1) / args.serial_steps
    log("serial kernel %.3f ms/solve" % serial_ms)

    if args.copy_calibration:
        a = torch.empty(1 << 25, dtype=torch.float64, device=dev)   # 256 MiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (a.numel() * 8, b.numel() * 8))

    flops = kernel_flops(n, m, T, J)
    bytes_ = kernel_bytes(n, m, T, J)
    dom = max(kern_ms, key=kern_ms.get)
    dom_ms = kern_ms[dom]
    achieved = flops[dom] / (dom_ms * 1e-3) / 1e12
    traffic = counted_traffic(KERNEL_NAMES[dom], args.workload)
    roofline = {
        "kernel": KERNEL_NAMES[dom],
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": traffic,
        "algorithmic_bytes": bytes_[dom],
        "kernel_ms": dom_ms,
    }

    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        t = time.perf_counter()
        oracle.solve(prob_np, with_lam=False)
        one = time.perf_counter() - t
        reps = max(1, int(args.cpu_seconds / max(one, 1e-6)))
        t = time.perf_counter()
        for _ in range(reps):
            oracle.solve(prob_np, with_lam=False)
        dt = time.perf_counter() - t
        cpu = {"value": reps / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "%d full serial FP64 solves of the same instance (n=%d, m=%d, T=%d) "
                         "on one host core, %.1f s" % (reps, n, m, T, dt)}
        log("cpu oracle %.3f solves/s" % cpu["value"])

    solves_per_s = 1e3 / ms_per_step
    result = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "m": m, "T": T, "segments": J, "instances": 1},
        "timesteps_per_s": solves_per_s * T,
        "max_rel_err": None if rel is None else max(rel.values()),
        "rel_err": rel,
        "info": info,
        "kernel_ms": {KERNEL_NAMES[p]: v for p, v in kern_ms.items()},
        "serial_gpu": {"solves_per_s": 1e3 / serial_ms, "ms_per_solve": serial_ms,
                       "kernel": "k_serial"},
        "speedup_vs_serial_gpu": serial_ms / ms_per_step,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
