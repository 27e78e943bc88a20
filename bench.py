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


def f_join(n):
    """One join of two segment summaries: P0_b Psi_a, P0_b Gam_a' (2 n^3 each),
    Gauss-Jordan with 2n+1 right-hand sides (~5.3 n^3), Gam_a X1, Gam_a X3,
    Psi_a Gam_b, X3' W (2 n^3 each)."""
    return 17.3 * n ** 3


def seg_lengths(T, J):
    L, e = divmod(T, J)
    return [L + (1 if j < e else 0) for j in range(J)]


def kernel_flops(n, m, T, J):
    lens = seg_lengths(T, J)
    mid = sum(lens[:-1])
    # phase 2: the serial chain does J - 1 linking steps; the scan (J >= 8)
    # does sum over rounds of (J - dist) joins of ~17.3 n^3 flops each plus
    # J - 1 link maps
    if J >= 8 and n <= 64:
        joins, dist = 0, 1
        while dist < J:
            joins += J - dist
            dist *= 2
        f2 = joins * f_join(n) + (J - 1) * f_link(n)
    else:
        f2 = (J - 1) * f_link(n)
    return {
        1: mid * (f_ric(n, m) + f_dual(n, m)) + lens[-1] * f_ric(n, m),
        2: f2,
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
    ap.add_argument("--workload", default="large", choices=["small", "large", "batched", "diff"])
    ap.add_argument("--no-batched-summary", action="store_true",
                    help="skip the short batched-workload measurement added to the single-instance line")
    ap.add_argument("--serial-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate budget of the oracle CPU-baseline sample (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of known size (for hardware-counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus %d is not supported "
              "(the batched instances and the segments of one instance would shard across GPUs)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1809_06360_amd as L
    from synthetic import WORKLOADS, make_instance

    if not os.path.exists(L.LIB_PATH):
        log("library not built; building")
        from paper_1809_06360_amd import build as hip_build
        hip_build.build()

    if args.workload == "batched":
        print(json.dumps(run_batched(args, WORKLOADS["batched"])), flush=True)
        return
    if args.workload == "diff":
        print(json.dumps(run_diff(args, WORKLOADS["diff"])), flush=True)
        return

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

    step()
    torch.cuda.synchronize()
    info = int(out["info"].item())
    gpu_out = {k: out[k].cpu().numpy() for k in ("K", "k", "P", "p", "x", "u", "lam")}
    rel = None

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

    # mixed precision (FP32 matrix-core bulk products, FP64 factorizations and
    # linking solve) on the same inputs and segments
    mout = {k: torch.empty_like(v) for k, v in out.items()}
    mprob = L._problem(data, mout, J)
    mopts = L.options("mixed", "parallel")
    mws_bytes = L.lqr_workspace_size(ctypes.byref(mprob), 1, mopts)
    mws = torch.empty(mws_bytes, dtype=torch.uint8, device=dev)
    for _ in range(max(1, args.warmup)):
        L.lqr_solve(mprob, mopts, mws.data_ptr(), mws_bytes, sh)
    torch.cuda.synchronize()
    me0, me1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    me0.record(stream)
    for _ in range(K):
        L.lqr_solve(mprob, mopts, mws.data_ptr(), mws_bytes, sh)
    me1.record(stream)
    torch.cuda.synchronize()
    mixed_ms = me0.elapsed_time(me1) / K
    mixed_out = {k: mout[k].cpu().numpy() for k in ("K", "k", "P", "p", "x", "u", "lam")}
    log("mixed precision %.3f ms/solve" % mixed_ms)

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
    # Phases 1 and 3 are one kernel each. Phase 2 is one kernel when it links
    # the segments serially (J < 8) and a sequence of about log2(J) + 3 kernels
    # otherwise; only a single kernel can carry the roofline, so a phase-2
    # sequence is reported next to it instead.
    tree = J >= 8 and n <= 64
    cands = {p: v for p, v in kern_ms.items() if not (tree and p == 2)}
    dom = max(cands, key=cands.get)
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
    if tree:
        roofline["phase2_sequence"] = {
            "kernels": "k_link_init, %d x k_link_combine, k_link_maps, k_link_forward"
                       % max(1, (J - 1).bit_length()),
            "ms": kern_ms[2], "flops": flops[2]}

    cpu = None
    mixed_rel = None
    if args.cpu_seconds > 0:
        # CPU baseline: the oracle timed on the host; its first solution also
        # gives the relative error of the timed GPU configuration
        import oracle
        ref = oracle.solve(prob_np)
        rel = {k: float(np.linalg.norm(gpu_out[k] - ref[k]) / np.linalg.norm(ref[k])) for k in gpu_out}
        mixed_rel = {k: float(np.linalg.norm(mixed_out[k] - ref[k]) / np.linalg.norm(ref[k]))
                     for k in mixed_out}
        log("max rel err vs oracle %.2e (info %d); mixed %.2e" % (max(rel.values()), info,
                                                                  max(mixed_rel.values())))
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
        "mixed_precision": {"ms_per_solve": mixed_ms, "solves_per_s": 1e3 / mixed_ms,
                            "rel_err": mixed_rel,
                            "note": "same instance and segments; FP32 matrix-core bulk products "
                                    "with FP32 accumulation, FP64 Cholesky, gains and linking solve"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if not args.no_batched_summary:
        bargs = argparse.Namespace(steps=5, warmup=2, serial_steps=2, cpu_seconds=0.0)
        try:
            b = run_batched(bargs, WORKLOADS["batched"])
            result["batched"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "config", "phased",
                                                   "serial_gpu", "speedup_vs_serial_gpu", "max_rel_err",
                                                   "roofline")}
        except Exception as exc:  # the headline line must still be printed
            result["batched"] = {"error": repr(exc)}
        try:
            dres = run_diff(bargs, WORKLOADS["diff"])
            result["differentiable"] = {k: dres[k] for k in ("value", "unit", "ms_per_step", "config",
                                                           "forward_ms", "backward_ms", "fp32",
                                                           "roofline")}
        except Exception as exc:
            result["differentiable"] = {"error": repr(exc)}
    print(json.dumps(result), flush=True)


def run_diff(args, w):
    """The differentiable workload: forward solve of the whole batch (one
    persistent launch) and the adjoint (lqr_backward: adjoint solve + gradient
    outer products) for the loss sum |x|^2 + |u|^2, timed with HIP events on
    the launch stream; the CPU baseline is the oracle's forward + adjoint on a
    sample of the instances."""
    import numpy as np
    import torch

    import paper_1809_06360_amd as L
    from synthetic import make_instance

    dev = torch.device("cuda:0")
    log("differentiable workload %s: %d instances" % (w.name, w.batch))
    probs = [make_instance(w.cfg, i, *w.dims[i]) for i in range(w.batch)]
    datas = [{k: torch.from_numpy(v).to(dev) for k, v in p.items()} for p in probs]
    keys = ("A", "B", "c", "Q", "q", "R", "r", "x0")
    stream = torch.cuda.current_stream(dev)
    K = args.steps

    def graphs(ds, precision):
        """Forward and adjoint calls captured in two graphs (each with its own
        workspace, whose plan the eager calls upload), so the timed region is
        device work only."""
        outs, ws_f = L.solve_batched(ds, precision=precision, with_chol=True)
        gx = [2.0 * o["x"] for o in outs]
        gu = [2.0 * o["u"] for o in outs]
        gs = L.backward(ds, outs, gx, gu, which=keys)
        ws_b = gs[0]["_workspace"]
        torch.cuda.synchronize()
        gf, gb = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(gf):
            L.solve_batched(ds, outputs=outs, workspace=ws_f, precision=precision)
        with torch.cuda.graph(gb):
            L.backward(ds, outs, gx, gu, which=keys, workspace=ws_b, outputs=gs)
        for _ in range(args.warmup):
            gf.replay()
            gb.replay()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
        t0 = time.perf_counter()
        for s_ in range(K):
            ev[s_][0].record(stream)
            gf.replay()
            ev[s_][1].record(stream)
            gb.replay()
            ev[s_][2].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / K
        f = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        b = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        return wall, f, b

    ms, fwd, bwd = graphs(datas, "fp64")
    # the same in the FP32 precision mode (float arrays; float matrix-core
    # products, double factorizations; adjoint in double on staged arrays)
    d32 = [{k: v.float() for k, v in d.items()} for d in datas]
    _, fwd32, bwd32 = graphs(d32, "fp32")
    log("fp64 forward %.3f ms backward %.3f ms; fp32 forward %.3f ms backward %.3f ms"
        % (fwd, bwd, fwd32, bwd32))
    n, m, T = w.dims[0]
    # the adjoint's algorithmic HBM bytes (FP64): read A, B, K, P, chol, x, u,
    # lam and the upstream gradients; write the adjoint solution scratch and
    # the gradients of A, B, c, Q, q, R, r, x0
    rd = T * (n * n + n * m + m * n + m * m) + (T + 1) * n * n + 3 * (T + 1) * n + 2 * T * m
    wr = (T * (n * n + n * m + n + m * m + m) + (T + 1) * (n * n + n) + n) + 3 * (T + 1) * n + 2 * T * m
    bbytes = 8.0 * w.batch * (rd + wr)
    achieved = bbytes / (bwd * 1e-3) / 1e9
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        t = time.perf_counter()
        done = 0
        while done < w.batch and time.perf_counter() - t < args.cpu_seconds:
            sol = oracle.solve(probs[done])
            oracle.backward(probs[done], sol, 2.0 * sol["x"], 2.0 * sol["u"])
            done += 1
        dt = time.perf_counter() - t
        cpu = {"value": done / dt, "unit": "forward+adjoint solves/s", "cores": 1, "kind": "oracle",
               "sample": "forward + adjoint of the first %d instances on one host core, %.1f s" % (done, dt)}
    return {
        "metric": METRIC, "value": w.batch * 1e3 / ms, "unit": "forward+adjoint solves/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "instances": w.batch, "n": n, "m": m, "T": T,
                   "loss": "sum |x_t|^2 + |u_t|^2", "gradients": list(keys)},
        "forward_ms": fwd, "backward_ms": bwd,
        "fp32": {"forward_ms": fwd32, "backward_ms": bwd32,
                 "solves_per_s": w.batch * 1e3 / (fwd32 + bwd32),
                 "note": "float inputs/outputs staged as double in the workspace; float "
                         "matrix-core products, double factorizations; adjoint in double"},
        "roofline": {"kernel": "lqr_backward (k_adjoint_solve + k_adjoint_grad)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel_ms": bwd},
        "cpu_baseline": cpu,
    }


def batch_flops(dims, segs):
    tot = 0.0
    for (n, m, T), J in zip(dims, segs):
        f = kernel_flops(n, m, T, J)
        tot += f[1] + f[2] + f[3] if J > 1 else f["serial"]
    return tot


def run_batched(args, w):
    """The batched workload: all instances in one persistent launch captured
    in a HIP graph (timed as graph replays), against the three-launch phased
    path and the plain serial kernel on the same instances."""
    import numpy as np
    import torch

    import paper_1809_06360_amd as L
    from synthetic import make_instance

    dev = torch.device("cuda:0")
    log("batched workload %s: %d instances" % (w.name, w.batch))
    probs = [make_instance(w.cfg, i, *w.dims[i]) for i in range(w.batch)]
    datas = [{k: torch.from_numpy(v).to(dev) for k, v in p.items()} for p in probs]
    segs, est = L.plan_segments(w.dims)
    outs, ws = L.solve_batched(datas)
    torch.cuda.synchronize()
    infos = [int(o["info"].item()) for o in outs]
    keys = ("K", "k", "P", "p", "x", "u", "lam")
    first = [{k: outs[i][k].cpu().numpy() for k in keys} for i in range(min(w.batch, 64))]
    rel = None
    stream = torch.cuda.current_stream(dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        L.solve_batched(datas, outputs=outs, workspace=ws)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    K = args.steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(K):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / K
    kern = e0.elapsed_time(e1) / K
    log("persistent graph: %.3f ms/step (events %.3f ms)" % (ms, kern))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ph_ms = timed(lambda: L.solve_batched(datas, outputs=outs, workspace=ws, phased=True), max(2, K // 2))
    se_ms = timed(lambda: L.solve_batched(datas, outputs=outs, workspace=ws, algo="serial"),
                  args.serial_steps)
    log("phased %.3f ms/step, serial kernel %.3f ms/step" % (ph_ms, se_ms))
    flops = batch_flops(w.dims, segs)
    achieved = flops / (kern * 1e-3) / 1e12
    cpu = None
    if args.cpu_seconds > 0:
        # CPU baseline: the oracle on the first instances of the batch, whose
        # solutions also give the relative error of the GPU results
        import oracle
        t = time.perf_counter()
        done, errs = 0, []
        while done < w.batch and time.perf_counter() - t < args.cpu_seconds:
            ref = oracle.solve(probs[done])
            if done < len(first):
                errs.append(max(float(np.linalg.norm(first[done][k] - ref[k]) / np.linalg.norm(ref[k]))
                                for k in keys))
            done += 1
        dt = time.perf_counter() - t
        rel = max(errs) if errs else None
        cpu = {"value": done / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "the first %d instances of the batch, serial FP64 solves on one host core, %.1f s"
                         % (done, dt)}
    steps_total = sum(T for (_, _, T) in w.dims)
    return {
        "metric": METRIC,
        "value": w.batch * 1e3 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": w.batch, "timesteps": steps_total,
                   "segments": "autotuned (%d..%d, %d in total)" % (min(segs), max(segs), sum(segs)),
                   "launch": "one persistent kernel, hipGraph replay", "predicted_ms": est / 1e3},
        "timesteps_per_s": steps_total * 1e3 / ms,
        "max_rel_err": rel,
        "info_max": max(infos),
        "phased": {"solves_per_s": w.batch * 1e3 / ph_ms, "ms_per_step": ph_ms},
        "serial_gpu": {"solves_per_s": w.batch * 1e3 / se_ms, "ms_per_step": se_ms, "kernel": "k_serial"},
        "speedup_vs_serial_gpu": se_ms / ms,
        "roofline": {"kernel": "k_persistent", "bound": "alu", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": None, "kernel_ms": kern},
        "cpu_baseline": cpu,
    }


if __name__ == "__main__":
    main()
