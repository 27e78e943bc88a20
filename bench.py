#!/usr/bin/env python
"""Benchmark of the parallel Riccati LQR solve on one MI355X.

A step is one full solve of the workload (segment sweeps, linking solve,
rebuild and forward simulation) on inputs already resident in HBM, launched
through the C ABI on torch's current stream. The launches of every timed step
are bracketed by HIP events (torch.cuda.Event on that same stream) to get
per-phase durations for the roofline of the dominant kernel. The plain serial
Riccati GPU kernel is timed on the same inputs for comparison, and the CPU
oracle on a bounded sample of the same workload for the CPU baseline; the
oracle's solutions also give the relative error of every output.

The headline line is the large workload (n=48, m=24, T=1024, J=64, FP64);
the line also carries the small, mixed-precision (n=128, m=64, T=2048,
J=128), batched (256 uneven instances) and differentiable (512 x forward +
adjoint) workloads as sub-objects. `--workload X` prints the line of one
workload alone.

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
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 (vector and matrix), dense
HBM_PEAK_GBS = 8000.0
OUTS = ("K", "k", "P", "p", "x", "u", "lam")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_info():
    """Host cores and CPU model, recorded with every CPU baseline."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count() or 1, "cpu_model": model}


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
    """One linking step of the method (eliminating one boundary): I + Psi P
    (2n^3), LU solve with n+1 right-hand sides (2/3 n^3 + 2 n^3), P F (2n^3),
    Gamma (P F) (2n^3)."""
    return 8.67 * n ** 3


def f_join(n, exact):
    """One join of two segment summaries in the logarithmic-depth scan:
    P0_b Psi_a, the inverse (or elimination) of M, Gamma_a M^{-1}, the P0
    update, and unless the right summary is exact also Psi_a Gamma_b,
    M^{-T}(.), Gamma_b and Psi updates (~17.3 n^3; ~9.3 n^3 when exact)."""
    return (9.3 if exact else 17.3) * n ** 3


def seg_lengths(T, J):
    L, e = divmod(T, J)
    return [L + (1 if j < e else 0) for j in range(J)]


def uses_scan(n, J):
    """Whether the single-instance linking solve is the logarithmic-depth scan
    (large-state path: always; otherwise from 8 segments on)."""
    return n > 64 or J >= 8


def scan_joins(J):
    full = exact = 0
    dist = 1
    while dist < J:
        for j in range(J - dist):
            if j + 2 * dist - 1 >= J - 1:
                exact += 1
            else:
                full += 1
        dist *= 2
    return full, exact


def kernel_flops(n, m, T, J):
    lens = seg_lengths(T, J)
    mid = sum(lens[:-1])
    if uses_scan(n, J):
        full, exact = scan_joins(J)
        f2 = full * f_join(n, False) + exact * f_join(n, True) + (J - 1) * 6.0 * n ** 3
    else:
        f2 = (J - 1) * f_link(n)
    return {
        1: mid * (f_ric(n, m) + f_dual(n, m)) + lens[-1] * f_ric(n, m),
        2: f2,
        "2_method": (J - 1) * f_link(n),
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


def rel_errors(got, ref, keys=OUTS):
    import numpy as np
    return {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])) for k in keys
            if k in got and k in ref}


def oracle_pool(fn, items, workers):
    """fn over items on `workers` host threads (the oracle's C calls release
    the GIL, so each thread runs one serial solve at a time)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


# ---------------------------------------------------------------------------
# Single-instance workloads (small, large, mixed)
# ---------------------------------------------------------------------------
def run_single(args, key, steps, warmup, serial_steps, cpu_seconds, with_mixed_leg=False):
    import numpy as np
    import torch

    import paper_1809_06360_amd as L
    from synthetic import WORKLOADS, make_instance

    w = WORKLOADS[key]
    (n, m, T), = w.dims
    J = w.segments
    prec = w.precision
    dev = torch.device("cuda:0")
    log("workload %s on %s" % (w.name, torch.cuda.get_device_name(0)))
    t = time.perf_counter()
    prob_np = make_instance(w.cfg, 0, n, m, T)
    log("inputs generated in %.1f s" % (time.perf_counter() - t))
    data = {k: torch.from_numpy(v).to(dev) for k, v in prob_np.items()}
    e = lambda *s: torch.empty(*s, dtype=torch.float64, device=dev)  # noqa: E731
    out = dict(K=e(T, m, n), k=e(T, m), P=e(T + 1, n, n), p=e(T + 1, n), x=e(T + 1, n), u=e(T, m),
               lam=e(T + 1, n), info=torch.zeros(1, dtype=torch.int32, device=dev))
    prob = L._problem(data, out, J)
    opts = L.options(prec, "parallel")
    ws_bytes = L.lqr_workspace_size(ctypes.byref(prob), 1, opts)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    big = n > 64

    L.lqr_solve(prob, opts, ws.data_ptr(), ws_bytes, sh)
    torch.cuda.synchronize()
    info = int(out["info"].item())
    gpu_out = {k: out[k].cpu().numpy() for k in OUTS}
    for _ in range(warmup):
        L.lqr_solve(prob, opts, ws.data_ptr(), ws_bytes, sh)
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record(stream)
        for ph in (1, 2, 3):
            L.lqr_solve_phase(prob, opts, ph, ws.data_ptr(), ws_bytes, sh)
            ev[s][ph].record(stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    kern_ms = {ph: float(np.mean([ev[s][ph - 1].elapsed_time(ev[s][ph]) for s in range(steps)]))
               for ph in (1, 2, 3)}
    names = ({1: "k_big_phase1", 2: "linking sequence", 3: "k_big_phase3"} if big else
             {1: "k_small_phase1" if max(n, m) <= 16 else "k_phase1",
              2: "linking sequence" if uses_scan(n, J) else "k_phase2",
              3: "k_small_phase3" if max(n, m) <= 16 else "k_phase3"})
    log("timed %d steps: %.3f ms/step; phases %s" % (steps, ms_per_step,
                                                     {names[p]: round(v, 4) for p, v in kern_ms.items()}))

    mixed = None
    if with_mixed_leg:
        # mixed precision (FP32 matrix-core bulk products, FP64 factorizations
        # and linking solve) on the same inputs and segments
        mout = {k: torch.empty_like(v) for k, v in out.items()}
        mprob = L._problem(data, mout, J)
        mopts = L.options("mixed", "parallel")
        mws_bytes = L.lqr_workspace_size(ctypes.byref(mprob), 1, mopts)
        mws = torch.empty(mws_bytes, dtype=torch.uint8, device=dev)
        for _ in range(max(1, warmup)):
            L.lqr_solve(mprob, mopts, mws.data_ptr(), mws_bytes, sh)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            L.lqr_solve(mprob, mopts, mws.data_ptr(), mws_bytes, sh)
        b.record(stream)
        torch.cuda.synchronize()
        mixed = {"ms_per_solve": a.elapsed_time(b) / steps,
                 "out": {k: mout[k].cpu().numpy() for k in OUTS}}
        log("mixed precision %.3f ms/solve" % mixed["ms_per_solve"])

    # plain serial Riccati kernel on the same inputs
    sopts = L.options(prec, "serial")
    sout = {k: torch.empty_like(v) for k, v in out.items()}
    sprob = L._problem(data, sout, 0)
    sws_bytes = L.lqr_workspace_size(ctypes.byref(sprob), 1, sopts)
    sws = torch.empty(max(sws_bytes, 256), dtype=torch.uint8, device=dev)
    L.lqr_solve(sprob, sopts, sws.data_ptr(), sws_bytes, sh)
    torch.cuda.synchronize()
    se0, se1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    se0.record(stream)
    for _ in range(serial_steps):
        L.lqr_solve(sprob, sopts, sws.data_ptr(), sws_bytes, sh)
    se1.record(stream)
    torch.cuda.synchronize()
    serial_ms = se0.elapsed_time(se1) / serial_steps
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
    # phase 2 is a kernel sequence when it runs the scan: the roofline is
    # carried by the dominant single kernel, the sequence reported beside it
    cands = {p: v for p, v in kern_ms.items() if not (p == 2 and uses_scan(n, J))}
    dom = max(cands, key=cands.get)
    dom_ms = kern_ms[dom]
    fp32 = prec != "fp64"
    peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
    achieved = flops[dom] / (dom_ms * 1e-3) / 1e12
    roofline = {
        "kernel": names[dom] + ("<2> (FP32 matrix cores)" if big and fp32 else ""),
        "bound": "mfma" if (big or n >= 32) else "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": counted_traffic(names[dom], key),
        "algorithmic_flops": flops[dom],
        "algorithmic_bytes": bytes_[dom],
        "kernel_ms": dom_ms,
    }
    ph2 = {"ms": kern_ms[2], "method_flops": flops["2_method"], "executed_flops": flops[2],
           "method_tflops": flops["2_method"] / (kern_ms[2] * 1e-3) / 1e12,
           "executed_tflops": flops[2] / (kern_ms[2] * 1e-3) / 1e12,
           "frac_fp64_peak_executed": flops[2] / (kern_ms[2] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
           "precision": "fp64"}
    if uses_scan(n, J):
        ph2["kernels"] = ("%s%d x %s, %s, %s" % (
            "k_link_init, " if big else "", max(1, (J - 1).bit_length()),
            "k_big_link_combine" if big else "k_link_combine",
            "k_big_link_maps" if big else "k_link_maps", "k_big_link_forward" if big else "k_link_forward"))
    roofline["phase2_sequence"] = ph2

    rel = None
    cpu = None
    mixed_rel = None
    if cpu_seconds > 0:
        import oracle
        t = time.perf_counter()
        ref = oracle.solve(prob_np)
        one = time.perf_counter() - t
        rel = rel_errors(gpu_out, ref)
        if mixed is not None:
            mixed_rel = rel_errors(mixed["out"], ref)
        log("max rel err vs oracle %.2e (info %d)%s" % (
            max(rel.values()), info, "" if mixed_rel is None else "; mixed %.2e" % max(mixed_rel.values())))
        reps = max(1, int(cpu_seconds / max(one, 1e-6))) if one < cpu_seconds else 0
        dt, done = one, 1
        if reps:
            t = time.perf_counter()
            for _ in range(reps):
                oracle.solve(prob_np, with_lam=False)
            dt, done = time.perf_counter() - t, reps
        cpu = dict(host_info(), value=done / dt, unit="solves/s", cores=1, kind="oracle",
                   sample="%d full serial FP64 solve(s) of the same instance (n=%d, m=%d, T=%d) "
                          "on one host core, %.1f s" % (done, n, m, T, dt))
        log("cpu oracle %.4f solves/s" % cpu["value"])

    solves_per_s = 1e3 / ms_per_step
    res = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32 matrix-core products, f64 factorizations"}[prec],
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "m": m, "T": T, "segments": J, "instances": 1,
                   "precision": prec},
        "timesteps_per_s": solves_per_s * T,
        "max_rel_err": None if rel is None else max(rel.values()),
        "rel_err": rel,
        "info": info,
        "phase_ms": {names[p]: v for p, v in kern_ms.items()},
        "serial_gpu": {"solves_per_s": 1e3 / serial_ms, "ms_per_solve": serial_ms,
                       "kernel": "k_big_serial" if big else
                                 "k_small_serial" if max(n, m) <= 16 else "k_serial"},
        "speedup_vs_serial_gpu": serial_ms / ms_per_step,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if mixed is not None:
        res["mixed_precision"] = {
            "ms_per_solve": mixed["ms_per_solve"], "solves_per_s": 1e3 / mixed["ms_per_solve"],
            "rel_err": mixed_rel, "max_rel_err": None if mixed_rel is None else max(mixed_rel.values()),
            "note": "same instance and segments; FP32 matrix-core bulk products with FP32 "
                    "accumulation, FP64 Cholesky, gains and linking solve"}
    return res


# ---------------------------------------------------------------------------
def run_diff(args, w, cpu_workers):
    """The differentiable workload: forward solve of the whole batch and the
    adjoint (lqr_backward: adjoint solve + gradient outer products) for the
    loss sum |x|^2 + |u|^2, each captured in a HIP graph and timed with HIP
    events on the launch stream; relative errors of x, u and every gradient
    over all instances against the oracle, which is also the CPU baseline
    (all host cores, one instance per thread)."""
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
        """Forward and adjoint captured in two graphs sharing one workspace
        (disjoint plan regions), timed as replays."""
        outs, ws = L.solve_batched(ds, precision=precision, with_chol=True)
        gx = [2.0 * o["x"] for o in outs]
        gu = [2.0 * o["u"] for o in outs]
        gs = L.backward(ds, outs, gx, gu, which=keys, workspace=ws)
        torch.cuda.synchronize()
        gf, gb = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(gf):
            L.solve_batched(ds, outputs=outs, workspace=ws, precision=precision)
        with torch.cuda.graph(gb):
            L.backward(ds, outs, gx, gu, which=keys, workspace=ws, outputs=gs)
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
        host_x = [o["x"].double().cpu().numpy() for o in outs]
        host_u = [o["u"].double().cpu().numpy() for o in outs]
        host_g = [{k: g[k].double().cpu().numpy() for k in keys} for g in gs]
        return wall, f, b, host_x, host_u, host_g

    ms, fwd, bwd, hx, hu, hg = graphs(datas, "fp64")
    d32 = [{k: v.float() for k, v in d.items()} for d in datas]
    _, fwd32, bwd32, hx32, hu32, hg32 = graphs(d32, "fp32")
    log("fp64 forward %.3f ms backward %.3f ms; fp32 forward %.3f ms backward %.3f ms"
        % (fwd, bwd, fwd32, bwd32))
    n, m, T = w.dims[0]
    rd = T * (n * n + n * m + m * n + m * m) + (T + 1) * n * n + 3 * (T + 1) * n + 2 * T * m
    wr = (T * (n * n + n * m + n + m * m + m) + (T + 1) * (n * n + n) + n) + 3 * (T + 1) * n + 2 * T * m
    bbytes = 8.0 * w.batch * (rd + wr)
    achieved = bbytes / (bwd * 1e-3) / 1e9
    cpu = rel = rel32 = None
    if args.cpu_seconds > 0:
        import oracle

        def one(p):
            sol = oracle.solve(p)
            return sol, oracle.backward(p, sol, 2.0 * sol["x"], 2.0 * sol["u"])
        t = time.perf_counter()
        refs = oracle_pool(one, probs, cpu_workers)
        dt = time.perf_counter() - t

        def worst(xs, us, gs_):
            e = 0.0
            for i, (sol, g) in enumerate(refs):
                e = max(e, float(np.linalg.norm(xs[i] - sol["x"]) / np.linalg.norm(sol["x"])),
                        float(np.linalg.norm(us[i] - sol["u"]) / np.linalg.norm(sol["u"])))
                for k in keys:
                    e = max(e, float(np.linalg.norm(gs_[i][k] - g[k]) / np.linalg.norm(g[k])))
            return e
        rel, rel32 = worst(hx, hu, hg), worst(hx32, hu32, hg32)
        log("differentiable max rel err fp64 %.2e fp32 %.2e" % (rel, rel32))
        cpu = dict(host_info(), value=w.batch / dt, unit="forward+adjoint solves/s", cores=cpu_workers,
                   kind="oracle", sample="forward + adjoint of all %d instances, one instance per "
                                         "thread on %d host threads, %.1f s" % (w.batch, cpu_workers, dt))
    return {
        "metric": METRIC, "value": w.batch * 1e3 / ms, "unit": "forward+adjoint solves/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "instances": w.batch, "n": n, "m": m, "T": T,
                   "loss": "sum |x_t|^2 + |u_t|^2", "gradients": list(keys)},
        "timesteps_per_s": w.batch * T * 1e3 / ms,
        "forward_ms": fwd, "backward_ms": bwd,
        "max_rel_err": rel,
        "fp32": {"forward_ms": fwd32, "backward_ms": bwd32, "max_rel_err": rel32,
                 "solves_per_s": w.batch * 1e3 / (fwd32 + bwd32),
                 "note": "float inputs/outputs staged as double in the workspace; at n, m <= 16 "
                         "the forward recursion runs in double (the small-size kernel), else "
                         "float matrix-core products with double factorizations; adjoint in double"},
        "roofline": {"kernel": "lqr_backward (k_adjoint_solve + k_adjoint_grad)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel_ms": bwd},
        "cpu_baseline": cpu,
    }


def batch_flops(dims, segs):
    tot = 0.0
    for (n, m, T), J in zip(dims, segs):
        f = kernel_flops(n, m, T, J)
        tot += f[1] + f["2_method"] + f[3] if J > 1 else f["serial"]
    return tot


def run_batched(args, w, cpu_workers):
    """The batched workload: all instances in one persistent launch captured
    in a HIP graph (timed as graph replays), against the three-launch phased
    path and the plain serial kernel on the same instances; relative errors
    over all instances against the oracle, which is also the CPU baseline
    (all host cores, one instance per thread)."""
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
    got = [{k: outs[i][k].cpu().numpy() for k in OUTS} for i in range(w.batch)]
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
    ms = (time.perf_counter() - t0) * 1e3 / K
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
    cpu = rel = None
    if args.cpu_seconds > 0:
        import oracle
        t = time.perf_counter()
        refs = oracle_pool(oracle.solve, probs, cpu_workers)
        dt = time.perf_counter() - t
        rel = max(max(rel_errors(got[i], refs[i]).values()) for i in range(w.batch))
        log("batched max rel err over all instances %.2e" % rel)
        cpu = dict(host_info(), value=w.batch / dt, unit="solves/s", cores=cpu_workers, kind="oracle",
                   sample="all %d instances, serial FP64 solves, one instance per thread on %d host "
                          "threads, %.1f s" % (w.batch, cpu_workers, dt))
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
        "roofline": {"kernel": "k_persistent", "bound": "mfma", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": None, "kernel_ms": kern},
        "cpu_baseline": cpu,
    }


SUB_KEYS = ("value", "unit", "ms_per_step", "timesteps_per_s", "config", "max_rel_err", "rel_err", "info",
            "info_max", "phase_ms", "phased", "serial_gpu", "speedup_vs_serial_gpu", "forward_ms",
            "backward_ms", "fp32", "roofline", "cpu_baseline")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=None, choices=["small", "large", "mixed", "batched", "diff"],
                    help="print the line of this workload alone (default: the large workload's line "
                         "with every other workload as a sub-object)")
    ap.add_argument("--serial-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate budget of the oracle CPU-baseline samples (0 = skip them and "
                         "the relative errors)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of known size (for hardware-counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus %d is not supported "
              "(the batched instances and the segments of one instance would shard across GPUs)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import paper_1809_06360_amd as L
    from synthetic import WORKLOADS

    if not os.path.exists(L.LIB_PATH):
        log("library not built; building")
        from paper_1809_06360_amd import build as hip_build
        hip_build.build()
    workers = max(1, min(64, os.cpu_count() or 1))

    def mixed_leg():
        return run_single(args, "mixed", max(3, min(args.steps, 10)), min(args.warmup, 2), 1,
                          args.cpu_seconds)

    def small_leg():
        return run_single(args, "small", args.steps, args.warmup, args.serial_steps,
                          min(args.cpu_seconds, 2.0))

    if args.workload == "batched":
        print(json.dumps(run_batched(args, WORKLOADS["batched"], workers)), flush=True)
        return
    if args.workload == "diff":
        print(json.dumps(run_diff(args, WORKLOADS["diff"], workers)), flush=True)
        return
    if args.workload == "mixed":
        print(json.dumps(mixed_leg()), flush=True)
        return
    if args.workload == "small":
        print(json.dumps(small_leg()), flush=True)
        return

    result = run_single(args, "large", args.steps, args.warmup, args.serial_steps, args.cpu_seconds,
                        with_mixed_leg=True)
    if args.workload is None:
        bargs = argparse.Namespace(steps=5, warmup=2, serial_steps=2, cpu_seconds=args.cpu_seconds)
        for name, fn in (("small", small_leg), ("mixed_workload", mixed_leg),
                         ("batched", lambda: run_batched(bargs, WORKLOADS["batched"], workers)),
                         ("differentiable", lambda: run_diff(bargs, WORKLOADS["diff"], workers))):
            try:
                sub = fn()
                result[name] = {k: sub[k] for k in SUB_KEYS if k in sub}
            except Exception as exc:  # the headline line must still be printed
                result[name] = {"error": repr(exc)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
