"""Measure the per-stage cost model of the solver kernels on the current GPU
and write it as ``csrc/lqr_cost_model.h`` (the planner's segment-count tuner
reads it at build time).

Usage: ``python -m paper_1809_06360_amd.calibrate [--out PATH] [--table PATH]``

For a grid of (n, m) it times single launches of lqr_solve_phase with HIP
events (median of repeated launches on one stream):
  phase 1 with J = 1       -> T plain Riccati stages      -> cost per plain stage
  phase 3 with J = 1       -> T forward-simulation stages -> cost per rollout stage
  phase 1 with J = 8       -> T/8 parametric stages       -> cost per dual stage
  phase 2 with J = 2, 7    -> 1 and 6 serial linking steps -> cost per linking step
and fits each cost, separately for the VALU (n < 32) and matrix-core
(n >= 32) kernel variants, as a non-negative combination of the features
named in the generated header.
"""

from __future__ import annotations

import argparse
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
T_CAL = 64
NS = (4, 8, 12, 16, 24, 31, 32, 40, 48, 52, 56, 60, 64)
MS = (2, 4, 8, 16, 24, 32)


def flops_plain(n, m):
    return 4.0 * n ** 3 + 6.0 * n * n * m + 4.0 * n * m * m + m ** 3 / 3.0


def flops_dual(n, m):
    return flops_plain(n, m) + 2.0 * n ** 3 + 6.0 * n * n * m + 2.0 * n * m * m


def pad_rows(m):
    for w in (8, 16, 24, 32, 48, 64):
        if m <= w:
            return w
    return 64


def streamed(n, m):
    """Whether phase 1 runs the streamed parametric sweep for this size (the
    resident layout of a width-w kernel exceeds 160 KiB of LDS; matrix-core
    kernels use widths of at least 16)."""
    w = pad_rows(max(m, 9) if n >= 32 else m)
    W = m + 2 * n + 1
    dbl = n * (n | 1) + n + n * (m + n + 1) + n * W + (w + 1) * W + 3 * w + n * n + 2 * n
    return dbl * 8 + 64 > 160 * 1024


def _instance(n, m, T, rng):
    """Well-conditioned random instance (value distributions of the seeded
    workloads; only timing depends on it)."""
    G = rng.standard_normal((T, n, n))
    A = np.eye(n) + 0.1 * G / np.sqrt(n)
    B = rng.standard_normal((T, n, m)) / np.sqrt(n)
    Lq = rng.standard_normal((T + 1, n, n)) / np.sqrt(n)
    Q = Lq @ np.swapaxes(Lq, 1, 2) + 0.1 * np.eye(n)
    M = rng.standard_normal((T, m, m)) / np.sqrt(m)
    R = np.eye(m) + 0.1 * M @ np.swapaxes(M, 1, 2)
    return dict(A=A, B=B, c=rng.standard_normal((T, n)), Q=Q, q=rng.standard_normal((T + 1, n)),
                R=R, r=rng.standard_normal((T, m)), x0=rng.standard_normal(n))


def time_phase(L, torch, data, J, phase, reps=9):
    """Median milliseconds of one lqr_solve_phase launch (after a full solve
    has filled the workspace)."""
    out = L.solve(data, segments=J, with_lam=False)
    ws = out["_workspace"]
    prob = L._problem(data, out, J)
    opts = L.options()
    s = torch.cuda.current_stream()
    times = []
    for r in range(reps + 2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        L.lqr_solve_phase(prob, opts, phase, ws.data_ptr(), ws.numel(), s.cuda_stream)
        e1.record(s)
        e1.synchronize()
        if r >= 2:
            times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def measure(L, torch):
    rng = np.random.default_rng(1)
    rows = []
    for n in NS:
        for m in MS:
            host = _instance(n, m, T_CAL, rng)
            data = {k: torch.from_numpy(v).cuda() for k, v in host.items()}
            row = dict(n=n, m=m, mw=pad_rows(max(m, 9) if n >= 32 else m), mf=int(n >= 32),
                       gs=int(streamed(n, m)))
            row["plain"] = 1e3 * time_phase(L, torch, data, 1, 1) / T_CAL
            row["roll"] = 1e3 * time_phase(L, torch, data, 1, 3) / T_CAL
            try:
                row["dual"] = 1e3 * time_phase(L, torch, data, 8, 1) / (T_CAL // 8)
                # the serial linking chain (single instances link J < 8
                # segments serially; batched launches always do)
                t2 = time_phase(L, torch, data, 2, 2)
                t7 = time_phase(L, torch, data, 7, 2)
                row["link"] = 1e3 * (t7 - t2) / 5.0
            except L.LQRError:
                row["dual"] = row["link"] = None  # cannot be split on this device
            rows.append(row)
            print("n=%2d m=%2d plain %7.2f roll %6.2f dual %s link %s us" % (
                n, m, row["plain"], row["roll"],
                "%7.2f" % row["dual"] if row["dual"] else "   -   ",
                "%7.2f" % row["link"] if row["link"] else "   -   "), flush=True)
    return rows


def features(kind, r):
    n, m, mw = r["n"], r["m"], r["mw"]
    if kind in ("dual", "dualgs"):
        return [1.0, mw, n, flops_dual(n, m) / 1e5]
    if kind == "plain":
        return [1.0, mw, n, flops_plain(n, m) / 1e5]
    if kind == "roll":
        return [1.0, n, m, n * (n + m) / 1e3]
    return [1.0, n, n * n / 1e2, n ** 3 / 1e4]


def fit(rows):
    from scipy.optimize import nnls
    coef = {}
    for kind in ("dual", "dualgs", "plain", "roll", "link"):
        coef[kind] = []
        for mf in (0, 1):
            if kind == "dualgs":
                sel = [dict(r, dualgs=r["dual"]) for r in rows
                       if r["mf"] == mf and r["gs"] and r.get("dual") is not None]
                if not sel:  # no streamed sizes for this engine
                    coef[kind].append(np.zeros(4))
                    continue
            elif kind == "dual":
                sel = [r for r in rows if r["mf"] == mf and not r["gs"] and r.get(kind) is not None]
            else:
                sel = [r for r in rows if r["mf"] == mf and r.get(kind) is not None]
            if kind == "link":  # one row per n
                seen = {}
                for r in sel:
                    seen.setdefault(r["n"], []).append(r["link"])
                sel = [dict(n=k, m=1, mw=8, mf=mf, link=float(np.median(v))) for k, v in seen.items()]
            X = np.array([features(kind, r) for r in sel])
            y = np.array([r[kind] for r in sel])
            # relative least squares: weight rows by 1/y
            w = 1.0 / np.maximum(y, 1e-3)
            c, _ = nnls(X * w[:, None], y * w)
            pred = X @ c
            err = np.abs(pred - y) / np.maximum(y, 1e-3)
            coef[kind].append(c)
            print("%-5s mf=%d  coef %s  median rel err %.3f  max %.3f" % (
                kind, mf, np.array2string(c, precision=4), float(np.median(err)), float(err.max())))
    return coef


HEADER = """// Per-stage cost model of the solver kernels on MI355X (microseconds),
// measured by `python -m paper_1809_06360_amd.calibrate` (single-launch
// phase timings with HIP events, T = {T} stages, non-negative least squares).
//
// Each cost is a non-negative combination of features (see lqr_tuner.cpp):
//   sweeps (dual, dual streamed, plain)  [1, mw, n, flops / 1e5]
//   rollout               [1, n, m, n (n + m) / 1e3]
//   link                  [1, n, n^2 / 1e2, n^3 / 1e4]
// indexed [mf][feature], mf = 1 for the matrix-core product variants.
#pragma once

namespace lqr {{
namespace cost {{

{body}
constexpr double kTask = 3.0;

}}  // namespace cost
}}  // namespace lqr
"""


def render(coef):
    lines = []
    for kind, name in (("dual", "kDual"), ("dualgs", "kDualStreamed"), ("plain", "kPlain"),
                       ("roll", "kRoll"), ("link", "kLink")):
        rows = ", ".join("{%s}" % ", ".join("%.6g" % v for v in c) for c in coef[kind])
        lines.append("constexpr double %s[2][4] = {%s};" % (name, rows))
    return HEADER.format(T=T_CAL, body="\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "lqr_cost_model.h"))
    ap.add_argument("--table", default=None, help="also write the measured table (markdown)")
    a = ap.parse_args(argv)
    import torch
    import paper_1809_06360_amd as L
    if not torch.cuda.is_available():
        sys.exit("calibration needs a GPU")
    rows = measure(L, torch)
    coef = fit(rows)
    with open(a.out, "w") as f:
        f.write(render(coef))
    print("wrote", a.out)
    if a.table:
        with open(a.table, "w") as f:
            f.write("| n | m | plain us/stage | rollout us/stage | dual us/stage | link us/step |\n")
            f.write("|---|---|---|---|---|---|\n")
            for r in rows:
                f.write("| %d | %d | %.2f | %.2f | %s | %s |\n" % (
                    r["n"], r["m"], r["plain"], r["roll"],
                    "%.2f" % r["dual"] if r["dual"] else "-", "%.2f" % r["link"] if r["link"] else "-"))


if __name__ == "__main__":
    main()
