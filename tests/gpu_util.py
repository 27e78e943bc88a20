"""Helpers shared by the GPU tests: moving seeded instances to the device and
comparing outputs with the oracle's (relative Frobenius error over the stacked
output, the definition the tolerances below refer to)."""

import numpy as np

OUTPUTS = ("K", "k", "P", "p", "x", "u", "lam")
FP64_TOL = 1e-9      # FP64 path vs the FP64 oracle
MIXED_TOL = 1e-4     # mixed-precision path vs the FP64 oracle


def to_device(prob, device="cuda:0", dtype=None):
    import torch
    dtype = dtype or torch.float64
    return {k: torch.as_tensor(v).to(device=device, dtype=dtype).contiguous() for k, v in prob.items()}


def host(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items() if not k.startswith("_")}


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def compare(got, ref, keys=OUTPUTS, tol=FP64_TOL, label=""):
    errs = {}
    for k in keys:
        if k in got and k in ref:
            errs[k] = rel_err(got[k], ref[k])
    bad = {k: e for k, e in errs.items() if not (e <= tol)}
    assert not bad, "%s relative errors above %.1e: %s (all: %s)" % (label, tol, bad, errs)
    return errs


def oracle_map(fn, items, workers=None):
    """fn over items on a thread pool. The oracle's C calls release the GIL, so
    the reference solutions of a whole batch take seconds on a multicore host."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = workers or max(1, min(16, os.cpu_count() or 4))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, items))
