"""Test infrastructure: the plain serial FP64 CPU oracle for the LQR solve.

NOT PART OF THE PRODUCT PATH. Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU path and imports nothing from it.

``lqr_oracle.c`` holds the arithmetic (serial Riccati recursion of Sec. II-B in
its unconstrained case, and implicit differentiation of the KKT system, eq. KKT);
this module only builds it with gcc and marshals numpy arrays through ctypes.
Every function here is pinned by the ``-m "not gpu"`` tests against a dense KKT
solve, the discrete algebraic Riccati equation, closed forms and finite
differences.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqr_oracle.c")
_LIB = os.path.join(_HERE, "liblqr_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liblqr_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def open_library(path: str):
    """Load an oracle build from ``path`` (the default build, or a variant the
    tests compile to show that the pins catch planted mistakes)."""
    lib = ctypes.CDLL(path)
    lib.lqr_oracle_solve.restype = ctypes.c_int
    lib.lqr_oracle_solve.argtypes = [ctypes.c_int] * 3 + [_dp] * 16
    lib.lqr_oracle_backward.restype = ctypes.c_int
    lib.lqr_oracle_backward.argtypes = [ctypes.c_int] * 3 + [_dp] * 18
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = open_library(_LIB)
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def dims(prob: dict):
    T, n, m = prob["B"].shape
    return int(n), int(m), int(T)


def solve(prob: dict, with_lam: bool = True, lib=None) -> dict:
    """Serial FP64 LQR solve. ``prob`` holds A, B, c, Q, q, R, r, x0 (and
    optionally S) as numpy arrays in the layouts of ``synthetic``.

    Returns a dict with K, k, P, p, x, u (and lam = P x + p) and ``info``
    (0 on success, t+1 if the input Hessian at stage t is not positive definite).
    """
    n, m, T = dims(prob)
    a = {key: _f64(prob.get(key)) for key in ("A", "B", "c", "Q", "q", "R", "r", "S", "x0")}
    out = dict(K=np.zeros((T, m, n)), k=np.zeros((T, m)), P=np.zeros((T + 1, n, n)),
               p=np.zeros((T + 1, n)), x=np.zeros((T + 1, n)), u=np.zeros((T, m)))
    if with_lam:
        out["lam"] = np.zeros((T + 1, n))
    info = (lib or _load()).lqr_oracle_solve(
        n, m, T, _p(a["A"]), _p(a["B"]), _p(a["c"]), _p(a["Q"]), _p(a["q"]), _p(a["R"]),
        _p(a["r"]), _p(a["S"]), _p(a["x0"]), _p(out["K"]), _p(out["k"]), _p(out["P"]),
        _p(out["p"]), _p(out["x"]), _p(out["u"]), _p(out.get("lam")))
    if info < 0:
        raise ValueError("oracle: invalid arguments")
    out["info"] = int(info)
    return out


def backward(prob: dict, sol: dict, dl_dx, dl_du, lib=None) -> dict:
    """Gradient of a loss l(x, u) w.r.t. A, B, c, Q, q, R, r, S, x0 given the
    upstream gradients dl/dx [T+1][n] and dl/du [T][m] (see lqr_oracle.c)."""
    n, m, T = dims(prob)
    a = {key: _f64(prob.get(key)) for key in ("A", "B", "Q", "R", "S")}
    x, u, lam = _f64(sol["x"]), _f64(sol["u"]), _f64(sol["lam"])
    gx, gu = _f64(dl_dx), _f64(dl_du)
    g = dict(A=np.zeros((T, n, n)), B=np.zeros((T, n, m)), c=np.zeros((T, n)),
             Q=np.zeros((T + 1, n, n)), q=np.zeros((T + 1, n)), R=np.zeros((T, m, m)),
             r=np.zeros((T, m)), S=np.zeros((T, m, n)), x0=np.zeros(n))
    info = (lib or _load()).lqr_oracle_backward(
        n, m, T, _p(a["A"]), _p(a["B"]), _p(a["Q"]), _p(a["R"]), _p(a["S"]),
        _p(x), _p(u), _p(lam), _p(gx), _p(gu),
        _p(g["A"]), _p(g["B"]), _p(g["c"]), _p(g["Q"]), _p(g["q"]), _p(g["R"]),
        _p(g["r"]), _p(g["S"]), _p(g["x0"]))
    if info != 0:
        raise ValueError("oracle backward failed: info=%d" % info)
    return g


def cost(prob: dict, x, u) -> float:
    """Objective of problem (opt:globalwords) with the 1/2-scaled stage costs of
    eq. (costtform) evaluated at a trajectory (used by the tests)."""
    Q, q, R, r = prob["Q"], prob["q"], prob["R"], prob["r"]
    S = prob.get("S")
    T = u.shape[0]
    total = 0.0
    for t in range(T):
        total += 0.5 * x[t] @ Q[t] @ x[t] + 0.5 * u[t] @ R[t] @ u[t] + q[t] @ x[t] + r[t] @ u[t]
        if S is not None:
            total += u[t] @ S[t] @ x[t]
    total += 0.5 * x[T] @ Q[T] @ x[T] + q[T] @ x[T]
    return float(total)
