"""Seeded synthetic LQR problem data.

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark. It holds the input recipe only (random draws and their shapes) and
none of the solver's arithmetic, so neither side depends on the other through it.

The paper times its method on problems whose state and input dimensions match a
legged robot (n = 40, m = 10; Sec. III-B, Table I) but does not publish the model
matrices, so every workload here is synthetic. Recipe, per instance, with fresh
draws for every time step:

    A_t = I + 0.1 * G / sqrt(n),        G ~ N(0,1)^{n x n}          t = 0..T-1
    B_t = N(0,1)^{n x m} / sqrt(n)                                   t = 0..T-1
    Q_t = L L^T + 0.1 I,                L ~ N(0,1)^{n x n} / sqrt(n) t = 0..T (T = terminal)
    R_t = I + 0.1 M M^T,                M ~ N(0,1)^{m x m} / sqrt(m) t = 0..T-1
    q_t ~ N(0,1)^n (t = 0..T),  r_t ~ N(0,1)^m,  c_t ~ N(0,1)^n,  x0 ~ N(0,1)^n

Random stream: ``numpy.random.default_rng(SeedSequence([cfg, instance, 18090636]))``,
drawn in the order G, B, L, M, q, r, c, x0 (then S when a cross term is asked for).

Layouts are row-major and time-major: A[T][n][n], B[T][n][m], c[T][n],
Q[T+1][n][n], q[T+1][n], R[T][m][m], r[T][m], S[T][m][n], x0[n].
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_TAG = 18090636
# instance index used for the draw of the batched workload's dimensions
DIMS_STREAM = 1 << 31

FIELDS = ("A", "B", "c", "Q", "q", "R", "r", "x0")


def _rng(cfg: int, instance: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(instance), SEED_TAG]))


def make_instance(cfg: int, instance: int, n: int, m: int, T: int,
                  cross_term: bool = False) -> dict:
    """One LQR instance as a dict of FP64 numpy arrays (see module docstring).

    With ``cross_term`` a state-input cross weight S_t = 0.05 N(0,1)^{m x n}/sqrt(n)
    is added; it is small enough that Q_t - S_t^T R_t^{-1} S_t stays positive
    definite (Q_t >= 0.1 I, R_t >= I), which keeps the problem strictly convex.
    """
    if n < 1 or m < 1 or T < 1:
        raise ValueError("n, m, T must be >= 1")
    g = _rng(cfg, instance)
    sn, sm = math.sqrt(n), math.sqrt(m)
    eye_n, eye_m = np.eye(n), np.eye(m)
    A = eye_n + 0.1 * g.standard_normal((T, n, n)) / sn
    B = g.standard_normal((T, n, m)) / sn
    L = g.standard_normal((T + 1, n, n)) / sn
    Q = L @ np.swapaxes(L, 1, 2) + 0.1 * eye_n
    M = g.standard_normal((T, m, m)) / sm
    R = eye_m + 0.1 * (M @ np.swapaxes(M, 1, 2))
    q = g.standard_normal((T + 1, n))
    r = g.standard_normal((T, m))
    c = g.standard_normal((T, n))
    x0 = g.standard_normal(n)
    out = dict(A=A, B=B, c=c, Q=Q, q=q, R=R, r=r, x0=x0)
    if cross_term:
        out["S"] = 0.05 * g.standard_normal((T, m, n)) / sn
    for key, val in out.items():
        out[key] = np.ascontiguousarray(val, dtype=np.float64)
    return out


def make_lti(cfg: int, n: int, m: int, T: int) -> dict:
    """A time-invariant instance (same A, B, Q, R at every step, zero linear
    terms and offsets) drawn with the same recipe; used to compare a long
    horizon's P_0 with the discrete algebraic Riccati solution."""
    one = make_instance(cfg, 0, n, m, 1)
    A = np.repeat(one["A"][:1], T, axis=0)
    B = np.repeat(one["B"][:1], T, axis=0)
    Q = np.repeat(one["Q"][:1], T + 1, axis=0)
    R = np.repeat(one["R"][:1], T, axis=0)
    return dict(A=A, B=B, c=np.zeros((T, n)), Q=Q, q=np.zeros((T + 1, n)),
                R=R, r=np.zeros((T, m)), x0=one["x0"].copy())


@dataclass(frozen=True)
class Workload:
    """A named workload: instance dimensions, segment count and precision."""
    name: str
    cfg: int
    dims: tuple          # tuple of (n, m, T) per instance
    segments: int        # 0 = chosen by the planner
    precision: str       # "fp64", "mixed" or "fp32"

    @property
    def batch(self) -> int:
        return len(self.dims)

    @property
    def total_steps(self) -> int:
        return sum(T for (_, _, T) in self.dims)


def batched_dims(count: int = 256, cfg: int = 2) -> tuple:
    """Dimensions of the uneven batch: n ~ U{12..64}, m ~ U{4..32}, T ~ U{64..512}."""
    g = _rng(cfg, DIMS_STREAM)
    n = g.integers(12, 65, size=count)
    m = g.integers(4, 33, size=count)
    T = g.integers(64, 513, size=count)
    return tuple((int(a), int(b), int(c)) for a, b, c in zip(n, m, T))


WORKLOADS = {
    "small": Workload("small: 1 x (n=4, m=2, T=64), J=4, fp64", 0, ((4, 2, 64),), 4, "fp64"),
    "large": Workload("large: 1 x (n=48, m=24, T=1024), J=64, fp64", 1, ((48, 24, 1024),), 64, "fp64"),
    "batched": Workload("batched: 256 x uneven (n 12..64, m 4..32, T 64..512), fp64", 2,
                        batched_dims(), 0, "fp64"),
    "mixed": Workload("mixed: 1 x (n=128, m=64, T=2048), J=128, fp32 GEMMs + fp64 factorizations", 3,
                      ((128, 64, 2048),), 128, "mixed"),
    "diff": Workload("diff: 512 x (n=16, m=8, T=128), forward + adjoint", 4,
                     tuple([(16, 8, 128)] * 512), 1, "fp64"),
}


def workload_instances(w: Workload, which=None):
    """Yield (index, instance dict) for the chosen instance indices of a workload."""
    idx = range(w.batch) if which is None else which
    for i in idx:
        n, m, T = w.dims[i]
        yield i, make_instance(w.cfg, i, n, m, T)
