"""Test infrastructure: the paper's own policy families of the segmented
solve (Sec. II-B feedback policy, eqs. Kx, Kz, k1; Sec. III-A parallel and
smoothed policies), in FP64 numpy.

NOT PART OF THE PRODUCT PATH. Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may use this module. It shares no code with
the GPU path and imports nothing from it.

Each segment j < J-1 is the end-point constrained problem of Sec. II-A: start
at x_{t_j}, end at the link point z = x_{t_{j+1}}, no cost on the end state
(the next segment owns it). Its tail from stage t, with a linear price mu on
the end state, has the value
    V_t(x; mu) = 1/2 x'P0_t x + (Gam_t mu + pbar_t)'x + psi_t'mu - 1/2 mu'Psi_t mu
and end state Gam_t'x + psi_t - Psi_t mu (the segment summaries of Sec. II-A,
written here by the plain backward recursion in its dual form, stage by stage).
With the end state fixed at z the price is the one that meets it,
mu = Psi_t^+ (Gam_t'x + psi_t - z), and the stage's optimal input is
    u_t = K0_t x + kbar_t - G_t mu,        G_t = H_t^{-1} B_t' Gam_{t+1},
i.e. the paper's affine policy u = K_x x + K_z x_term + k_1 with
    K_x = K0_t - G_t Psi_t^+ Gam_t',  K_z = G_t Psi_t^+,  k_1 = kbar_t - G_t Psi_t^+ psi_t.
Reading (the paper's rank-revealing split of the constraint-to-go): where the
tail is too short to reach every end state (Psi_t singular), the
Moore-Penrose pseudo-inverse takes the minimum-norm price; for a reachable
end state the constraint is met and the input is optimal either way.
The last segment has no end-point constraint: its policy is the serial one.

The smoothed policy (Sec. III-A) re-runs each segment j < J-1 as a plain
Riccati recursion whose terminal cost is segment j+1's cost-to-go at its
start with that segment's end fixed at its link point,
    C_{j+1}(x) = 1/2 x'(P0 + Gam Psi^+ Gam')x + (pbar + Gam Psi^+ (psi - z))'x + const
(maximising V(x; mu) - mu'z over mu), or the exact value (P, p) when j+1 is
the last segment.
"""

from __future__ import annotations

import numpy as np


def _sym(M):
    return 0.5 * (M + M.T)


def _data(prob, t):
    S = prob.get("S")
    n, m = prob["B"].shape[1], prob["B"].shape[2]
    return (prob["A"][t], prob["B"][t], prob["c"][t], _sym(prob["Q"][t]), prob["q"][t],
            _sym(prob["R"][t]), prob["r"][t], S[t] if S is not None else np.zeros((m, n)))


def tail_summaries(prob: dict, t0: int, t1: int):
    """Backward over stages t1-1 .. t0 of a segment with no end cost: per stage
    the dict of K0, kbar, G (policy pieces) and the tail summary P0, pbar, Gam,
    Psi, psi at t (after the stage's update). Index s = t - t0; entry t1 - t0
    holds the empty tail (P0 = 0, Gam = I, Psi = 0)."""
    n = prob["B"].shape[1]
    P0 = np.zeros((n, n))
    pbar = np.zeros(n)
    Gam = np.eye(n)
    Psi = np.zeros((n, n))
    psi = np.zeros(n)
    out = [None] * (t1 - t0 + 1)
    out[t1 - t0] = dict(P0=P0, pbar=pbar, Gam=Gam, Psi=Psi, psi=psi)
    for t in range(t1 - 1, t0 - 1, -1):
        A, B, c, Q, q, R, r, S = _data(prob, t)
        H = R + B.T @ P0 @ B
        Hux = B.T @ P0 @ A + S
        K0 = -np.linalg.solve(H, Hux)
        g = P0 @ c + pbar
        kbar = -np.linalg.solve(H, r + B.T @ g)
        G = np.linalg.solve(H, B.T @ Gam)
        W = B.T @ Gam
        Psi_n = Psi + W.T @ np.linalg.solve(H, W)
        psi_n = psi + Gam.T @ (c + B @ kbar)
        Gam_n = (A + B @ K0).T @ Gam
        P0_n = Q + A.T @ P0 @ A + Hux.T @ K0
        pbar_n = q + A.T @ g + Hux.T @ kbar
        P0, pbar, Gam, Psi, psi = _sym(P0_n), pbar_n, Gam_n, _sym(Psi_n), psi_n
        out[t - t0] = dict(K0=K0, kbar=kbar, G=G, P0=P0, pbar=pbar, Gam=Gam, Psi=Psi, psi=psi)
    return out


def constrained_value(summ: dict, z, rcond: float = 1e-12):
    """Hessian and gradient (at 0) in x of the tail's cost with its end state
    fixed at z: max over mu of V(x; mu) - mu'z."""
    Pp = np.linalg.pinv(summ["Psi"], rcond=rcond, hermitian=True)
    Vxx = summ["P0"] + summ["Gam"] @ Pp @ summ["Gam"].T
    vx = summ["pbar"] + summ["Gam"] @ Pp @ (summ["psi"] - z)
    return _sym(Vxx), vx


def segment_policy(prob: dict, t0: int, t1: int, rcond: float = 1e-12):
    """The paper's parallel policy on segment [t0, t1): per stage K_x (m x n),
    K_z (m x n), k_1 (m) with u_t = K_x x_t + K_z x_{t1} + k_1."""
    summ = tail_summaries(prob, t0, t1)
    Kx, Kz, k1 = [], [], []
    for s in range(t1 - t0):
        a = summ[s]  # stage t0 + s: its policy pieces and the tail summary from it
        Pp = np.linalg.pinv(a["Psi"], rcond=rcond, hermitian=True)
        GP = a["G"] @ Pp
        Kx.append(a["K0"] - GP @ a["Gam"].T)
        Kz.append(GP)
        k1.append(a["kbar"] - GP @ a["psi"])
    return np.array(Kx), np.array(Kz), np.array(k1)


def bounds(T: int, J: int):
    L, e = divmod(T, J)
    return [j * L + min(j, e) for j in range(J + 1)]


def parallel_policies(prob: dict, J: int, serial: dict):
    """The parallel policy family over the whole horizon: segments j < J-1 by
    segment_policy, the last one by the serial gains (serial: the oracle's
    solution dict with K, k). Returns (Kx, Kz, k1, seg_of_stage, bounds)."""
    T, n, m = prob["B"].shape
    b = bounds(T, J)
    Kx = np.zeros((T, m, n))
    Kz = np.zeros((T, m, n))
    k1 = np.zeros((T, m))
    seg = np.zeros(T, dtype=int)
    for j in range(J):
        t0, t1 = b[j], b[j + 1]
        seg[t0:t1] = j
        if j < J - 1:
            Kx[t0:t1], Kz[t0:t1], k1[t0:t1] = segment_policy(prob, t0, t1)
        else:
            Kx[t0:t1] = serial["K"][t0:t1]
            k1[t0:t1] = serial["k"][t0:t1]
    return Kx, Kz, k1, seg, b


def riccati_from(prob: dict, t0: int, t1: int, Vxx, vx):
    """Plain Riccati gains over [t0, t1) from the terminal cost (Vxx, vx) at t1."""
    P, p = _sym(Vxx), vx
    T, n, m = prob["B"].shape
    K = np.zeros((t1 - t0, m, n))
    k = np.zeros((t1 - t0, m))
    for t in range(t1 - 1, t0 - 1, -1):
        A, B, c, Q, q, R, r, S = _data(prob, t)
        H = R + B.T @ P @ B
        Hux = B.T @ P @ A + S
        g = P @ c + p
        Kt = -np.linalg.solve(H, Hux)
        kt = -np.linalg.solve(H, r + B.T @ g)
        p = q + A.T @ g + Hux.T @ kt
        P = _sym(Q + A.T @ P @ A + Hux.T @ Kt)
        K[t - t0], k[t - t0] = Kt, kt
    return K, k


def smoothed_policies(prob: dict, J: int, serial: dict):
    """The smoothed policy family: serial-form gains K, k per stage, each
    segment j < J-1 re-run from segment j+1's constrained cost-to-go at its
    start (its end fixed at its link point, from serial["x"]), the last
    segment from the terminal cost."""
    T, n, m = prob["B"].shape
    b = bounds(T, J)
    K = np.array(serial["K"], dtype=np.float64)
    k = np.array(serial["k"], dtype=np.float64)
    x = serial["x"]
    for j in range(J - 1):
        t0, t1, t2 = b[j], b[j + 1], b[j + 2]
        if j + 1 < J - 1:
            Vxx, vx = constrained_value(tail_summaries(prob, t1, t2)[0], x[t2])
        else:
            Vxx, vx = serial["P"][t1], serial["p"][t1]
        K[t0:t1], k[t0:t1] = riccati_from(prob, t0, t1, Vxx, vx)
    return K, k


def rollout(prob: dict, policy, disturbance=None):
    """Simulate x_{t+1} = A x + B u + c (+ disturbance(t, x)) from x0 under
    policy(t, x) -> u; returns (x, u, cost) with the problem's quadratic cost."""
    T, n, m = prob["B"].shape
    x = np.zeros((T + 1, n))
    u = np.zeros((T, m))
    x[0] = prob["x0"]
    cost = 0.0
    for t in range(T):
        A, B, c, Q, q, R, r, S = _data(prob, t)
        u[t] = policy(t, x[t])
        cost += 0.5 * x[t] @ Q @ x[t] + q @ x[t] + 0.5 * u[t] @ R @ u[t] + r @ u[t] + u[t] @ S @ x[t]
        x[t + 1] = A @ x[t] + B @ u[t] + c
        if disturbance is not None:
            x[t + 1] = x[t + 1] + disturbance(t, x[t])
    QT = _sym(prob["Q"][T])
    cost += 0.5 * x[T] @ QT @ x[T] + prob["q"][T] @ x[T]
    return x, u, cost
