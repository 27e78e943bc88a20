"""Test infrastructure: the paper's explicit route to the Lagrange multipliers
of one segment subproblem (Sec. II-B, "Lagrange Multipliers").

NOT PART OF THE PRODUCT PATH. Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may use this module. It shares no code with
the GPU path, imports nothing from it, and uses numpy only.

With a segment's optimal states and inputs known, the stationarity conditions
that involve the multipliers (eqs. mults and mu) are linear in them: for each
stage s of the segment (global stage t = t0 + s),

    x-rows:  lam_s - A_t' lam_{s+1}           = -(Q_t x_s + S_t' u_s + q_t)
    u-rows:        - B_t' lam_{s+1}           = -(S_t x_s + R_t u_s + r_t)

and at the segment end either the end-point constraint's row

    lam_T + mu_T = -(Qe x_T + qe)     (segment end cost Qe, qe; zero between
                                       segments, where the next segment owns
                                       the stage cost of the link state)

or, for a segment that ends at the horizon with no end-point constraint, the
terminal row Q_T x_T + q_T + lam_T = 0. Stacked, these read A' lam = b
(eq. multsglobal) with A' of full column rank, and the multipliers are the
solution of the normal equations A A' lam = A b (eq. pseudoinverse). A A' is
block tridiagonal with n x n blocks (eq. bandedAA: I, Sigma_t = I + A_t A_t'
+ B_t B_t' on the diagonal, -A_t beside it, and the [I I; I I] corner of the
end-point multiplier); it is solved here by block forward elimination and back
substitution, the block substitution the paper names.

Sign: the paper's multipliers. Its lam_t is the negative of the costate
P_t x_t + p_t of the Riccati recursion, and the end-point multiplier mu_T of a
segment that ends at a link point equals that costate at the link point.
"""

from __future__ import annotations

import numpy as np


def _sym(M):
    return 0.5 * (M + M.T)


def stacked_system(prob: dict, t0: int, t1: int, x, u, end_constraint: bool = True):
    """A' (rows: equations, columns: multipliers) and b of eq. multsglobal for
    the segment [t0, t1] of `prob`, given its optimal states x[t0..t1] and
    inputs u[t0..t1-1] (global stage indexing). Multiplier order:
    lam_0..lam_T (T = t1 - t0), then mu_T if `end_constraint`."""
    A, B, Q, q, R, r = (prob[k] for k in ("A", "B", "Q", "q", "R", "r"))
    S = prob.get("S")
    n, m = B.shape[1], B.shape[2]
    T = t1 - t0
    nl = (T + 2 if end_constraint else T + 1) * n
    rows = T * (n + m) + n
    At = np.zeros((rows, nl))
    b = np.zeros(rows)
    I = np.eye(n)
    row = 0
    for s in range(T):
        t = t0 + s
        xs, us = x[t], u[t]
        # x-rows
        At[row:row + n, s * n:(s + 1) * n] = I
        At[row:row + n, (s + 1) * n:(s + 2) * n] = -A[t].T
        g = _sym(Q[t]) @ xs + q[t]
        if S is not None:
            g = g + S[t].T @ us
        b[row:row + n] = -g
        row += n
        # u-rows
        At[row:row + m, (s + 1) * n:(s + 2) * n] = -B[t].T
        h = _sym(R[t]) @ us + r[t]
        if S is not None:
            h = h + S[t] @ xs
        b[row:row + m] = -h
        row += m
    At[row:row + n, T * n:(T + 1) * n] = I
    if end_constraint:
        # end-point constraint x_T = x_term; the segment owns no cost at x_T
        At[row:row + n, (T + 1) * n:(T + 2) * n] = I
        b[row:row + n] = 0.0
    else:
        b[row:row + n] = -(_sym(Q[t1]) @ x[t1] + q[t1])
    return At, b


def block_tridiagonal_solve(D, L, rhs):
    """Solve the symmetric block-tridiagonal system with diagonal blocks D[i],
    sub-diagonal blocks L[i] (block row i + 1, block column i) and right-hand
    side rhs[i]: block forward elimination, then back substitution."""
    N = len(D)
    Dh = [None] * N
    yh = [None] * N
    Dh[0] = D[0].copy()
    yh[0] = rhs[0].copy()
    for i in range(1, N):
        G = np.linalg.solve(Dh[i - 1].T, L[i - 1].T).T      # L_{i-1} Dh_{i-1}^{-1}
        Dh[i] = D[i] - G @ L[i - 1].T
        yh[i] = rhs[i] - G @ yh[i - 1]
    z = [None] * N
    z[N - 1] = np.linalg.solve(Dh[N - 1], yh[N - 1])
    for i in range(N - 2, -1, -1):
        z[i] = np.linalg.solve(Dh[i], yh[i] - L[i].T @ z[i + 1])
    return z


def segment_multipliers(prob: dict, t0: int, t1: int, x, u, end_constraint: bool = True):
    """The multipliers of segment [t0, t1] by the normal equations
    A A' lam = A b (eqs. pseudoinverse, bandedAA) solved block by block.
    Returns (lam, mu): lam of shape (t1 - t0 + 1, n), paper sign; mu (n,) the
    end-point multiplier (None without an end-point constraint)."""
    n = prob["B"].shape[1]
    At, b = stacked_system(prob, t0, t1, x, u, end_constraint)
    AAt = At.T @ At
    Ab = At.T @ b
    nb = AAt.shape[0] // n
    blk = lambda i, j: AAt[i * n:(i + 1) * n, j * n:(j + 1) * n]  # noqa: E731
    # A A' has no blocks beyond the first off-diagonal (eq. bandedAA)
    D = [blk(i, i) for i in range(nb)]
    L = [blk(i + 1, i) for i in range(nb - 1)]
    rhs = [Ab[i * n:(i + 1) * n] for i in range(nb)]
    z = block_tridiagonal_solve(D, L, rhs)
    T = t1 - t0
    lam = np.stack(z[:T + 1])
    mu = z[T + 1] if end_constraint else None
    return lam, mu


def link_multipliers(prob: dict, bounds, x, u):
    """The end-point multiplier mu_j of every segment but the last, for the
    segment boundaries `bounds` (t_0 = 0 < t_1 < ... < t_J = T) and the optimal
    trajectory (x, u) of the whole problem: each inner segment's subproblem,
    with x_init and x_term at their optimal values, through
    segment_multipliers. Shape (J - 1, n)."""
    J = len(bounds) - 1
    return np.stack([segment_multipliers(prob, bounds[j], bounds[j + 1], x, u)[1] for j in range(J - 1)])
