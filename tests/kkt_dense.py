"""Dense KKT reference used to pin the oracle (test helper, numpy only).

Assembles the optimality conditions of problem (opt:globalwords) exactly as
printed in eq. (KKT) -- stationarity in (x_t, u_t) with the paper's multiplier
sign, the terminal condition (multsT1) -- together with the dynamics
(eq. dynamicsform) and the initial condition (eq. init), and solves the
resulting square system with a dense LU (numpy.linalg.solve). This route shares
nothing with the Riccati recursion.

Unknown order: x_0..x_T, u_0..u_{T-1}, lam_0..lam_T (paper's lambda).
"""

import numpy as np


def _sym(M):
    return 0.5 * (M + M.T)


def assemble(prob):
    A, B, c, Q, q, R, r, x0 = (prob[k] for k in ("A", "B", "c", "Q", "q", "R", "r", "x0"))
    S = prob.get("S")
    T, n, m = B.shape
    nx, nu = (T + 1) * n, T * m
    N = nx + nu + (T + 1) * n
    K = np.zeros((N, N))
    b = np.zeros(N)
    X = lambda t: slice(t * n, (t + 1) * n)                      # noqa: E731
    U = lambda t: slice(nx + t * m, nx + (t + 1) * m)            # noqa: E731
    L = lambda t: slice(nx + nu + t * n, nx + nu + (t + 1) * n)  # noqa: E731
    I = np.eye(n)
    row = 0
    for t in range(T):
        # x_t row of eq. (mults1): Q_xx x + Q_ux' u + q_x1 + lam_t - F_x' lam_{t+1} = 0
        rs = slice(row, row + n)
        K[rs, X(t)] = _sym(Q[t])
        if S is not None:
            K[rs, U(t)] = S[t].T
        K[rs, L(t)] = I
        K[rs, L(t + 1)] = -A[t].T
        b[rs] = -q[t]
        row += n
        # u_t row: Q_ux x + Q_uu u + q_u1 - F_u' lam_{t+1} = 0
        rs = slice(row, row + m)
        if S is not None:
            K[rs, X(t)] = S[t]
        K[rs, U(t)] = _sym(R[t])
        K[rs, L(t + 1)] = -B[t].T
        b[rs] = -r[t]
        row += m
    # terminal condition (multsT1): Q_xx_T x_T + q_x1_T + lam_T = 0
    rs = slice(row, row + n)
    K[rs, X(T)] = _sym(Q[T])
    K[rs, L(T)] = I
    b[rs] = -q[T]
    row += n
    # initial condition (eq. init): x_0 = x_init
    rs = slice(row, row + n)
    K[rs, X(0)] = I
    b[rs] = x0
    row += n
    # dynamics (eq. dynamicsform): x_{t+1} - F_x x_t - F_u u_t - f_1 = 0
    for t in range(T):
        rs = slice(row, row + n)
        K[rs, X(t + 1)] = I
        K[rs, X(t)] = -A[t]
        K[rs, U(t)] = -B[t]
        b[rs] = c[t]
        row += n
    assert row == N
    return K, b, (n, m, T)


def split(z, n, m, T):
    nx, nu = (T + 1) * n, T * m
    x = z[:nx].reshape(T + 1, n)
    u = z[nx:nx + nu].reshape(T, m)
    lam_paper = z[nx + nu:].reshape(T + 1, n)
    return x, u, lam_paper


def solve(prob):
    """Returns x, u and the paper's multipliers lambda_t (= -(P_t x_t + p_t))."""
    K, b, (n, m, T) = assemble(prob)
    z = np.linalg.solve(K, b)
    return split(z, n, m, T)


def tail(prob, t0, x_start):
    """The same problem restricted to stages t0..T with x_{t0} = x_start."""
    T = prob["B"].shape[0]
    out = {}
    for key in ("A", "B", "c", "R", "r", "S"):
        if prob.get(key) is not None:
            out[key] = prob[key][t0:T]
    out["Q"] = prob["Q"][t0:T + 1]
    out["q"] = prob["q"][t0:T + 1]
    out["x0"] = np.asarray(x_start, dtype=np.float64)
    return out


def grad(prob, dl_dx, dl_du, keys=("A", "B", "c", "Q", "q", "R", "r", "S", "x0")):
    """Gradient of l(x, u) with respect to every datum by implicit
    differentiation of the dense system K(theta) z = b(theta):
    dl/dtheta = zhat' (db/dtheta - dK/dtheta z) with K' zhat = dl/dz.
    K and b are affine in each datum, so one-sided differences of the assembly
    are exact."""
    K, b, (n, m, T) = assemble(prob)
    z = np.linalg.solve(K, b)
    g = np.zeros_like(z)
    g[:(T + 1) * n] = np.asarray(dl_dx).ravel()
    g[(T + 1) * n:(T + 1) * n + T * m] = np.asarray(dl_du).ravel()
    zhat = np.linalg.solve(K.T, g)
    out = {}
    for key in keys:
        if prob.get(key) is None:
            continue
        base = prob[key]
        G = np.zeros(base.size)
        for i in range(base.size):
            pert = dict(prob)
            arr = base.copy().ravel()
            arr[i] += 1.0
            pert[key] = arr.reshape(base.shape)
            K1, b1, _ = assemble(pert)
            G[i] = zhat @ ((b1 - b) - (K1 - K) @ z)
        out[key] = G.reshape(base.shape)
    return out
