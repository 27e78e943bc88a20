"""Pins of the oracle's policy families (Sec. II-B feedback policy, eqs. Kx,
Kz, k1; Sec. III-A parallel and smoothed policies), CPU only.

A dense end-point constrained KKT solve (numpy LU over states, inputs and
multipliers of one segment tail: dynamics, initial state and end state as
equality constraints, no cost on the end state) is the independent reference:
  * the parallel policy's input u_t = K_x x_t + K_z z + k_1 equals the dense
    solve's first input for random start states x_t and reachable end states
    z, at every stage whose tail can reach any end state;
  * on the optimal trajectory with z at the link points the policy gives the
    optimal inputs at every stage, also where the tail is too short
    (pseudo-inverse price);
  * the constrained cost-to-go used by the smoothing pass has the dense
    solve's cost as its quadratic (Hessian and gradient by exact second
    differences);
  * the smoothed and parallel families reproduce the optimal trajectory on the
    undisturbed dynamics (the paper's statement) while their gains differ from
    the serial ones (not serial-exact);
  * the last segment's parallel policy is the serial one.
"""

import numpy as np
import pytest

import oracle
from oracle import policies as PO
from synthetic import make_instance


def _sym(M):
    return 0.5 * (M + M.T)


def dense_tail(prob, t0, t1, x_init, z):
    """Minimise sum_{t0 <= t < t1} of the stage costs subject to the dynamics,
    x_{t0} = x_init and x_{t1} = z. Returns (x, u, cost)."""
    A, B, c, Q, q, R, r = (prob[k] for k in ("A", "B", "c", "Q", "q", "R", "r"))
    S = prob.get("S")
    n, m = B.shape[1], B.shape[2]
    L = t1 - t0
    nx, nu = (L + 1) * n, L * m
    neq = n + L * n + n
    N = nx + nu + neq
    K = np.zeros((N, N))
    b = np.zeros(N)
    X = lambda s: slice(s * n, (s + 1) * n)                 # noqa: E731
    U = lambda s: slice(nx + s * m, nx + (s + 1) * m)       # noqa: E731
    # Hessian of the cost
    for s in range(L):
        t = t0 + s
        K[X(s), X(s)] += _sym(Q[t])
        K[U(s), U(s)] += _sym(R[t])
        if S is not None:
            K[U(s), X(s)] += S[t]
            K[X(s), U(s)] += S[t].T
        b[X(s)] -= q[t]
        b[U(s)] -= r[t]
    # constraints C z = d, with multipliers in the last neq unknowns
    C = np.zeros((neq, nx + nu))
    d = np.zeros(neq)
    C[:n, X(0)] = np.eye(n)
    d[:n] = x_init
    for s in range(L):
        t = t0 + s
        rs = slice(n + s * n, n + (s + 1) * n)
        C[rs, X(s + 1)] = np.eye(n)
        C[rs, X(s)] = -A[t]
        C[rs, U(s)] = -B[t]
        d[rs] = c[t]
    C[n + L * n:, X(L)] = np.eye(n)
    d[n + L * n:] = z
    K[nx + nu:, :nx + nu] = C
    K[:nx + nu, nx + nu:] = C.T
    b[nx + nu:] = d
    sol = np.linalg.solve(K, b)
    x = sol[:nx].reshape(L + 1, n)
    u = sol[nx:nx + nu].reshape(L, m)
    cost = 0.0
    for s in range(L):
        t = t0 + s
        cost += 0.5 * x[s] @ Q[t] @ x[s] + q[t] @ x[s] + 0.5 * u[s] @ R[t] @ u[s] + r[t] @ u[s]
        if S is not None:
            cost += u[s] @ S[t] @ x[s]
    return x, u, cost


@pytest.mark.parametrize("n,m,cross", [(4, 2, True), (3, 1, False), (5, 3, True)])
def test_parallel_policy_matches_the_endpoint_constrained_solve(n, m, cross):
    T = 16
    prob = make_instance(170, 0, n, m, T)
    if not cross:
        prob.pop("S", None)
    rng = np.random.default_rng(1)
    t0, t1 = 3, 14
    Kx, Kz, k1 = PO.segment_policy(prob, t0, t1)
    checked = 0
    for t in range(t0, t1):
        if (t1 - t) * m < n:
            continue  # the tail cannot reach every end state
        xt = rng.standard_normal(n)
        z = rng.standard_normal(n)
        _, u_ref, _ = dense_tail(prob, t, t1, xt, z)
        u = Kx[t - t0] @ xt + Kz[t - t0] @ z + k1[t - t0]
        np.testing.assert_allclose(u, u_ref[0], rtol=0, atol=1e-9 * (1 + np.abs(u_ref).max()))
        checked += 1
    assert checked >= 5


def test_parallel_policy_reproduces_the_optimum_at_every_stage():
    prob = make_instance(171, 0, 4, 2, 30)
    sol = oracle.solve(prob)
    J = 3
    Kx, Kz, k1, seg, b = PO.parallel_policies(prob, J, sol)
    x, u = sol["x"], sol["u"]
    for t in range(30):
        z = x[b[seg[t] + 1]] if seg[t] < J - 1 else np.zeros(4)
        ut = Kx[t] @ x[t] + Kz[t] @ z + k1[t]
        np.testing.assert_allclose(ut, u[t], rtol=0, atol=1e-9 * (1 + np.abs(u).max()))
    # the last segment carries no end-point constraint: its policy is the serial one
    np.testing.assert_array_equal(Kx[b[J - 1]:], sol["K"][b[J - 1]:])
    assert not Kz[b[J - 1]:].any()


def test_constrained_cost_to_go_is_the_dense_cost():
    prob = make_instance(172, 0, 3, 2, 20)
    t1, t2 = 8, 17
    z = np.array([0.3, -0.2, 0.5])
    Vxx, vx = PO.constrained_value(PO.tail_summaries(prob, t1, t2)[0], z)
    n = 3
    f = lambda x: dense_tail(prob, t1, t2, x, z)[2]   # noqa: E731
    f0 = f(np.zeros(n))
    E = np.eye(n)
    H = np.zeros((n, n))
    g = np.zeros(n)
    for i in range(n):
        fi, fmi = f(E[i]), f(-E[i])
        g[i] = 0.5 * (fi - fmi)
        for j in range(n):
            H[i, j] = f(E[i] + E[j]) - fi - f(E[j]) + f0
    np.testing.assert_allclose(H, Vxx, rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(g, vx, rtol=1e-8, atol=1e-8)


def test_smoothed_policy_keeps_the_optimum_but_not_the_serial_gains():
    prob = make_instance(173, 0, 4, 2, 36)
    sol = oracle.solve(prob)
    J = 3
    K, k = PO.smoothed_policies(prob, J, sol)
    x, _, _ = PO.rollout(prob, lambda t, xt: K[t] @ xt + k[t])
    np.testing.assert_allclose(x, sol["x"], rtol=0, atol=1e-9 * (1 + np.abs(sol["x"]).max()))
    b = PO.bounds(36, J)
    assert np.abs(K[:b[1]] - sol["K"][:b[1]]).max() > 1e-6      # differs on the first segment
    np.testing.assert_allclose(K[b[1]:b[2]], sol["K"][b[1]:b[2]], rtol=0, atol=1e-9)  # exact value next to the last
