"""Pins for the CPU oracle's forward solve (no GPU).

Each check ties the serial Riccati oracle to something other than itself:
  * the dense KKT system of eq. (KKT) solved by LU (x, u, multipliers);
  * the tail problem solved densely from several start states, which fixes the
    policy K_t, k_t and the value function P_t, p_t by their definitions;
  * the discrete algebraic Riccati equation (scipy) for a long time-invariant
    horizon;
  * a scalar problem solved by hand;
  * structural facts: P_t symmetric positive semidefinite, optimal cost below
    the cost of perturbed controls.
"""

import numpy as np
import pytest
import scipy.linalg

import kkt_dense
from synthetic import make_instance, make_lti

CASES = [
    # (cfg, inst, n, m, T, cross_term)
    (100, 0, 1, 1, 1, False),
    (100, 1, 3, 2, 5, False),
    (100, 2, 5, 3, 9, True),
    (100, 3, 2, 4, 7, True),     # more inputs than states
    (100, 4, 6, 1, 12, False),
    (100, 5, 8, 5, 20, True),
]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("cfg,inst,n,m,T,cross", CASES)
def test_oracle_matches_dense_kkt(oracle_mod, cfg, inst, n, m, T, cross):
    prob = make_instance(cfg, inst, n, m, T, cross_term=cross)
    sol = oracle_mod.solve(prob)
    assert sol["info"] == 0
    x, u, lam_paper = kkt_dense.solve(prob)
    assert rel(sol["x"], x) < 1e-11
    assert rel(sol["u"], u) < 1e-11
    # costate sign: lam = P x + p is minus the paper's multiplier
    assert rel(sol["lam"], -lam_paper) < 1e-11


@pytest.mark.parametrize("cfg,inst,n,m,T,cross", CASES[1:])
def test_oracle_policy_and_value_by_definition(oracle_mod, cfg, inst, n, m, T, cross):
    """K_t, k_t are the optimal first control of the tail problem as an affine
    function of the start state; P_t, p_t are the start multiplier (minus the
    paper's lambda) as an affine function of the start state."""
    prob = make_instance(cfg, inst, n, m, T, cross_term=cross)
    sol = oracle_mod.solve(prob)
    for t0 in sorted({0, T // 2, T - 1}):
        _, u0, l0 = kkt_dense.solve(kkt_dense.tail(prob, t0, np.zeros(n)))
        assert rel(sol["k"][t0], u0[0]) < 1e-10
        assert rel(sol["p"][t0], -l0[0]) < 1e-10
        Kcols, Pcols = [], []
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            _, ui, li = kkt_dense.solve(kkt_dense.tail(prob, t0, e))
            Kcols.append(ui[0] - u0[0])
            Pcols.append(-(li[0] - l0[0]))
        assert rel(sol["K"][t0], np.array(Kcols).T) < 1e-9
        assert rel(sol["P"][t0], np.array(Pcols).T) < 1e-9


def test_oracle_terminal_condition(oracle_mod):
    prob = make_instance(101, 0, 4, 2, 6)
    sol = oracle_mod.solve(prob)
    assert np.array_equal(sol["P"][-1], prob["Q"][-1])
    assert np.array_equal(sol["p"][-1], prob["q"][-1])


def test_oracle_p_symmetric_psd(oracle_mod):
    prob = make_instance(102, 0, 10, 4, 40)
    sol = oracle_mod.solve(prob)
    P = sol["P"]
    assert np.array_equal(P, np.swapaxes(P, 1, 2))
    for t in range(P.shape[0]):
        w = np.linalg.eigvalsh(P[t])
        assert w.min() > 0.0     # Q_t >= 0.1 I here, so P_t is positive definite


@pytest.mark.parametrize("n,m", [(2, 1), (4, 2), (6, 3)])
def test_oracle_long_horizon_reaches_dare(oracle_mod, n, m):
    """For a time-invariant problem over a long horizon, P_0 converges to the
    stabilising solution of the discrete algebraic Riccati equation, and K_0
    to the matching infinite-horizon gain."""
    prob = make_lti(103 + n, n, m, 400)
    sol = oracle_mod.solve(prob)
    A, B, Q, R = prob["A"][0], prob["B"][0], prob["Q"][0], prob["R"][0]
    X = scipy.linalg.solve_discrete_are(A, B, Q, R)
    Kinf = -np.linalg.solve(R + B.T @ X @ B, B.T @ X @ A)
    assert rel(sol["P"][0], X) < 1e-10
    assert rel(sol["K"][0], Kinf) < 1e-10


def test_oracle_scalar_closed_form(oracle_mod):
    """n = m = 1, T = 2, A = B = Q = R = 1, no linear terms, x0 = 1, solved by
    hand: P_2 = 1; P_1 = 1 + 1 - 1/2 = 3/2 with K_1 = -1/2; P_0 = 1 + 3/2 -
    (3/2)^2/(5/2) = 8/5 with K_0 = -3/5; x_1 = 2/5, u_0 = -3/5, u_1 = -1/5,
    x_2 = 1/5."""
    one = np.ones((2, 1, 1))
    prob = dict(A=one.copy(), B=one.copy(), c=np.zeros((2, 1)), Q=np.ones((3, 1, 1)),
                q=np.zeros((3, 1)), R=one.copy(), r=np.zeros((2, 1)), x0=np.ones(1))
    sol = oracle_mod.solve(prob)
    np.testing.assert_allclose(sol["P"][:, 0, 0], [8 / 5, 3 / 2, 1.0], rtol=1e-15)
    np.testing.assert_allclose(sol["K"][:, 0, 0], [-3 / 5, -1 / 2], rtol=1e-15)
    np.testing.assert_allclose(sol["x"][:, 0], [1.0, 2 / 5, 1 / 5], rtol=1e-15)
    np.testing.assert_allclose(sol["u"][:, 0], [-3 / 5, -1 / 5], rtol=1e-15)


def test_oracle_affine_terms_closed_form(oracle_mod):
    """n = m = 1, T = 1 with offsets and linear terms, by hand:
    A=2, B=1, c=3, Q_0=1, q_0=1, R=2, r=-1, Q_1=3, q_1=2, x0=1.
    v = P_1 c + p_1 = 11; M_uu = 2 + 3 = 5; M_ux = 6; m_u1 = -1 + 11 = 10;
    K = -6/5, k = -2; P_0 = 1 + 12 - 36/5 = 29/5; p_0 = 1 + 22 - 12 = 11;
    u_0 = -6/5 - 2 = -16/5; x_1 = 2 - 16/5 + 3 = 9/5."""
    prob = dict(A=np.full((1, 1, 1), 2.0), B=np.ones((1, 1, 1)), c=np.full((1, 1), 3.0),
                Q=np.array([[[1.0]], [[3.0]]]), q=np.array([[1.0], [2.0]]),
                R=np.full((1, 1, 1), 2.0), r=np.full((1, 1), -1.0), x0=np.ones(1))
    sol = oracle_mod.solve(prob)
    np.testing.assert_allclose(sol["K"][0, 0, 0], -6 / 5, rtol=1e-15)
    np.testing.assert_allclose(sol["k"][0, 0], -2.0, rtol=1e-15)
    np.testing.assert_allclose(sol["P"][0, 0, 0], 29 / 5, rtol=1e-15)
    np.testing.assert_allclose(sol["p"][0, 0], 11.0, rtol=1e-15)
    np.testing.assert_allclose(sol["u"][0, 0], -16 / 5, rtol=1e-15)
    np.testing.assert_allclose(sol["x"][1, 0], 9 / 5, rtol=1e-15)


def test_oracle_cost_is_minimal(oracle_mod):
    prob = make_instance(104, 0, 5, 3, 15, cross_term=True)
    sol = oracle_mod.solve(prob)
    A, B, c = prob["A"], prob["B"], prob["c"]
    best = oracle_mod.cost(prob, sol["x"], sol["u"])
    rng = np.random.default_rng(0)
    for _ in range(20):
        u = sol["u"] + 1e-3 * rng.standard_normal(sol["u"].shape)
        x = np.zeros_like(sol["x"])
        x[0] = prob["x0"]
        for t in range(u.shape[0]):
            x[t + 1] = A[t] @ x[t] + B[t] @ u[t] + c[t]
        assert oracle_mod.cost(prob, x, u) > best


def test_oracle_reports_indefinite_input_hessian(oracle_mod):
    prob = make_instance(105, 0, 4, 2, 10)
    prob["R"][6] = -50.0 * np.eye(2)
    sol = oracle_mod.solve(prob)
    assert sol["info"] == 7


def test_oracle_rejects_bad_arguments(oracle_mod):
    prob = make_instance(105, 1, 3, 2, 4)
    lib = oracle_mod._load()
    rc = lib.lqr_oracle_solve(0, 2, 4, *([None] * 16))
    assert rc == -1
    assert oracle_mod.solve(prob)["info"] == 0
