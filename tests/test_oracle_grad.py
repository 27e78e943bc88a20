"""Pins for the CPU oracle's gradient (no GPU).

The oracle differentiates through a second Riccati solve on the KKT-transposed
right-hand side. It is checked against (a) implicit differentiation of the
dense KKT system of eq. (KKT), which never runs a Riccati recursion, and (b)
central finite differences (h = 1e-6) of the oracle's own forward solve.
"""

import numpy as np
import pytest

import kkt_dense
from synthetic import make_instance

KEYS = ("A", "B", "c", "Q", "q", "R", "r", "S", "x0")


def loss_and_grads(sol):
    """l = sum_t |x_t|^2 + sum_t |u_t|^2."""
    x, u = sol["x"], sol["u"]
    return float((x * x).sum() + (u * u).sum()), 2.0 * x, 2.0 * u


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,m,T,cross", [(3, 2, 3, True), (2, 3, 4, True), (4, 1, 5, False)])
def test_grad_matches_dense_implicit_differentiation(oracle_mod, n, m, T, cross):
    prob = make_instance(200, n, n, m, T, cross_term=cross)
    sol = oracle_mod.solve(prob)
    _, gx, gu = loss_and_grads(sol)
    g = oracle_mod.backward(prob, sol, gx, gu)
    ref = kkt_dense.grad(prob, gx, gu)
    for key, G in ref.items():
        assert rel(g[key], G) < 1e-9, key


@pytest.mark.parametrize("n,m,T", [(4, 2, 6), (3, 3, 8)])
def test_grad_matches_central_differences(oracle_mod, n, m, T):
    prob = make_instance(201, n, n, m, T, cross_term=True)
    sol = oracle_mod.solve(prob)
    _, gx, gu = loss_and_grads(sol)
    g = oracle_mod.backward(prob, sol, gx, gu)
    rng = np.random.default_rng(7)
    h = 1e-6
    for key in KEYS:
        base = prob[key]
        flat = base.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            sym_partner = None
            if key in ("Q", "R"):
                t, i, j = np.unravel_index(idx, base.shape)
                if i != j:
                    sym_partner = np.ravel_multi_index((t, j, i), base.shape)
            vals = []
            for s in (+1.0, -1.0):
                pert = dict(prob)
                arr = flat.copy()
                arr[idx] += s * h
                if sym_partner is not None:
                    arr[sym_partner] += s * h
                pert[key] = arr.reshape(base.shape)
                vals.append(loss_and_grads(oracle_mod.solve(pert, with_lam=False))[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            an = g[key].reshape(-1)[idx]
            if sym_partner is not None:
                an = an + g[key].reshape(-1)[sym_partner]
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (key, idx, fd, an)
