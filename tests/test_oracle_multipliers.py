"""Pins of the oracle's explicit multiplier route (Sec. II-B, "Lagrange
Multipliers": eqs. mults, mu, multsglobal, pseudoinverse, bandedAA), CPU only.

The route takes a segment's optimal trajectory and recovers its multipliers
from the normal equations A A' lam = A b by block substitution. It is pinned
against things computed another way:
  * the whole horizon as one segment (terminal row, no end-point constraint)
    gives the dense KKT solve's multipliers (eq. KKT, numpy LU);
  * an inner segment with x_init, x_term at the global optimum gives
    lam_t = -(P_t x_t + p_t) of the serial Riccati oracle on the segment and
    mu_T = P x + p at its link point (the link multiplier matched across
    segments, Sec. II-A);
  * A A' really is block tridiagonal, and the block solve equals a library
    least-squares solve of A' lam = b, whose residual is zero (the stacked
    system is consistent);
  * mutants of the assembly (a wrong sign on one stage's -A' coupling, a
    flipped end-point sign) break the pins.
"""

import numpy as np
import pytest

import oracle
from oracle import multipliers as M
from synthetic import make_instance
import kkt_dense

pytestmark = pytest.mark.filterwarnings("ignore")


def _bounds(T, J):
    L, e = divmod(T, J)
    return [j * L + min(j, e) for j in range(J + 1)]


def _costate(sol):
    return sol["lam"]  # P_t x_t + p_t


@pytest.mark.parametrize("n,m,T,cross", [(3, 2, 9, False), (4, 2, 12, True), (5, 3, 10, False)])
def test_whole_horizon_matches_dense_kkt(n, m, T, cross):
    prob = make_instance(150, 0, n, m, T)
    if not cross:
        prob.pop("S", None)
    x, u, lam_kkt = kkt_dense.solve(prob)
    lam, mu = M.segment_multipliers(prob, 0, T, x, u, end_constraint=False)
    assert mu is None
    np.testing.assert_allclose(lam, lam_kkt, rtol=0, atol=1e-10 * (1 + np.abs(lam_kkt).max()))


@pytest.mark.parametrize("n,m,T,J", [(4, 2, 24, 3), (6, 3, 40, 4), (5, 5, 21, 5)])
def test_inner_segments_give_the_costate_and_link_multiplier(n, m, T, J):
    prob = make_instance(151, 1, n, m, T)
    sol = oracle.solve(prob)
    x, u, lam = sol["x"], sol["u"], _costate(sol)
    b = _bounds(T, J)
    for j in range(J - 1):
        t0, t1 = b[j], b[j + 1]
        assert (t1 - t0) * m >= n  # the segment's stacked system has full column rank
        lam_s, mu = M.segment_multipliers(prob, t0, t1, x, u)
        scale = 1 + np.abs(lam).max()
        np.testing.assert_allclose(lam_s, -lam[t0:t1 + 1], rtol=0, atol=1e-9 * scale)
        np.testing.assert_allclose(mu, lam[t1], rtol=0, atol=1e-9 * scale)
    mus = M.link_multipliers(prob, b, x, u)
    np.testing.assert_allclose(mus, lam[b[1:-1]], rtol=0, atol=1e-9 * (1 + np.abs(lam).max()))


def test_normal_equations_are_block_tridiagonal_and_match_least_squares():
    prob = make_instance(152, 0, 5, 2, 30)
    sol = oracle.solve(prob)
    t0, t1 = 8, 19
    At, b = M.stacked_system(prob, t0, t1, sol["x"], sol["u"])
    n = 5
    AAt = At.T @ At
    nb = AAt.shape[0] // n
    for i in range(nb):
        for j in range(nb):
            if abs(i - j) > 1:
                assert not AAt[i * n:(i + 1) * n, j * n:(j + 1) * n].any()
    # diagonal blocks: I for lam_0, Sigma = I + A A' + B B' inside, I for mu
    A, B = prob["A"], prob["B"]
    np.testing.assert_allclose(AAt[:n, :n], np.eye(n))
    s = 3
    t = t0 + s - 1
    np.testing.assert_allclose(AAt[s * n:(s + 1) * n, s * n:(s + 1) * n],
                               np.eye(n) + A[t] @ A[t].T + B[t] @ B[t].T, atol=1e-14)
    np.testing.assert_allclose(AAt[-n:, -n:], np.eye(n))
    z_ls, *_ = np.linalg.lstsq(At, b, rcond=None)
    lam, mu = M.segment_multipliers(prob, t0, t1, sol["x"], sol["u"])
    z = np.concatenate([lam.ravel(), mu])
    np.testing.assert_allclose(z, z_ls, rtol=0, atol=1e-10 * (1 + np.abs(z_ls).max()))
    assert np.abs(At @ z - b).max() < 1e-10 * (1 + np.abs(b).max())


def test_block_solve_on_a_random_spd_system():
    rng = np.random.default_rng(3)
    n, N = 3, 6
    D, L = [], []
    big = np.zeros((N * n, N * n))
    for i in range(N):
        X = rng.standard_normal((n, n))
        D.append(X @ X.T + 4 * n * np.eye(n))
        big[i * n:(i + 1) * n, i * n:(i + 1) * n] = D[-1]
    for i in range(N - 1):
        L.append(rng.standard_normal((n, n)))
        big[(i + 1) * n:(i + 2) * n, i * n:(i + 1) * n] = L[-1]
        big[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = L[-1].T
    rhs = rng.standard_normal(N * n)
    z = np.concatenate(M.block_tridiagonal_solve(D, L, [rhs[i * n:(i + 1) * n] for i in range(N)]))
    np.testing.assert_allclose(z, np.linalg.solve(big, rhs), atol=1e-12)


@pytest.mark.parametrize("mutant", ["flip_A", "flip_mu"])
def test_planted_mistakes_break_the_pins(mutant, monkeypatch):
    prob = make_instance(153, 0, 4, 2, 18)
    sol = oracle.solve(prob)
    x, u, lam = sol["x"], sol["u"], _costate(sol)
    orig = M.stacked_system

    def broken(prob, t0, t1, x, u, end_constraint=True):
        At, b = orig(prob, t0, t1, x, u, end_constraint)
        n, m = prob["B"].shape[1], prob["B"].shape[2]
        T = t1 - t0
        if mutant == "flip_A":     # +A' instead of -A' in stage 2's x-rows
            r0 = 2 * (n + m)
            At[r0:r0 + n, 3 * n:4 * n] *= -1.0
        else:                      # end-point multiplier with the wrong sign
            At[T * (n + m):, (T + 1) * n:] *= -1.0
        return At, b

    monkeypatch.setattr(M, "stacked_system", broken)
    lam_s, mu = M.segment_multipliers(prob, 6, 12, x, u)
    ok_lam = np.allclose(lam_s, -lam[6:13], atol=1e-8)
    ok_mu = np.allclose(mu, lam[12], atol=1e-8)
    assert not (ok_lam and ok_mu)
