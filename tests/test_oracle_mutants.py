"""The oracle's pins must catch plausible mistakes (no GPU).

Each case plants one mistake -- a dropped term, a wrong sign, a wrong index, a
transposed operand -- into a private copy of the oracle's C source, builds it
with gcc, and checks that at least one pin (the dense KKT solve of eq. KKT, the
tail-problem definition of K_t/P_t, or the dense implicit-differentiation
gradient) rejects it. Nothing here touches the real oracle build.
"""

import os
import subprocess

import numpy as np
import pytest

import kkt_dense
import oracle
from synthetic import make_instance

SRC = os.path.join(os.path.dirname(oracle.__file__), "lqr_oracle.c")

MUTANTS = {
    "drop_offset_in_value": ("s += Pn[IDX(i, l, n)] * ct[l];", ""),
    "policy_sign": ("Kt[IDX(i, j, n)] = -sol[IDX(i, j, n + 1)];", "Kt[IDX(i, j, n)] = sol[IDX(i, j, n + 1)];"),
    "transposed_A": ("s += Pn[IDX(i, l, n)] * At[IDX(l, j, n)];", "s += Pn[IDX(i, l, n)] * At[IDX(j, l, n)];"),
    "drop_cross_term": ("double s = St ? St[IDX(i, j, n)] : 0.0;", "double s = 0.0;"),
    "terminal_index": ("memcpy(P + (size_t)T * nn, Q + (size_t)T * nn,", "memcpy(P + (size_t)T * nn, Q + (size_t)(T - 1) * nn,"),
    "drop_feedback_in_P": ("for (int l = 0; l < m; ++l) s += rhs[IDX(l, i, n + 1)] * Kt[IDX(l, j, n)];", ""),
    "drop_feedback_in_p": ("for (int l = 0; l < m; ++l) s += rhs[IDX(l, i, n + 1)] * kt[l];", ""),
    "rollout_drops_offset": ("double s = ct[i];", "double s = 0.0;"),
    "k_uses_wrong_rhs_column": ("kt[i] = -sol[IDX(i, n, n + 1)];", "kt[i] = -sol[IDX(i, 0, n + 1)];"),
    "grad_A_swapped_indices": ("-(lh1[i] * xt[j] + l1[i] * xht[j]);", "-(lh1[i] * xt[j] + l1[j] * xht[i]);"),
    "grad_c_wrong_time": ("dc[(size_t)t * n + i] = -lh1[i];", "dc[(size_t)t * n + i] = -lh[(size_t)t * n + i];"),
    "grad_Q_sign": ("= -0.5 * (xht[i] * xt[j] + xt[i] * xht[j]);", "= 0.5 * (xht[i] * xt[j] + xt[i] * xht[j]);"),
    "grad_B_drops_term": ("-(lh1[i] * ut[j] + l1[i] * uht[j]);", "-(lh1[i] * ut[j]);"),
}


def _pins_pass(lib) -> bool:
    """True if the mutant passes every pin (which would be a miss)."""
    for (n, m, T) in [(3, 2, 4), (4, 3, 5)]:
        prob = make_instance(300, n, n, m, T, cross_term=True)
        sol = oracle.solve(prob, lib=lib)
        if sol["info"] != 0:
            return False
        x, u, lam_paper = kkt_dense.solve(prob)
        for got, ref in ((sol["x"], x), (sol["u"], u), (sol["lam"], -lam_paper)):
            if not np.allclose(got, ref, rtol=1e-9, atol=1e-12):
                return False
        t0 = T // 2
        _, u0, l0 = kkt_dense.solve(kkt_dense.tail(prob, t0, np.zeros(n)))
        Kc, Pc = [], []
        for i in range(n):
            e = np.eye(n)[i]
            _, ui, li = kkt_dense.solve(kkt_dense.tail(prob, t0, e))
            Kc.append(ui[0] - u0[0])
            Pc.append(-(li[0] - l0[0]))
        if not (np.allclose(sol["K"][t0], np.array(Kc).T, rtol=1e-9, atol=1e-12) and
                np.allclose(sol["P"][t0], np.array(Pc).T, rtol=1e-9, atol=1e-12)):
            return False
        gx, gu = 2 * sol["x"], 2 * sol["u"]
        g = oracle.backward(prob, sol, gx, gu, lib=lib)
        ref = kkt_dense.grad(prob, gx, gu)
        for key, G in ref.items():
            if not np.allclose(g[key], G, rtol=1e-8, atol=1e-11):
                return False
    return True


def test_unmutated_copy_passes(tmp_path):
    so = tmp_path / "orig.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so), SRC, "-lm"])
    assert _pins_pass(oracle.open_library(str(so)))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not unique: %s" % name
    src = tmp_path / ("%s.c" % name)
    src.write_text(text.replace(old, new))
    so = tmp_path / ("%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-w", "-o", str(so), str(src), "-lm"])
    assert not _pins_pass(oracle.open_library(str(so))), "pins missed mutant %s" % name
