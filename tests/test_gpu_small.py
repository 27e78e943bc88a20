"""The small-size plain recursion (n, m <= 16; one workgroup per instance with
16 x 16 zero-padded blocks) against the oracle's serial solve: every output
element by element (K, k, P, p, x, u, costates) and the Cholesky factor of
each stage's input Hessian, at the edges of the padding (n or m equal to 1
and to 16), ragged sizes, with and without the cross term, with optional
outputs left out, as single serial solves and as batches of uneven instances
(the one-segment batched path)."""

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, compare, host, oracle_map, to_device
from synthetic import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _check_chol(prob, got, ref):
    P = ref["P"]
    for t in range(prob["B"].shape[0]):
        R = 0.5 * (prob["R"][t] + prob["R"][t].T)
        H = R + prob["B"][t].T @ P[t + 1] @ prob["B"][t]
        L = got["chol"][t]
        assert np.allclose(np.triu(L, 1), 0.0)
        np.testing.assert_allclose(L, np.linalg.cholesky(H), rtol=0, atol=1e-11 * np.abs(H).max() ** 0.5)


@pytest.mark.parametrize("n,m,T,cross", [
    (1, 1, 5, True), (4, 2, 64, True), (16, 8, 128, True), (16, 16, 40, False),
    (7, 13, 33, True), (16, 1, 20, False), (3, 16, 17, True),
])
def test_small_serial_solve_matches_the_oracle(n, m, T, cross):
    import paper_1809_06360_amd as L
    prob = make_instance(190, 0, n, m, T, cross_term=cross)
    out = L.solve(to_device(prob), segments=1, algo="serial", with_chol=True)
    torch.cuda.synchronize()
    got = host(out)
    assert int(got["info"][0]) == 0
    ref = oracle.solve(prob)
    compare(got, ref, label="small serial %s" % ((n, m, T),))
    _check_chol(prob, got, ref)


def test_small_serial_without_optional_outputs():
    import paper_1809_06360_amd as L
    prob = make_instance(191, 0, 9, 5, 30)
    out = L.solve(to_device(prob), segments=1, algo="serial", with_P=False, with_lam=False)
    torch.cuda.synchronize()
    got = host(out)
    assert "P" not in got and "lam" not in got
    compare(got, oracle.solve(prob), keys=("K", "k", "x", "u"), label="small serial, no P")


@pytest.mark.parametrize("algo", ["serial", "parallel"])
def test_small_batch_of_uneven_instances(algo):
    import paper_1809_06360_amd as L
    rng = np.random.default_rng(5)
    probs = [make_instance(192, i, int(rng.integers(1, 17)), int(rng.integers(1, 17)),
                           int(rng.integers(1, 90)), cross_term=bool(i % 2)) for i in range(40)]
    outs, _ = L.solve_batched([to_device(p) for p in probs], segments=[1] * len(probs), algo=algo,
                              with_chol=True)
    torch.cuda.synchronize()
    refs = oracle_map(oracle.solve, probs)
    for p, o, r in zip(probs, outs, refs):
        got = host(o)
        assert int(got["info"][0]) == 0
        compare(got, r, label="small batch %s" % (p["B"].shape,))
        _check_chol(p, got, r)


def test_small_batch_mixed_with_a_larger_instance_takes_the_general_path():
    import paper_1809_06360_amd as L
    probs = [make_instance(193, 0, 8, 4, 20), make_instance(193, 1, 17, 4, 20)]
    outs, _ = L.solve_batched([to_device(p) for p in probs], segments=[1, 1])
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        compare(host(o), oracle.solve(p), label="general path %s" % (p["B"].shape,))


@pytest.mark.parametrize("n,m,T,J,algo,smoothed", [
    (6, 3, 40, 4, "parallel", False), (12, 8, 64, 8, "parallel", False),
    (12, 8, 64, 8, "parallel", True), (5, 2, 20, 1, "serial", False)])
def test_small_phase_by_phase_equals_lqr_solve(n, m, T, J, algo, smoothed):
    """lqr_solve_phase (phase by phase, the small-size kernels for phases 1
    and 3) gives lqr_solve's results bitwise, and the oracle's."""
    import ctypes
    import paper_1809_06360_amd as L
    prob = make_instance(194, 0, n, m, T, cross_term=True)
    a = host(L.solve(to_device(prob), segments=J, algo=algo, smoothed=smoothed))
    data = to_device(prob)
    out = L._outputs(n, m, T, torch.float64, data["A"].device, True, True, False)
    pr = L._problem(data, out, J)
    opts = L.options("fp64", algo, smoothed=smoothed)
    nb = L.lqr_workspace_size(ctypes.byref(pr), 1, opts)
    ws = torch.empty(nb, dtype=torch.uint8, device=data["A"].device)
    s = torch.cuda.current_stream().cuda_stream
    for ph in ((1,) if algo == "serial" else (1, 2, 3)):
        L.lqr_solve_phase(pr, opts, ph, ws.data_ptr(), nb, s)
    torch.cuda.synchronize()
    c = host(out)
    assert int(c["info"][0]) == 0
    for k in ("K", "k", "P", "p", "x", "u", "lam"):
        assert np.array_equal(a[k], c[k]), k
    ref = oracle.solve(prob)
    keys = ("x", "u", "lam") if smoothed else ("K", "k", "P", "p", "x", "u", "lam")
    compare(c, ref, keys=keys, label="small phases %s" % ((n, m, T, J, algo, smoothed),))
