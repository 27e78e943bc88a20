"""lqr_solve_noalloc (the entry point that allocates nothing and uses the
library's own scratch array) against lqr_solve through the C ABI.

Two calls in a row on the same device share the array; the second is a
smaller problem, so it runs over what the first left behind. Both must equal
lqr_solve on the same inputs bitwise (same kernels, same launch sequence) and
match the oracle to the FP64 bound. A problem whose scratch exceeds the array
is refused with LQR_ERR_WORKSPACE before anything is launched.
"""

import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, compare, to_device
from synthetic import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OUTS = ("K", "k", "P", "p", "x", "u", "lam")


def _outputs(n, m, T, dev):
    e = lambda *s: torch.full(s, float("nan"), dtype=torch.float64, device=dev)  # noqa: E731
    return dict(K=e(T, m, n), k=e(T, m), P=e(T + 1, n, n), p=e(T + 1, n), x=e(T + 1, n), u=e(T, m),
                lam=e(T + 1, n), info=torch.full((1,), 12345, dtype=torch.int32, device=dev))


def _run_pair(prob_np, J, algo, smoothed=False):
    import paper_1809_06360_amd as L
    dev = torch.device("cuda:0")
    data = to_device(prob_np)
    T, n, m = prob_np["B"].shape
    opts = L.options("fp64", algo, smoothed=smoothed)
    stream = torch.cuda.current_stream(dev).cuda_stream
    a = _outputs(n, m, T, dev)
    pa = L._problem(data, a, J)
    L.lqr_solve_noalloc(pa, opts, stream)
    b = _outputs(n, m, T, dev)
    pb = L._problem(data, b, J)
    nbytes = L.lqr_workspace_size(ctypes.byref(pb), 1, opts)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    L.lqr_solve(pb, opts, ws.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("algo", ["parallel", "serial"])
def test_noalloc_matches_lqr_solve_on_two_calls_in_a_row(algo):
    big = make_instance(150, 0, 48, 24, 512)       # J = 32: logarithmic-depth linking
    small = make_instance(150, 1, 12, 5, 60)       # J = 5: serial linking
    for prob, J in ((big, 32), (small, 5)):
        a, b = _run_pair(prob, J, algo)
        assert int(a["info"][0]) == 0 and int(b["info"][0]) == 0
        for k in OUTS:
            assert torch.equal(a[k], b[k]), (algo, prob["B"].shape, k)
        got = {k: a[k].cpu().numpy() for k in OUTS}
        compare(got, oracle.solve(prob), tol=FP64_TOL, label="noalloc %s %s" % (algo, prob["B"].shape))


def test_noalloc_refuses_problems_larger_than_its_scratch():
    import paper_1809_06360_amd as L
    prob = L.LqrProblem(64, 32, 4096, 512)
    opts = L.options("fp64", "parallel")
    need = L.lqr_workspace_size(ctypes.byref(prob), 1, opts)
    assert need > L.NOALLOC_SCRATCH_BYTES
    for name in ("A", "B", "c", "Q", "q", "R", "r", "x0", "K", "k", "x", "u", "info"):
        setattr(prob, name, 256)          # never dereferenced: the size check comes first
    with pytest.raises(L.LQRError) as e:
        L.lqr_solve_noalloc(prob, opts, 0)
    assert e.value.status == L.ERR_WORKSPACE
    assert np.isfinite(need)


def test_noalloc_smoothed_policies_match_lqr_solve():
    """The smoothed-policy option through the no-allocation entry point: two
    calls in a row, bitwise equal to lqr_solve, gains equal to the oracle's
    smoothed family."""
    from oracle import policies as PO
    big = make_instance(151, 0, 48, 24, 192)       # J = 12: logarithmic-depth linking
    small = make_instance(151, 1, 12, 6, 96)       # J = 6: serial linking
    for prob, J in ((big, 12), (small, 6)):
        a, b = _run_pair(prob, J, "parallel", smoothed=True)
        assert int(a["info"][0]) == 0 and int(b["info"][0]) == 0
        for k in OUTS:
            assert torch.equal(a[k], b[k]), ("smoothed", prob["B"].shape, k)
        Ks, ks = PO.smoothed_policies(prob, J, oracle.solve(prob))
        got = {k: a[k].cpu().numpy() for k in ("K", "k")}
        compare(got, {"K": Ks, "k": ks}, keys=("K", "k"), tol=FP64_TOL,
                label="noalloc smoothed %s" % (prob["B"].shape,))
