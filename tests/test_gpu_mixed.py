"""GPU parity of the mixed-precision mode (FP32 matrix-core products with
float accumulation; Cholesky factorization of the input Hessian, gains and
linking solve in FP64) against the FP64 oracle, output by output, at the
relative-error bound of 1e-4."""

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, MIXED_TOL, OUTPUTS, compare, host, rel_err, to_device
from synthetic import WORKLOADS, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mixed(prob, segments, algo="parallel"):
    import paper_1809_06360_amd as L
    out = L.solve(to_device(prob), segments=segments, precision="mixed", algo=algo)
    torch.cuda.synchronize()
    return host(out)


@pytest.mark.parametrize("n,m,T,J,cross", [
    (4, 2, 64, 4, False), (5, 3, 40, 4, False), (20, 7, 50, 7, False), (33, 17, 40, 5, True),
    (56, 8, 48, 6, False), (64, 8, 48, 1, False), (12, 24, 30, 30, False), (48, 24, 200, 13, False)])
def test_mixed_matches_fp64_oracle(n, m, T, J, cross):
    prob = make_instance(70, n, n, m, T, cross_term=cross)
    got = _mixed(prob, J)
    assert int(got["info"][0]) == 0
    errs = compare(got, oracle.solve(prob), tol=MIXED_TOL, label="mixed %s" % ((n, m, T, J),))
    # the products really ran in float: the error is far above FP64 rounding
    # (at n, m <= 16 the small-size kernels compute in double for every precision)
    if max(n, m) > 16:
        assert max(errs.values()) > 1e-12
    else:
        assert max(errs.values()) < 1e-12


def test_mixed_serial_kernel_matches_oracle():
    prob = make_instance(71, 0, 24, 6, 300)
    got = _mixed(prob, 0, algo="serial")
    compare(got, oracle.solve(prob), tol=MIXED_TOL)


def test_mixed_large_workload_shape():
    w = WORKLOADS["large"]
    (n, m, T), = w.dims
    prob = make_instance(w.cfg, 0, n, m, T)
    got = _mixed(prob, w.segments)
    errs = compare(got, oracle.solve(prob), tol=MIXED_TOL)
    print("mixed large: " + " ".join("%s %.1e" % kv for kv in errs.items()))


def test_mixed_batched_persistent_and_phased():
    import paper_1809_06360_amd as L
    dims = [(16, 8, 96, 0), (40, 20, 160, 0), (7, 3, 33, 3), (60, 30, 64, 1)]
    probs = [make_instance(72, i, n, m, T) for i, (n, m, T, _) in enumerate(dims)]
    datas = [to_device(p) for p in probs]
    segs = [d[3] for d in dims]
    per, _ = L.solve_batched(datas, segments=segs, precision="mixed")
    pha, _ = L.solve_batched(datas, segments=segs, precision="mixed", phased=True)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        a, b = host(per[i]), host(pha[i])
        compare(a, oracle.solve(p), tol=MIXED_TOL, label="batched mixed %d" % i)
        for k in OUTPUTS:
            assert np.array_equal(a[k], b[k]), (i, k)


def test_backward_after_mixed_forward_is_close():
    """lqr_backward computes in FP64 from the forward outputs it is given; after
    a mixed-precision forward its gradient is within the mixed bound of the
    oracle's."""
    import paper_1809_06360_amd as L
    prob = make_instance(73, 0, 6, 3, 24)
    data = to_device(prob)
    outs, _ = L.solve_batched([data], segments=[3], precision="mixed", with_chol=True)
    g = L.backward([data], outs, [2.0 * outs[0]["x"]], [2.0 * outs[0]["u"]],
                   which=("A", "B", "q", "x0"))[0]
    torch.cuda.synchronize()
    sol = oracle.solve(prob)
    ref = oracle.backward(prob, sol, 2.0 * sol["x"], 2.0 * sol["u"])
    for k in ("A", "B", "q", "x0"):
        assert rel_err(g[k].cpu().numpy(), ref[k]) <= MIXED_TOL, k
    assert FP64_TOL < MIXED_TOL
