"""GPU parity of the large-state path (65..128 states, up to 64 inputs:
512-thread workgroups, products on matrix cores fed from the workspace, FP64
input-Hessian factorizations and linking solve) against the CPU oracle.

FP64 cases at 1e-9 on short horizons (ragged sizes, one-stage segments, one
segment, the serial kernel, a cross term); the mixed-precision workload at its
full size (n = 128, m = 64, T = 2048, J = 128, FP32 matrix-core products with
float accumulation) at 1e-4 on every output; the FP32 mode; info codes.
"""

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, MIXED_TOL, compare, host, to_device
from synthetic import WORKLOADS, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve(prob, **kw):
    import paper_1809_06360_amd as L
    out = L.solve(to_device(prob), **kw)
    torch.cuda.synchronize()
    return host(out)


FP64_CASES = [
    # (n, m, T, J, cross)
    (128, 64, 48, 6, False),
    (72, 20, 37, 5, True),      # ragged: 37 stages over 5 segments
    (128, 1, 9, 9, False),      # one stage per segment, one input
    (97, 33, 30, 1, False),     # single segment
    (65, 64, 24, 4, False),
    (120, 7, 50, 16, True),
]


@pytest.mark.parametrize("n,m,T,J,cross", FP64_CASES)
def test_large_fp64_matches_oracle(n, m, T, J, cross):
    prob = make_instance(160, n * 1000 + m, n, m, T, cross_term=cross)
    ref = oracle.solve(prob)
    got = _solve(prob, segments=J, with_chol=True)
    assert int(got["info"][0]) == 0
    compare(got, ref, label="fp64 large %s" % ((n, m, T, J),))
    # Cholesky factors of the input Hessians (row-major, lower)
    t = T // 2
    H = prob["R"][t] + prob["B"][t].T @ ref["P"][t + 1] @ prob["B"][t]  # the cross term enters H_ux only
    Lt = got["chol"][t]
    assert np.allclose(np.triu(Lt, 1), 0.0)
    assert np.linalg.norm(Lt @ Lt.T - H) <= 1e-11 * np.linalg.norm(H)


@pytest.mark.parametrize("n,m,T", [(128, 64, 40), (80, 17, 25)])
def test_large_serial_kernel_matches_oracle(n, m, T):
    prob = make_instance(161, n, n, m, T)
    got = _solve(prob, algo="serial")
    assert int(got["info"][0]) == 0
    compare(got, oracle.solve(prob), label="serial large %s" % ((n, m, T),))


def test_large_single_segment_equals_serial_kernel_bitwise():
    prob = make_instance(162, 0, 90, 12, 20)
    a = _solve(prob, segments=1)
    b = _solve(prob, algo="serial")
    for k in ("K", "k", "P", "p", "x", "u", "lam"):
        assert np.array_equal(a[k], b[k]), k


def test_mixed_workload_full_size_matches_oracle():
    """The mixed-precision workload exactly as the benchmark runs it."""
    w = WORKLOADS["mixed"]
    (n, m, T), = w.dims
    prob = make_instance(w.cfg, 0, n, m, T)
    got = _solve(prob, segments=w.segments, precision="mixed")
    assert int(got["info"][0]) == 0
    errs = compare(got, oracle.solve(prob), tol=MIXED_TOL, label=w.name)
    print(w.name, {k: "%.2e" % v for k, v in errs.items()})


@pytest.mark.parametrize("n,m,T,J", [(128, 64, 64, 8), (100, 30, 33, 4)])
def test_large_mixed_and_fp32_match_oracle(n, m, T, J):
    prob = make_instance(163, n, n, m, T)
    ref = oracle.solve(prob)
    got = _solve(prob, segments=J, precision="mixed")
    compare(got, ref, tol=MIXED_TOL, label="mixed %s" % ((n, m, T, J),))
    import paper_1809_06360_amd as L
    out = L.solve(to_device(prob, dtype=torch.float32), segments=J, precision="fp32")
    torch.cuda.synchronize()
    assert out["x"].dtype == torch.float32
    compare(host(out), ref, tol=MIXED_TOL, label="fp32 %s" % ((n, m, T, J),))


def test_large_batch_of_one_and_phases():
    """lqr_solve_batched with one large instance, and the phase-by-phase entry,
    give lqr_solve's results bitwise."""
    import ctypes
    import paper_1809_06360_amd as L
    prob = make_instance(164, 0, 70, 9, 30)
    a = _solve(prob, segments=5)
    outs, _ = L.solve_batched([to_device(prob)], segments=[5])
    torch.cuda.synchronize()
    b = host(outs[0])
    data = to_device(prob)
    out = L._outputs(70, 9, 30, torch.float64, data["A"].device, True, True, False)
    pr = L._problem(data, out, 5)
    opts = L.options()
    nb = L.lqr_workspace_size(ctypes.byref(pr), 1, opts)
    ws = torch.empty(nb, dtype=torch.uint8, device=data["A"].device)
    s = torch.cuda.current_stream().cuda_stream
    for ph in (1, 2, 3):
        L.lqr_solve_phase(pr, opts, ph, ws.data_ptr(), nb, s)
    torch.cuda.synchronize()
    c = host(out)
    for k in ("K", "k", "P", "p", "x", "u", "lam"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


@pytest.mark.parametrize("J,algo", [(1, "serial"), (4, "parallel"), (12, "parallel")])
def test_large_info_codes(J, algo):
    import paper_1809_06360_amd as L
    prob = make_instance(165, 0, 80, 6, 24)
    prob["R"][9] = -40.0 * np.eye(6)
    assert oracle.solve(prob)["info"] == 10
    assert int(_solve(prob, segments=J, algo=algo)["info"][0]) == 10
    prob = make_instance(165, 1, 80, 6, 24)
    prob["q"][11, 3] = np.nan
    assert int(_solve(prob, segments=J, algo=algo)["info"][0]) == L.INFO_NONFINITE
