"""GPU parity of the FP32 precision mode (float inputs and outputs; float
matrix-core products, double factorizations and linking solve; adjoint in
double on the staged arrays) against the FP64 oracle on the same data, at the
1e-4 relative-error bound of the reduced-precision modes."""

import pytest

import oracle
from gpu_util import MIXED_TOL, compare, host, oracle_map, rel_err, to_device
from synthetic import WORKLOADS, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")



def _dev32(prob):
    return to_device(prob, dtype=torch.float32)


@pytest.mark.parametrize("n,m,T,J,algo", [
    (6, 3, 24, 4, "parallel"), (16, 8, 128, 1, "parallel"), (16, 8, 128, 0, "serial"),
    (33, 6, 40, 3, "parallel"), (48, 24, 256, 16, "parallel")])
def test_fp32_solve_matches_fp64_oracle(n, m, T, J, algo):
    import paper_1809_06360_amd as L
    prob = make_instance(110, n, n, m, T)
    out = L.solve(_dev32(prob), segments=J, precision="fp32", algo=algo)
    torch.cuda.synchronize()
    got = host(out)
    assert out["x"].dtype == torch.float32
    assert int(got["info"][0]) == 0
    compare(got, oracle.solve(prob), tol=MIXED_TOL, label="fp32 %s" % ((n, m, T, J, algo),))


def test_fp32_batched_matches_oracle():
    import paper_1809_06360_amd as L
    dims = [(16, 8, 96), (40, 20, 160), (7, 3, 33), (12, 4, 64)]
    probs = [make_instance(111, i, *d) for i, d in enumerate(dims)]
    outs, _ = L.solve_batched([_dev32(p) for p in probs], precision="fp32")
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        compare(host(outs[i]), oracle.solve(p), tol=MIXED_TOL, label="fp32 batched %d" % i)


def test_fp32_backward_matches_oracle_gradient():
    import paper_1809_06360_amd as L
    probs = [make_instance(112, i, 16, 8, 128) for i in range(3)]
    datas = [_dev32(p) for p in probs]
    outs, _ = L.solve_batched(datas, precision="fp32", with_chol=True)
    gs = L.backward(datas, outs, [2.0 * o["x"] for o in outs], [2.0 * o["u"] for o in outs],
                    which=("A", "B", "c", "Q", "q", "R", "r", "x0"))
    torch.cuda.synchronize()
    for p, g in zip(probs, gs):
        sol = oracle.solve(p)
        ref = oracle.backward(p, sol, 2.0 * sol["x"], 2.0 * sol["u"])
        for k in ("A", "B", "c", "Q", "q", "R", "r", "x0"):
            assert g[k].dtype == torch.float32
            assert rel_err(g[k].cpu().numpy(), ref[k]) <= MIXED_TOL, k


def test_lqr_function_fp32_on_differentiable_workload():
    """All 512 instances of the differentiable workload in the FP32 mode:
    every state trajectory and every gradient against the FP64 oracle."""
    import paper_1809_06360_amd as L
    w = WORKLOADS["diff"]
    probs = [make_instance(w.cfg, i, *w.dims[i]) for i in range(w.batch)]
    keys = ("A", "B", "c", "Q", "q", "R", "r", "x0")
    stack = {k: torch.stack([torch.from_numpy(p[k]) for p in probs]).to("cuda", torch.float32)
             .requires_grad_(True) for k in keys}
    x, u = L.LQRFunction.apply(*(stack[k] for k in keys))
    loss = (x * x).sum() + (u * u).sum()
    loss.backward()
    torch.cuda.synchronize()
    def ref_of(p):
        sol = oracle.solve(p)
        return sol, oracle.backward(p, sol, 2.0 * sol["x"], 2.0 * sol["u"])
    refs = oracle_map(ref_of, probs)
    grads = {k: stack[k].grad.cpu().numpy() for k in keys}
    xs = x.detach().cpu().numpy()
    for i, (sol, ref) in enumerate(refs):
        assert rel_err(xs[i], sol["x"]) <= MIXED_TOL, i
        for k in keys:
            assert rel_err(grads[k][i], ref[k]) <= MIXED_TOL, (i, k)
