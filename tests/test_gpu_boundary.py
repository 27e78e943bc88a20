"""Boundary behaviour on the GPU: the info codes of non-finite data, and one
workspace shared by calls and graphs.

Non-finite inputs must be reported as LQR_INFO_NONFINITE (negative), distinct
from an input Hessian that is not positive definite (t + 1), on every launch
path. A workspace that serves lqr_solve_batched and lqr_backward of the same
problem set keeps both plans (disjoint regions), so their graphs replay in any
order after eager calls; a call on another problem set invalidates them, and a
capture that relies on a plan that is no longer resident is rejected.
"""

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, compare, host, rel_err, to_device
from synthetic import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PATHS = [("serial", 1, False), ("parallel", 1, False), ("parallel", 3, False),
         ("parallel", 10, False), ("parallel", 10, True)]


def _solve_info(prob, algo, J, batched):
    import paper_1809_06360_amd as L
    if batched:  # persistent launch (two instances so that J = 10 is kept)
        other = make_instance(140, 1, 4, 2, 12)
        outs, _ = L.solve_batched([to_device(prob), to_device(other)], segments=[J, 3], algo=algo)
        torch.cuda.synchronize()
        assert int(outs[1]["info"][0]) == 0
        return int(outs[0]["info"][0])
    out = L.solve(to_device(prob), segments=J, algo=algo)
    torch.cuda.synchronize()
    return int(out["info"][0])


@pytest.mark.parametrize("algo,J,batched", PATHS)
@pytest.mark.parametrize("where", ["q_mid", "q_first", "A", "R_inf", "c", "x0", "Q_T"])
def test_nonfinite_input_is_reported(algo, J, batched, where):
    import paper_1809_06360_amd as L
    prob = make_instance(141, 0, 5, 3, 20)
    if where == "q_mid":
        prob["q"][9, 2] = np.nan
    elif where == "q_first":
        prob["q"][0, 1] = np.nan     # only p_0 and the costate at t = 0 see it
    elif where == "A":
        prob["A"][13, 1, 4] = np.nan
    elif where == "R_inf":
        prob["R"][4, 0, 0] = np.inf
    elif where == "c":
        prob["c"][17, 0] = np.nan
    elif where == "x0":
        prob["x0"][3] = np.nan
    else:
        prob["Q"][20, 0, 0] = np.nan
    assert _solve_info(prob, algo, J, batched) == L.INFO_NONFINITE


@pytest.mark.parametrize("algo,J,batched", PATHS)
def test_indefinite_stage_outranks_nonfinite(algo, J, batched):
    """An indefinite input Hessian at stage 6 yields info 7 even though it
    fills the outputs with NaN (which would otherwise read as non-finite)."""
    prob = make_instance(142, 0, 4, 2, 20)
    prob["R"][6] = -50.0 * np.eye(2)
    assert oracle.solve(prob)["info"] == 7
    assert _solve_info(prob, algo, J, batched) == 7


def test_forward_and_backward_graphs_share_a_workspace():
    """Forward (persistent launch) and adjoint captured on ONE workspace,
    replayed in both orders after eager calls; every replay matches the eager
    results bitwise and the oracle."""
    import paper_1809_06360_amd as L
    dims = [(6, 3, 40, 4), (20, 7, 50, 5), (12, 4, 33, 3)]
    probs = [make_instance(143, i, n, m, T) for i, (n, m, T, _) in enumerate(dims)]
    datas = [to_device(p) for p in probs]
    segs = [d[3] for d in dims]
    keys = ("A", "B", "c", "Q", "q", "R", "r", "x0")
    outs, ws = L.solve_batched(datas, segments=segs, with_chol=True)
    gx = [2.0 * o["x"] for o in outs]
    gu = [2.0 * o["u"] for o in outs]
    gs = L.backward(datas, outs, gx, gu, which=keys, workspace=ws)
    torch.cuda.synchronize()
    eager_x = [o["x"].clone() for o in outs]
    eager_g = [{k: g[k].clone() for k in keys} for g in gs]
    gf, gb = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(gf):
        L.solve_batched(datas, segments=segs, outputs=outs, workspace=ws)
    with torch.cuda.graph(gb):
        L.backward(datas, outs, gx, gu, which=keys, workspace=ws, outputs=gs)
    for rep in range(3):
        for o in outs:
            o["x"].zero_()
        for g in gs:
            g["A"].zero_()
        torch.cuda.synchronize()
        if rep == 1:           # backward graph first: it reads the forward's outputs
            gf.replay()
            L.backward(datas, outs, gx, gu, which=keys, workspace=ws, outputs=gs)
            gb.replay()
            gf.replay()
        else:
            gf.replay()
            gb.replay()
        torch.cuda.synchronize()
        for i in range(len(dims)):
            assert torch.equal(outs[i]["x"], eager_x[i]), (rep, i)
            for k in keys:
                assert torch.equal(gs[i][k], eager_g[i][k]), (rep, i, k)
    sol = oracle.solve(probs[1])
    ref = oracle.backward(probs[1], sol, 2.0 * sol["x"], 2.0 * sol["u"])
    compare(host(outs[1]), sol, keys=("x", "u", "K", "P"), tol=FP64_TOL)
    assert rel_err(gs[1]["A"].cpu().numpy(), ref["A"]) <= FP64_TOL


def test_capture_after_call_on_another_problem_set_is_rejected():
    """A single solve of a different problem on the same workspace overwrites
    the batched plan's region: a capture that relies on it must be refused
    (until an uncaptured batched call uploads the plan again)."""
    import paper_1809_06360_amd as L
    probs = [make_instance(144, i, 8, 4, 64) for i in range(6)]
    datas = [to_device(p) for p in probs]
    outs, ws = L.solve_batched(datas, segments=[4] * 6)
    torch.cuda.synchronize()
    other = make_instance(144, 9, 4, 2, 16)
    out = L.solve(to_device(other), segments=2, workspace=ws)
    torch.cuda.synchronize()
    assert out["_workspace"] is ws          # the single solve really used this workspace
    assert int(out["info"][0]) == 0
    g = torch.cuda.CUDAGraph()
    with pytest.raises(L.LQRError) as e:
        with torch.cuda.graph(g):
            L.solve_batched(datas, segments=[4] * 6, outputs=outs, workspace=ws)
    assert e.value.status == L.ERR_INVALID_ARG
    torch.cuda.synchronize()
    # an uncaptured call uploads the plan again; then capture and replay work
    L.solve_batched(datas, segments=[4] * 6, outputs=outs, workspace=ws)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        L.solve_batched(datas, segments=[4] * 6, outputs=outs, workspace=ws)
    outs[2]["x"].zero_()
    g2.replay()
    torch.cuda.synchronize()
    compare(host(outs[2]), oracle.solve(probs[2]), tol=FP64_TOL)


def test_lqr_function_backward_raises_on_failed_forward():
    import paper_1809_06360_amd as L
    probs = [make_instance(145, i, 4, 2, 12) for i in range(3)]
    probs[1]["q"][5, 0] = np.nan
    keys = ("A", "B", "c", "Q", "q", "R", "r", "x0")
    stack = {k: torch.stack([torch.from_numpy(p[k]) for p in probs]).cuda().requires_grad_(True)
             for k in keys}
    x, u = L.LQRFunction.apply(*(stack[k] for k in keys))
    loss = (x * x).sum() + (u * u).sum()
    with pytest.raises(L.LQRError) as e:
        loss.backward()
    assert e.value.status == L.ERR_NONFINITE
