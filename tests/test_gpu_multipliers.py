"""Link multipliers on the GPU (lqr_link_multipliers) against the oracle's
explicit multiplier route (Sec. II-B, eqs. mults, mu, pseudoinverse,
bandedAA: each inner segment's end-point multiplier from the normal
equations of its stationarity conditions, solved by block substitution), on
the serial linking solve, the logarithmic-depth one, the large-state path and
the FP32 mode."""

import numpy as np
import pytest

import oracle
from oracle import multipliers as OM
from gpu_util import host, to_device
from synthetic import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bounds(T, J):
    L, e = divmod(T, J)
    return [j * L + min(j, e) for j in range(J + 1)]


@pytest.mark.parametrize("n,m,T,J,precision,tol", [
    (6, 3, 40, 4, "fp64", 1e-9),        # serial linking solve
    (16, 8, 256, 16, "fp64", 1e-9),     # logarithmic-depth linking solve
    (48, 24, 192, 12, "fp64", 1e-9),    # matrix-core variants
    (80, 40, 96, 6, "fp64", 1e-9),      # large-state path
    (12, 6, 96, 8, "fp32", 1e-3),       # FP32 outputs
])
def test_link_multipliers_match_the_explicit_route(n, m, T, J, precision, tol):
    import paper_1809_06360_amd as L
    prob = make_instance(160, 0, n, m, T)
    dev = to_device(prob, dtype=torch.float32 if precision == "fp32" else torch.float64)
    out = L.solve(dev, segments=J, precision=precision)
    mu = L.link_multipliers(dev, out, segments=J, precision=precision)
    torch.cuda.synchronize()
    assert int(out["info"][0]) == 0
    ref_sol = oracle.solve(prob)
    b = _bounds(T, J)
    ref = OM.link_multipliers(prob, b, ref_sol["x"], ref_sol["u"])
    got = mu.cpu().numpy().astype(np.float64)
    assert got.shape == (J - 1, n)
    rel = np.abs(got - ref).max() / np.abs(ref).max()
    assert rel <= tol, rel
    # the same value as the solve's own costate output at the link points
    lam = host(out)["lam"].astype(np.float64)
    assert np.abs(got - lam[b[1:-1]]).max() / np.abs(ref).max() <= tol


def test_link_multipliers_argument_checks():
    import paper_1809_06360_amd as L
    prob = make_instance(161, 0, 5, 2, 20)
    dev = to_device(prob)
    out = L.solve(dev, segments=4)
    assert L.link_multipliers(dev, out, segments=1).shape == (0, 5)
    with pytest.raises(L.LQRError):
        L.link_multipliers(dev, out, segments=21)
    del out["P"]
    with pytest.raises(L.LQRError):
        L.link_multipliers(dev, out, segments=4)
