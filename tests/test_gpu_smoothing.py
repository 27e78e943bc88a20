"""Smoothed policies on the GPU (LQR_FLAG_SMOOTHED, Sec. III-A) against the
oracle's smoothed family (each segment before the last two re-run as a plain
Riccati recursion from the next segment's cost-to-go with its end fixed at
its link point; the segment before the last from the exact value):
  * K and k equal the oracle's smoothed gains;
  * x, u and the costate are still the optimal ones (the serial oracle);
  * the gains really differ from the serial-exact ones;
  * two segments (no inner segment to smooth from) give the serial gains.
Also the option's rejections on the serial algorithm, batched and adjoint
calls."""

import numpy as np
import pytest

import oracle
from oracle import policies as PO
from gpu_util import FP64_TOL, MIXED_TOL, compare, host, rel_err, to_device
from synthetic import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n,m,T,J,precision", [
    (6, 3, 48, 4, "fp64"),        # serial linking solve
    (16, 8, 256, 16, "fp64"),     # logarithmic-depth linking solve
    (48, 24, 192, 12, "fp64"),    # matrix-core variants
    (33, 17, 103, 9, "fp64"),     # ragged: T mod J != 0, n off the tile grid
    (12, 6, 96, 16, "mixed"),     # FP32 sweeps, FP64 seeds
])
def test_smoothed_gains_match_the_oracle(n, m, T, J, precision):
    import paper_1809_06360_amd as L
    prob = make_instance(180, 0, n, m, T)
    out = L.solve(to_device(prob), segments=J, precision=precision, smoothed=True)
    torch.cuda.synchronize()
    got = host(out)
    assert int(got["info"][0]) == 0
    ref = oracle.solve(prob)
    Ks, ks = PO.smoothed_policies(prob, J, ref)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    compare(got, {"K": Ks, "k": ks}, keys=("K", "k"), tol=tol, label="smoothed gains")
    compare(got, ref, keys=("x", "u", "lam"), tol=tol, label="smoothed trajectory")
    # the smoothed gains are not the serial-exact ones (the difference decays
    # geometrically with the segment length: these cases keep it well above
    # the tolerance)
    assert rel_err(got["K"], ref["K"]) > 10 * tol


def test_two_segments_give_the_serial_gains():
    import paper_1809_06360_amd as L
    prob = make_instance(181, 0, 8, 4, 40)
    out = L.solve(to_device(prob), segments=2, smoothed=True)
    torch.cuda.synchronize()
    got = host(out)
    assert int(got["info"][0]) == 0
    compare(got, oracle.solve(prob), label="smoothed, two segments")


def test_smoothed_option_rejections():
    """Serial algorithm: invalid; the large-state path (n above 64): not built.
    Batched and adjoint calls are refused on the host (test_abi)."""
    import paper_1809_06360_amd as L
    dev = to_device(make_instance(182, 0, 6, 3, 24))
    with pytest.raises(L.LQRError) as e:
        L.solve(dev, segments=1, algo="serial", smoothed=True)
    assert e.value.status == L.ERR_INVALID_ARG
    big = to_device(make_instance(183, 0, 80, 40, 24))
    with pytest.raises(L.LQRError) as e:
        L.solve(big, segments=3, smoothed=True)
    assert e.value.status == L.ERR_UNSUPPORTED
