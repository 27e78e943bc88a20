"""GPU parity of every (product engine, register width) kernel variant the
launcher can select, against the CPU oracle.

A launch's product engine follows from the largest state dimension and the
precision (FP64 vector ALUs below 32 states, FP64 matrix cores from 32, FP32
matrix cores in the mixed mode) and its register width from the largest input
dimension (padded to 8, 16, 24, 32, 48 or 64; the matrix-core engines start at
16). Each case below is a resident-layout size that selects one variant; it
runs the parallel algorithm with several segments and the plain serial kernel
through lqr_solve, and the persistent batched launch through lqr_solve_batched
(next to a small instance, which then runs padded to the same variant).
"""

import pytest

import oracle
from gpu_util import FP64_TOL, MIXED_TOL, compare, host, to_device
from synthetic import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (precision, n, m, T, J): engine / width selected
VARIANTS = [
    ("fp64", 10, 6, 40, 5),      # vector ALUs, width 8
    ("fp64", 14, 13, 40, 5),     # vector ALUs, width 16
    ("fp64", 20, 24, 36, 4),     # vector ALUs, width 24
    ("fp64", 12, 30, 36, 4),     # vector ALUs, width 32
    ("fp64", 24, 40, 30, 3),     # vector ALUs, width 48
    ("fp64", 16, 60, 30, 3),     # vector ALUs, width 64
    ("fp64", 40, 12, 40, 5),     # FP64 matrix cores, width 16
    ("fp64", 36, 20, 40, 5),     # FP64 matrix cores, width 24
    ("fp64", 33, 28, 40, 5),     # FP64 matrix cores, width 32
    ("fp64", 34, 44, 30, 3),     # FP64 matrix cores, width 48
    ("fp64", 32, 56, 30, 3),     # FP64 matrix cores, width 64
    ("mixed", 20, 5, 40, 5),     # FP32 matrix cores, width 16 (small n)
    ("mixed", 40, 20, 40, 5),    # FP32 matrix cores, width 24
    ("mixed", 36, 30, 40, 5),    # FP32 matrix cores, width 32
    ("mixed", 40, 40, 30, 3),    # FP32 matrix cores, width 48
    ("mixed", 36, 60, 30, 3),    # FP32 matrix cores, width 64
]


def _ids(v):
    return "%s-n%d-m%d-T%d-J%d" % v


@pytest.mark.parametrize("prec,n,m,T,J", VARIANTS, ids=[_ids(v) for v in VARIANTS])
def test_variant_matches_oracle(prec, n, m, T, J):
    import paper_1809_06360_amd as L
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    prob = make_instance(120, n * 100 + m, n, m, T)
    small = make_instance(121, n * 100 + m, 3, 2, 12)
    ref, ref_small = oracle.solve(prob), oracle.solve(small)
    label = "%s n=%d m=%d T=%d" % (prec, n, m, T)
    for algo, segs in (("parallel", J), ("serial", 0)):
        out = L.solve(to_device(prob), segments=segs, precision=prec, algo=algo)
        torch.cuda.synchronize()
        got = host(out)
        assert int(got["info"][0]) == 0, (algo, int(got["info"][0]))
        compare(got, ref, tol=tol, label="%s %s J=%d" % (label, algo, segs))
    outs, _ = L.solve_batched([to_device(prob), to_device(small)], segments=[J, 2], precision=prec)
    torch.cuda.synchronize()
    for o, r, what in ((outs[0], ref, "batched"), (outs[1], ref_small, "batched small")):
        got = host(o)
        assert int(got["info"][0]) == 0, what
        compare(got, r, tol=tol, label="%s %s" % (label, what))
