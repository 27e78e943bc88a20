"""The C-ABI library loads and exports what include/mi355lqr.h declares (no GPU).

Also checks that the ctypes mirror of every struct has the C layout (a tiny C
program compiled with gcc prints sizeof/offsetof from the header), and the
host-side argument validation of the entry points, none of which launches a
kernel.
"""

import ctypes
import os
import re
import subprocess

import pytest

import paper_1809_06360_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi355lqr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.library()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_struct_layouts_match_the_header(tmp_path):
    fields = {"lqr_problem_t": L.LqrProblem, "lqr_options_t": L.LqrOptions, "lqr_grad_t": L.LqrGrad}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mi355lqr.h"', 'int main(void) {']
    for cname, py in fields.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, py in fields.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_status_strings():
    for code in range(8):
        assert L.lqr_status_string(code)
    assert L.lqr_status_string(0) == "success"


def _prob(n=4, m=2, T=8, J=0):
    return L.LqrProblem(n, m, T, J)


@pytest.mark.parametrize("n,m,T,J", [(0, 1, 4, 0), (2, 0, 4, 0), (2, 1, 0, 0), (2, 1, 4, 5), (2, 1, 4, -1)])
def test_workspace_size_rejects_bad_dimensions(n, m, T, J):
    with pytest.raises(L.LQRError) as e:
        L.lqr_workspace_size(ctypes.byref(_prob(n, m, T, J)), 1, L.options())
    assert e.value.status == L.ERR_INVALID_ARG


def test_workspace_size_rejects_bad_options():
    opts = L.options()
    opts.flags = 4          # only LQR_FLAG_PHASED (1) and LQR_FLAG_SMOOTHED (2) are defined
    with pytest.raises(L.LQRError) as e:
        L.lqr_workspace_size(ctypes.byref(_prob()), 1, opts)
    assert e.value.status == L.ERR_INVALID_ARG
    with pytest.raises(L.LQRError) as e:     # smoothing needs the segmented algorithm
        L.lqr_workspace_size(ctypes.byref(_prob()), 1, L.options(algo="serial", smoothed=True))
    assert e.value.status == L.ERR_INVALID_ARG
    assert L.lqr_workspace_size(ctypes.byref(_prob()), 1, L.options(smoothed=True)) == \
        L.lqr_workspace_size(ctypes.byref(_prob()), 1, L.options())
    with pytest.raises(L.LQRError):
        L.lqr_workspace_size(ctypes.byref(_prob()), 0, L.options())


def test_workspace_size_is_machine_independent_and_monotone():
    (J,), _ = L.lqr_plan_segments(ctypes.byref(_prob(48, 24, 1024, 0)), 1, L.options())
    assert 1 < J <= 1024
    a = L.lqr_workspace_size(ctypes.byref(_prob(48, 24, 1024, J)), 1, L.options())
    b = L.lqr_workspace_size(ctypes.byref(_prob(48, 24, 1024, 0)), 1, L.options())
    c = L.lqr_workspace_size(ctypes.byref(_prob(48, 24, 1024, max(1, J // 2))), 1, L.options())
    assert a == b     # segments = 0 means the planner's choice
    assert c < a
    arr = (L.LqrProblem * 2)(_prob(8, 4, 64, 4), _prob(12, 3, 50, 7))
    both = L.lqr_workspace_size(arr, 2, L.options())
    assert both > L.lqr_workspace_size(ctypes.byref(arr[1]), 1, L.options())


def test_solve_rejects_null_pointers_and_small_workspace():
    prob = _prob(4, 2, 8, 2)
    with pytest.raises(L.LQRError) as e:     # all data pointers NULL
        L.lqr_solve(prob, L.options(), 256, 1 << 20, 0)
    assert e.value.status == L.ERR_INVALID_ARG
    for name in ("A", "B", "c", "Q", "q", "R", "r", "x0", "K", "k", "x", "u", "info"):
        setattr(prob, name, 256)
    prob.lam = 256        # the costate needs P and p
    with pytest.raises(L.LQRError) as e:
        L.lqr_solve(prob, L.options(), 256, 1 << 20, 0)
    assert e.value.status == L.ERR_INVALID_ARG
    prob.lam = None
    with pytest.raises(L.LQRError) as e:
        L.lqr_solve(prob, L.options(), 256, 16, 0)
    assert e.value.status == L.ERR_WORKSPACE
    with pytest.raises(L.LQRError) as e:
        L.lqr_solve(prob, L.options(), None, 1 << 20, 0)
    assert e.value.status == L.ERR_WORKSPACE


@pytest.mark.parametrize("n,m", [(129, 4), (8, 65), (65, 65), (200, 100)])
def test_sizes_beyond_the_kernels_are_unsupported(n, m):
    """Up to 64 inputs (the input Hessian's factorization holds a column per
    lane) and up to 128 states (the large-state kernels); larger problems are
    rejected at planning time, for every algorithm."""
    for algo in ("parallel", "serial"):
        with pytest.raises(L.LQRError) as e:
            L.lqr_workspace_size(ctypes.byref(_prob(n, m, 16, 0)), 1, L.options(algo=algo))
        assert e.value.status == L.ERR_UNSUPPORTED


@pytest.mark.parametrize("n,m,T,J", [(65, 4, 16, 0), (128, 64, 2048, 128), (100, 1, 7, 7), (128, 64, 40, 1)])
def test_large_state_instances_are_planned_alone(n, m, T, J):
    """65..128 states run the large-state kernels: a single instance (through
    lqr_solve, or lqr_solve_batched with a batch of one) for every precision
    and algorithm; in a batch with other instances it is refused."""
    for prec in ("fp64", "mixed", "fp32"):
        for algo in ("parallel", "serial"):
            assert L.lqr_workspace_size(ctypes.byref(_prob(n, m, T, J)), 1, L.options(prec, algo)) > 0
    (got,), _ = L.lqr_plan_segments(ctypes.byref(_prob(n, m, T, J)), 1, L.options())
    assert got == (J if J else max(1, min(256, T, (T + 8) // 16)))
    arr = (L.LqrProblem * 2)(_prob(n, m, T, J), _prob(8, 4, 32, 0))
    with pytest.raises(L.LQRError) as e:
        L.lqr_workspace_size(arr, 2, L.options())
    assert e.value.status == L.ERR_UNSUPPORTED


def test_oversized_problem_is_unsupported_not_crashing():
    with pytest.raises(L.LQRError) as e:
        L.lqr_workspace_size(ctypes.byref(_prob(200, 100, 16, 0)), 1, L.options())
    assert e.value.status == L.ERR_UNSUPPORTED


def test_every_named_workload_fits_the_device_limits():
    """The planner accepts every instance of the named workloads (LDS
    footprints within the 160 KiB a gfx950 workgroup may allocate)."""
    from synthetic import WORKLOADS
    for key in ("small", "large", "batched", "mixed", "diff"):
        w = WORKLOADS[key]
        arr = (L.LqrProblem * w.batch)(*[L.LqrProblem(n, m, T, w.segments) for (n, m, T) in w.dims])
        assert L.lqr_workspace_size(arr, w.batch, L.options(w.precision)) > 0, key


def test_backward_rejects_bad_arguments():
    prob = _prob(4, 2, 8, 1)
    arr = (L.LqrProblem * 1)(prob)
    grads = (L.LqrGrad * 1)()
    with pytest.raises(L.LQRError) as e:      # forward outputs missing
        L.lqr_backward(arr, 1, grads, L.options(), 256, 1 << 20, 0)
    assert e.value.status == L.ERR_INVALID_ARG
    for name in ("A", "B", "K", "P", "x", "u", "lam", "chol"):
        setattr(arr[0], name, 256)
    with pytest.raises(L.LQRError) as e:      # upstream gradients missing
        L.lqr_backward(arr, 1, grads, L.options(), 256, 1 << 20, 0)
    assert e.value.status == L.ERR_INVALID_ARG
    grads[0].dl_dx = 256
    grads[0].dl_du = 256
    with pytest.raises(L.LQRError) as e:      # workspace too small
        L.lqr_backward(arr, 1, grads, L.options(), 256, 8, 0)
    assert e.value.status == L.ERR_WORKSPACE


def test_plan_segments_respects_fixed_counts_and_algorithm():
    dims = [(4, 2, 64), (48, 24, 1024), (12, 3, 50), (60, 30, 400)]
    segs, est = L.plan_segments(dims, segments=[4, 64, 0, 0])
    assert segs[0] == 4 and segs[1] == 64
    assert all(1 <= J <= T for J, (_, _, T) in zip(segs, dims))
    assert est > 0
    serial, est_s = L.plan_segments(dims, algo="serial")
    assert serial == [1] * 4 and est_s == 0.0
    again, est2 = L.plan_segments(dims, segments=[4, 64, 0, 0])
    assert again == segs and est2 == est          # deterministic (and cached)
    with pytest.raises(L.LQRError) as e:
        L.plan_segments([(4, 2, 10)], segments=[11])
    assert e.value.status == L.ERR_INVALID_ARG


def test_planner_splits_long_single_instances_more_than_short_ones():
    (j_long,), _ = L.plan_segments([(16, 8, 4096)])
    (j_short,), _ = L.plan_segments([(16, 8, 64)])
    assert j_long > j_short >= 1
    # a batch that fills the device on its own needs no splitting
    segs, _ = L.plan_segments([(16, 8, 128)] * 512)
    assert set(segs) == {1}


def test_precision_modes():
    """FP64 and mixed precision plan the same workspace; FP32 adds the staging
    area; the mixed-precision workload (n = 128, m = 64, T = 2048, J = 128)
    is planned with its 128 segments."""
    a = L.lqr_workspace_size(ctypes.byref(_prob(48, 24, 1024, 64)), 1, L.options("fp64"))
    b = L.lqr_workspace_size(ctypes.byref(_prob(48, 24, 1024, 64)), 1, L.options("mixed"))
    assert a == b
    # FP32 stages the float arrays as doubles in the workspace
    c = L.lqr_workspace_size(ctypes.byref(_prob(48, 24, 1024, 64)), 1, L.options("fp32"))
    assert c > a
    prob = _prob(4, 2, 8, 2)
    for name in ("A", "B", "c", "Q", "q", "R", "r", "x0", "K", "k", "x", "u", "info"):
        setattr(prob, name, 256)
    with pytest.raises(L.LQRError) as e:     # the phase-by-phase entry works on FP64 arrays
        L.lqr_solve_phase(prob, L.options("fp32"), 1, 256, 1 << 30, 0)
    assert e.value.status == L.ERR_UNSUPPORTED
    from synthetic import WORKLOADS
    (n, m, T), = WORKLOADS["mixed"].dims
    J = WORKLOADS["mixed"].segments
    assert L.lqr_workspace_size(ctypes.byref(_prob(n, m, T, J)), 1, L.options("mixed")) > 0
    (got,), _ = L.lqr_plan_segments(ctypes.byref(_prob(n, m, T, J)), 1, L.options("mixed"))
    assert got == J == 128


@pytest.mark.parametrize("dims", [
    [(4, 2, 64, 4)],
    [(48, 24, 1024, 64)],
    [(8, 4, 32, 0), (20, 7, 50, 5), (1, 1, 5, 0), (64, 32, 48, 6)],
    [(16, 8, 128, 1)] * 37,
])
def test_workspace_plan_regions_are_disjoint(dims):
    """lqr_backward's plan and lqr_solve_batched's plan of one problem set sit
    in disjoint regions before the scratch region, for every option set, and
    each plan fits its region; the regions depend on the problem set only, so
    every call on it agrees on them."""
    arr = (L.LqrProblem * len(dims))(*[L.LqrProblem(n, m, T, J) for (n, m, T, J) in dims])
    seen = None
    for prec in ("fp64", "mixed", "fp32"):
        for algo in ("parallel", "serial"):
            for phased in (False, True):
                lay = L.lqr_workspace_layout(arr, len(dims), L.options(prec, algo, phased))
                a0, a1 = lay["adj_off"], lay["adj_off"] + lay["adj_cap"]
                f0, f1 = lay["fwd_off"], lay["fwd_off"] + lay["fwd_cap"]
                assert a1 <= f0 or f1 <= a0, lay                 # disjoint plan regions
                assert lay["scratch_off"] >= max(a1, f1), lay     # scratch after both
                assert 0 < lay["adj_plan"] <= lay["adj_cap"], lay
                assert 0 < lay["fwd_plan"] <= lay["fwd_cap"], lay
                assert lay["total"] == L.lqr_workspace_size(arr, len(dims), L.options(prec, algo, phased))
                assert lay["total"] > lay["scratch_off"]
                regions = (a0, a1, f0, f1, lay["scratch_off"])
                assert seen is None or regions == seen, (prec, algo, phased)
                seen = regions


def test_link_multipliers_checks_its_arguments_on_the_host():
    """lqr_link_multipliers rejects a segment count outside 1..T, missing
    outputs and n above 128 before it touches the device, and J = 1 (no link
    point) is a no-op."""
    prob = _prob(4, 2, 8, 2)
    L.lqr_link_multipliers(prob, L.options(), 1, None, 0)        # nothing to write
    for J in (0, 9):
        with pytest.raises(L.LQRError) as e:
            L.lqr_link_multipliers(prob, L.options(), J, 256, 0)
        assert e.value.status == L.ERR_INVALID_ARG
    with pytest.raises(L.LQRError) as e:                      # P, p, x are NULL
        L.lqr_link_multipliers(prob, L.options(), 2, 256, 0)
    assert e.value.status == L.ERR_INVALID_ARG
    prob.P = prob.p = prob.x = 256
    with pytest.raises(L.LQRError) as e:                      # no output array
        L.lqr_link_multipliers(prob, L.options(), 2, None, 0)
    assert e.value.status == L.ERR_INVALID_ARG
    big = _prob(129, 2, 8, 2)
    big.P = big.p = big.x = 256
    with pytest.raises(L.LQRError) as e:
        L.lqr_link_multipliers(big, L.options(), 2, 256, 0)
    assert e.value.status == L.ERR_INVALID_ARG


def test_smoothed_policies_are_refused_where_they_are_not_built():
    """LQR_FLAG_SMOOTHED is rejected by the batched and adjoint calls before
    they touch the device."""
    arr = (L.LqrProblem * 1)(_prob(4, 2, 8, 2))
    with pytest.raises(L.LQRError) as e:
        L.lqr_solve_batched(arr, 1, L.options(smoothed=True), 256, 1 << 20, 0)
    assert e.value.status == L.ERR_UNSUPPORTED
    grads = (L.LqrGrad * 1)()
    with pytest.raises(L.LQRError) as e:
        L.lqr_backward(arr, 1, grads, L.options(smoothed=True), 256, 1 << 20, 0)
    assert e.value.status == L.ERR_UNSUPPORTED


def test_python_constants_match_the_header():
    """The binding's status, precision, info and flag constants are the
    header's #define and enum values."""
    text = open(HEADER).read()
    defines = {k: int(v, 0) for k, v in re.findall(r"#define\s+(LQR_\w+)\s+\(?(-?0x[0-9a-fA-F]+|-?\d+)u?\)?", text)}
    assert defines["LQR_FLAG_PHASED"] == L.FLAG_PHASED
    assert defines["LQR_FLAG_SMOOTHED"] == L.FLAG_SMOOTHED
    assert defines["LQR_INFO_COUPLING"] == L.INFO_COUPLING
    assert defines["LQR_INFO_QUEUE"] == L.INFO_QUEUE
    assert defines["LQR_INFO_NONFINITE"] == L.INFO_NONFINITE
    enums = {k: int(v) for k, v in re.findall(r"(LQR_(?:PREC|ALGO)_\w+)\s*=\s*(\d+)", text)}
    assert (enums["LQR_PREC_FP64"], enums["LQR_PREC_MIXED"], enums["LQR_PREC_FP32"]) == \
        (L.PREC_FP64, L.PREC_MIXED, L.PREC_FP32)
    assert (enums["LQR_ALGO_PARALLEL"], enums["LQR_ALGO_SERIAL"]) == (L.ALGO_PARALLEL, L.ALGO_SERIAL)
