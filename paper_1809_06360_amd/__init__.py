"""MI355X-native parallel Riccati recursion for time-varying finite-horizon LQR.

Thin Python binding of the C ABI in ``include/mi355lqr.h`` (library
``libmi355lqr.so``, built in-tree for gfx950 by ``paper_1809_06360_amd.build``).
The functions ``lqr_workspace_size``, ``lqr_solve``, ``lqr_solve_batched``,
``lqr_backward`` and ``lqr_status_string`` mirror the C entry points and only
marshal arguments; every step of the solve runs in the library's HIP kernels.
PyTorch supplies device memory and the current stream.

There is no CPU fallback: if the library has not been built, loading it raises.
"""

from __future__ import annotations

import ctypes
import os

__all__ = [
    "LIB_PATH", "library", "LqrProblem", "LqrOptions", "LqrGrad",
    "lqr_workspace_size", "lqr_workspace_layout", "lqr_plan_segments", "lqr_solve",
    "lqr_solve_noalloc", "lqr_solve_phase", "lqr_solve_batched", "lqr_backward", "lqr_status_string",
    "solve", "solve_batched", "plan_segments", "backward", "LQRError",
    "SUCCESS", "PREC_FP64", "PREC_MIXED", "PREC_FP32", "ALGO_PARALLEL", "ALGO_SERIAL",
    "INFO_COUPLING", "INFO_QUEUE", "INFO_NONFINITE", "FLAG_PHASED", "FLAG_SMOOTHED",
    "link_multipliers",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmi355lqr.so")

SUCCESS, ERR_INVALID_ARG, ERR_NOT_PD, ERR_SINGULAR_COUPLING = 0, 1, 2, 3
ERR_NONFINITE, ERR_WORKSPACE, ERR_HIP, ERR_UNSUPPORTED = 4, 5, 6, 7
PREC_FP64, PREC_MIXED, PREC_FP32 = 0, 1, 2
ALGO_PARALLEL, ALGO_SERIAL = 0, 1
INFO_COUPLING = 0x40000000
INFO_QUEUE = 0x20000000
INFO_NONFINITE = -1
FLAG_PHASED = 0x1
FLAG_SMOOTHED = 0x2

_vp = ctypes.c_void_p


class LqrProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("T", ctypes.c_int32),
                ("segments", ctypes.c_int32)] + \
               [(name, _vp) for name in ("A", "B", "c", "Q", "q", "R", "r", "S", "x0",
                                         "K", "k", "P", "p", "x", "u", "lam", "chol", "info")]


class LqrOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("algo", ctypes.c_int), ("flags", ctypes.c_uint32)]


class LqrGrad(ctypes.Structure):
    _fields_ = [(name, _vp) for name in ("dl_dx", "dl_du", "dA", "dB", "dc", "dQ", "dq",
                                         "dR", "dr", "dS", "dx0")]


EXPORTS = ("lqr_workspace_size", "lqr_workspace_layout", "lqr_plan_segments", "lqr_solve",
           "lqr_solve_noalloc", "lqr_solve_phase", "lqr_solve_batched", "lqr_backward",
           "lqr_link_multipliers", "lqr_status_string")
NOALLOC_SCRATCH_BYTES = 32 << 20

_lib = None


class LQRError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (where, lqr_status_string(status), status))


def library():
    """Load ``libmi355lqr.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmi355lqr.so is not built; run `python -m paper_1809_06360_amd.build` "
                               "(or __graft_entry__.build()) first")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        lib.lqr_workspace_size.argtypes = [P(LqrProblem), ctypes.c_int32, P(LqrOptions), P(ctypes.c_size_t)]
        lib.lqr_workspace_size.restype = ctypes.c_int
        lib.lqr_workspace_layout.argtypes = [P(LqrProblem), ctypes.c_int32, P(LqrOptions),
                                             P(ctypes.c_size_t)]
        lib.lqr_workspace_layout.restype = ctypes.c_int
        lib.lqr_plan_segments.argtypes = [P(LqrProblem), ctypes.c_int32, P(LqrOptions), P(ctypes.c_int32),
                                          P(ctypes.c_double)]
        lib.lqr_plan_segments.restype = ctypes.c_int
        lib.lqr_solve.argtypes = [P(LqrProblem), P(LqrOptions), _vp, ctypes.c_size_t, _vp]
        lib.lqr_solve.restype = ctypes.c_int
        lib.lqr_solve_noalloc.argtypes = [P(LqrProblem), P(LqrOptions), _vp]
        lib.lqr_solve_noalloc.restype = ctypes.c_int
        lib.lqr_solve_phase.argtypes = [P(LqrProblem), P(LqrOptions), ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
        lib.lqr_link_multipliers.restype = ctypes.c_int
        lib.lqr_link_multipliers.argtypes = [P(LqrProblem), P(LqrOptions), ctypes.c_int32, _vp, _vp]
        lib.lqr_solve_phase.restype = ctypes.c_int
        lib.lqr_solve_batched.argtypes = [P(LqrProblem), ctypes.c_int32, P(LqrOptions), _vp,
                                          ctypes.c_size_t, _vp]
        lib.lqr_solve_batched.restype = ctypes.c_int
        lib.lqr_backward.argtypes = [P(LqrProblem), ctypes.c_int32, P(LqrGrad), P(LqrOptions), _vp,
                                     ctypes.c_size_t, _vp]
        lib.lqr_backward.restype = ctypes.c_int
        lib.lqr_status_string.argtypes = [ctypes.c_int]
        lib.lqr_status_string.restype = ctypes.c_char_p
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# C entry points, same names and arguments (structs by ctypes pointer/array).
# ---------------------------------------------------------------------------
def lqr_status_string(status: int) -> str:
    return library().lqr_status_string(int(status)).decode()


def lqr_workspace_size(probs, batch: int, opts: LqrOptions) -> int:
    out = ctypes.c_size_t(0)
    st = library().lqr_workspace_size(probs, int(batch), ctypes.byref(opts), ctypes.byref(out))
    if st != SUCCESS:
        raise LQRError(st, "lqr_workspace_size")
    return int(out.value)


def lqr_workspace_layout(probs, batch: int, opts: LqrOptions) -> dict:
    """Byte regions of the workspace (see the C header): the two plan regions,
    the scratch offset, the plans' sizes and the total workspace size."""
    out = (ctypes.c_size_t * 8)()
    st = library().lqr_workspace_layout(probs, int(batch), ctypes.byref(opts), out)
    if st != SUCCESS:
        raise LQRError(st, "lqr_workspace_layout")
    v = [int(x) for x in out]
    return dict(adj_off=v[0], adj_cap=v[1], fwd_off=v[2], fwd_cap=v[3], scratch_off=v[4],
                adj_plan=v[5], fwd_plan=v[6], total=v[7])


def lqr_plan_segments(probs, batch: int, opts: LqrOptions):
    """Per-instance segment counts the planner picks, and the predicted
    makespan (microseconds) of the persistent batched launch."""
    segs = (ctypes.c_int32 * int(batch))()
    est = ctypes.c_double(0.0)
    st = library().lqr_plan_segments(probs, int(batch), ctypes.byref(opts), segs, ctypes.byref(est))
    if st != SUCCESS:
        raise LQRError(st, "lqr_plan_segments")
    return list(segs), float(est.value)


def lqr_solve(prob: LqrProblem, opts: LqrOptions, ws: int, ws_bytes: int, stream: int) -> None:
    st = library().lqr_solve(ctypes.byref(prob), ctypes.byref(opts), ws, ws_bytes, stream)
    if st != SUCCESS:
        raise LQRError(st, "lqr_solve")


def lqr_solve_noalloc(prob: LqrProblem, opts: LqrOptions, stream: int) -> None:
    st = library().lqr_solve_noalloc(ctypes.byref(prob), ctypes.byref(opts), stream)
    if st != SUCCESS:
        raise LQRError(st, "lqr_solve_noalloc")


def lqr_solve_phase(prob: LqrProblem, opts: LqrOptions, phase: int, ws: int, ws_bytes: int,
                    stream: int) -> None:
    st = library().lqr_solve_phase(ctypes.byref(prob), ctypes.byref(opts), int(phase), ws, ws_bytes, stream)
    if st != SUCCESS:
        raise LQRError(st, "lqr_solve_phase")


def lqr_link_multipliers(prob: LqrProblem, opts: LqrOptions, segments: int, mu: int, stream: int) -> None:
    st = library().lqr_link_multipliers(ctypes.byref(prob), ctypes.byref(opts), int(segments), mu, stream)
    if st != SUCCESS:
        raise LQRError(st, "lqr_link_multipliers")


def lqr_solve_batched(probs, batch: int, opts: LqrOptions, ws: int, ws_bytes: int, stream: int) -> None:
    st = library().lqr_solve_batched(probs, int(batch), ctypes.byref(opts), ws, ws_bytes, stream)
    if st != SUCCESS:
        raise LQRError(st, "lqr_solve_batched")


def lqr_backward(probs, batch: int, grads, opts: LqrOptions, ws: int, ws_bytes: int, stream: int) -> None:
    st = library().lqr_backward(probs, int(batch), grads, ctypes.byref(opts), ws, ws_bytes, stream)
    if st != SUCCESS:
        raise LQRError(st, "lqr_backward")


# ---------------------------------------------------------------------------
# Tensor-level convenience wrappers (marshalling only).
# ---------------------------------------------------------------------------
_PREC = {"fp64": PREC_FP64, "mixed": PREC_MIXED, "fp32": PREC_FP32}
_ALGO = {"parallel": ALGO_PARALLEL, "serial": ALGO_SERIAL}
INPUTS = ("A", "B", "c", "Q", "q", "R", "r", "x0")


def options(precision: str = "fp64", algo: str = "parallel", phased: bool = False,
            smoothed: bool = False) -> LqrOptions:
    return LqrOptions(_PREC[precision], _ALGO[algo],
                      (FLAG_PHASED if phased else 0) | (FLAG_SMOOTHED if smoothed else 0))


def plan_segments(dims, segments=None, algo: str = "parallel"):
    """Planner's segment counts for instances of the given (n, m, T) and its
    predicted makespan in microseconds (host only, no device needed)."""
    arr = (LqrProblem * len(dims))()
    for i, (n, m, T) in enumerate(dims):
        arr[i] = LqrProblem(int(n), int(m), int(T), 0 if segments is None else int(segments[i]))
    return lqr_plan_segments(arr, len(dims), options("fp64", algo))


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_input(name, t, shape, dtype, device):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dtype, device))


def _outputs(n, m, T, dtype, device, with_P, with_lam, with_chol):
    import torch
    e = lambda *s: torch.empty(*s, dtype=dtype, device=device)  # noqa: E731
    out = dict(K=e(T, m, n), k=e(T, m), x=e(T + 1, n), u=e(T, m),
               info=torch.zeros(1, dtype=torch.int32, device=device))
    if with_P or with_lam:
        out["P"] = e(T + 1, n, n)
        out["p"] = e(T + 1, n)
    if with_lam:
        out["lam"] = e(T + 1, n)
    if with_chol:
        out["chol"] = e(T, m, m)
    return out


def _problem(data: dict, out: dict, segments: int) -> LqrProblem:
    T, n, m = data["B"].shape
    return LqrProblem(n, m, T, int(segments),
                      _ptr(data["A"]), _ptr(data["B"]), _ptr(data["c"]), _ptr(data["Q"]),
                      _ptr(data["q"]), _ptr(data["R"]), _ptr(data["r"]), _ptr(data.get("S")),
                      _ptr(data["x0"]), _ptr(out["K"]), _ptr(out["k"]), _ptr(out.get("P")),
                      _ptr(out.get("p")), _ptr(out["x"]), _ptr(out["u"]), _ptr(out.get("lam")),
                      _ptr(out.get("chol")), _ptr(out["info"]))


def _validate(data: dict, dtype, device):
    T, n, m = data["B"].shape
    shapes = dict(A=(T, n, n), B=(T, n, m), c=(T, n), Q=(T + 1, n, n), q=(T + 1, n),
                  R=(T, m, m), r=(T, m), x0=(n,), S=(T, m, n))
    for key in INPUTS + ("S",):
        if key == "S" and data.get("S") is None:
            continue
        _check_input(key, data[key], shapes[key], dtype, device)
    return int(n), int(m), int(T)


def _workspace(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def solve(data: dict, segments: int = 0, precision: str = "fp64", algo: str = "parallel",
          with_P: bool = True, with_lam: bool = True, with_chol: bool = False,
          workspace=None, stream=None, smoothed: bool = False) -> dict:
    """Solve one LQR instance given as a dict of device tensors (A, B, c, Q, q,
    R, r, x0 and optionally S; float64). Returns a dict of output tensors
    (K, k, P, p, x, u, lam, chol, info). Asynchronous on the current stream.
    ``smoothed``: the paper's smoothed policies instead of the serial-exact
    ones (LQR_FLAG_SMOOTHED)."""
    import torch
    dtype = torch.float32 if precision == "fp32" else torch.float64
    device = data["A"].device
    n, m, T = _validate(data, dtype, device)
    out = _outputs(n, m, T, dtype, device, with_P, with_lam, with_chol)
    prob = _problem(data, out, segments)
    opts = options(precision, algo, smoothed=smoothed)
    nbytes = lqr_workspace_size(ctypes.byref(prob), 1, opts)
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _workspace(nbytes, device)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    lqr_solve(prob, opts, ws.data_ptr(), ws.numel(), s)
    out["_workspace"] = ws
    return out


def link_multipliers(data: dict, out: dict, segments: int = 0, precision: str = "fp64",
                     algo: str = "parallel", stream=None):
    """The link multipliers mu_j (J - 1 rows of n) of an instance solved by
    ``solve`` with these arguments (its outputs P, p and x must be present).
    ``segments`` 0 means the planner's choice, as in ``solve``."""
    import torch
    T, n, m = data["B"].shape
    prob = _problem(data, out, segments)
    opts = options(precision, algo)
    J = int(segments) if segments else int(lqr_plan_segments(ctypes.byref(prob), 1, opts)[0][0])
    mu = torch.empty(max(J - 1, 0), n, dtype=out["x"].dtype, device=out["x"].device)
    s = (stream or torch.cuda.current_stream(out["x"].device)).cuda_stream
    lqr_link_multipliers(prob, opts, J, mu.data_ptr() if J > 1 else 0, s)
    return mu


def solve_batched(datas, segments=None, precision: str = "fp64", algo: str = "parallel",
                  with_P: bool = True, with_lam: bool = True, with_chol: bool = False,
                  workspace=None, stream=None, outputs=None, phased: bool = False):
    """Solve a list of instances (dicts of device tensors, possibly different
    n, m, T) with one batched call. ``segments``: None (planner) or a list of
    per-instance segment counts. ``phased``: three launches instead of the
    persistent one. Returns (list of output dicts, workspace)."""
    import torch
    dtype = torch.float32 if precision == "fp32" else torch.float64
    device = datas[0]["A"].device
    batch = len(datas)
    arr = (LqrProblem * batch)()
    outs = []
    for i, data in enumerate(datas):
        n, m, T = _validate(data, dtype, device)
        out = outputs[i] if outputs is not None else _outputs(n, m, T, dtype, device, with_P, with_lam, with_chol)
        outs.append(out)
        # the segment count is part of the workspace layout: backward() reuses it
        out["_segments"] = 0 if segments is None else int(segments[i])
        arr[i] = _problem(data, out, out["_segments"])
    opts = options(precision, algo, phased)
    nbytes = lqr_workspace_size(arr, batch, opts)
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _workspace(nbytes, device)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    lqr_solve_batched(arr, batch, opts, ws.data_ptr(), ws.numel(), s)
    return outs, ws


GRAD_KEYS = ("A", "B", "c", "Q", "q", "R", "r", "S", "x0")


def backward(datas, outs, dl_dx, dl_du, which=GRAD_KEYS, workspace=None, stream=None,
             precision: str = None, outputs=None):
    """Gradients of a loss l(x, u) with respect to the problem data of a batch
    already solved by ``solve_batched`` (``outs`` must hold K, P, x, u, lam,
    chol). ``dl_dx[i]``, ``dl_du[i]``: upstream gradients of instance i.
    Returns a list of dicts of gradient tensors (keys in ``which``); ``outputs``:
    such a list from an earlier call to write into (needed to replay the call in
    a captured graph, whose plan holds the output addresses)."""
    import torch
    batch = len(datas)
    probs = (LqrProblem * batch)()
    grads = (LqrGrad * batch)()
    res = []
    for i, (data, out) in enumerate(zip(datas, outs)):
        T, n, m = data["B"].shape
        for key in ("K", "P", "x", "u", "lam", "chol"):
            if out.get(key) is None:
                raise ValueError("backward needs the forward output %r (solve with with_lam=True, "
                                 "with_chol=True)" % key)
        probs[i] = _problem(data, out, out.get("_segments", 0))
        z = lambda *s: torch.empty(*s, dtype=data["A"].dtype, device=data["A"].device)  # noqa: E731
        shapes = dict(A=(T, n, n), B=(T, n, m), c=(T, n), Q=(T + 1, n, n), q=(T + 1, n),
                      R=(T, m, m), r=(T, m), S=(T, m, n), x0=(n,))
        g = outputs[i] if outputs is not None else {k: z(*shapes[k]) for k in which}
        res.append(g)
        gx, gu = dl_dx[i].contiguous(), dl_du[i].contiguous()
        g["_keep"] = (gx, gu)
        grads[i] = LqrGrad(gx.data_ptr(), gu.data_ptr(), *[_ptr(g.get(k)) for k in
                                                           ("A", "B", "c", "Q", "q", "R", "r", "S", "x0")])
    if precision is None:
        precision = "fp32" if datas[0]["A"].dtype == torch.float32 else "fp64"
    opts = options(precision, "parallel")
    nbytes = lqr_workspace_size(probs, batch, opts)
    device = datas[0]["A"].device
    ws = workspace if workspace is not None and workspace.numel() >= nbytes else _workspace(nbytes, device)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    lqr_backward(probs, batch, grads, opts, ws.data_ptr(), ws.numel(), s)
    for g in res:
        g["_workspace"] = ws
    return res


def _instances(A, B, c, Q, q, R, r, x0, S=None):
    """Per-instance views of batched tensors [N, ...] (contiguous)."""
    N = A.shape[0]
    out = []
    for i in range(N):
        d = dict(A=A[i], B=B[i], c=c[i], Q=Q[i], q=q[i], R=R[i], r=r[i], x0=x0[i])
        if S is not None:
            d["S"] = S[i]
        out.append(d)
    return out


def _lqr_function():
    import torch

    class LQRFunction(torch.autograd.Function):
        """Differentiable batched LQR: (A, B, c, Q, q, R, r, x0) -> (x, u).

        Inputs are float64 CUDA tensors with a leading batch dimension N
        (A [N,T,n,n], B [N,T,n,m], c [N,T,n], Q [N,T+1,n,n], q [N,T+1,n],
        R [N,T,m,m], r [N,T,m], x0 [N,n]); outputs x [N,T+1,n], u [N,T,m].
        Forward: one lqr_solve_batched call; backward: one lqr_backward call
        (adjoint re-solve on the KKT-transposed right-hand side). Backward
        raises LQRError if the forward solve reported a non-zero info word for
        any instance (an indefinite stage, a linking failure or a non-finite
        value): the gradients are not defined there."""

        @staticmethod
        def forward(ctx, A, B, c, Q, q, R, r, x0):
            ts = [t.contiguous() for t in (A, B, c, Q, q, R, r, x0)]
            N, T, n, m = ts[1].shape[0], ts[1].shape[1], ts[1].shape[2], ts[1].shape[3]
            dev, dt = ts[0].device, ts[0].dtype
            e = lambda *s: torch.empty(*s, dtype=dt, device=dev)  # noqa: E731
            big = dict(K=e(N, T, m, n), k=e(N, T, m), P=e(N, T + 1, n, n), p=e(N, T + 1, n),
                       x=e(N, T + 1, n), u=e(N, T, m), lam=e(N, T + 1, n), chol=e(N, T, m, m),
                       info=torch.zeros(N, 1, dtype=torch.int32, device=dev))
            datas = _instances(*ts)
            outs = [{k: v[i] for k, v in big.items()} for i in range(N)]
            solve_batched(datas, outputs=outs, precision="fp32" if dt == torch.float32 else "fp64")
            ctx.save_for_backward(*ts)
            ctx.big = big
            return big["x"], big["u"]

        @staticmethod
        def backward(ctx, gx, gu):
            ts = ctx.saved_tensors
            big = ctx.big
            N = ts[0].shape[0]
            bad = big["info"].ne(0).any(dim=1).nonzero().flatten().tolist()
            if bad:
                codes = big["info"][bad, 0].tolist()
                raise LQRError(ERR_NOT_PD if all(c > 0 for c in codes) else ERR_NONFINITE,
                               "LQRFunction.backward (forward solve info %s for instances %s)"
                               % (codes[:8], bad[:8]))
            if gx is None:
                gx = torch.zeros_like(big["x"])
            if gu is None:
                gu = torch.zeros_like(big["u"])
            gx, gu = gx.contiguous(), gu.contiguous()
            datas = _instances(*ts)
            outs = [{k: v[i] for k, v in big.items()} for i in range(N)]
            keys = ("A", "B", "c", "Q", "q", "R", "r", "x0")
            need = [k for k, flag in zip(keys, ctx.needs_input_grad) if flag]
            gs = backward(datas, outs, [gx[i] for i in range(N)], [gu[i] for i in range(N)],
                          which=tuple(need) or ("x0",))
            result = []
            for k, flag in zip(keys, ctx.needs_input_grad):
                result.append(torch.stack([g[k] for g in gs]) if flag else None)
            return tuple(result)

    return LQRFunction


def __getattr__(name):
    if name == "LQRFunction":
        fn = _lqr_function()
        globals()["LQRFunction"] = fn
        return fn
    raise AttributeError(name)
