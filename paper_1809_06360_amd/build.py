"""Build the HIP library ``libmi355lqr.so`` for gfx950 (in-tree, no JIT cache).

Run as ``python -m paper_1809_06360_amd.build`` or through
``__graft_entry__.build()``. Always recompiles.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmi355lqr.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep hipcc from emitting packed-FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def sources():
    """Every translation unit, the slowest to compile first (the sweep and
    persistent kernel variants), so that a parallel build ends sooner."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    heavy = ("k_sweep_phase1", "k_persistent_w", "k_sweep_phase3", "k_sweep_serial")

    def rank(path):
        name = os.path.basename(path)
        for i, h in enumerate(heavy):
            if name.startswith(h):
                return i
        return len(heavy)
    return sorted(srcs, key=lambda p: (rank(p), p))


def _compile(src, obj, verbose):
    cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-I", INCLUDE, "-I", CSRC, "-MMD",
                                                             "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def _stale(src, obj):
    """Whether obj must be rebuilt: missing, or older than its source or any
    header listed in the dependency file the compiler wrote next to it."""
    dep = os.path.splitext(obj)[0] + ".d"
    if not os.path.exists(obj) or not os.path.exists(dep):
        return True
    t = os.path.getmtime(obj)
    text = open(dep).read().replace("\\\n", " ")
    paths = text.split(":", 1)[1].split() if ":" in text else [src]
    return any(not os.path.exists(p) or os.path.getmtime(p) > t for p in paths)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source to an object in parallel, then link the library.
    With ``incremental`` the objects are kept in ``_build/`` next to the package
    and only those whose source or headers changed are recompiled."""
    import concurrent.futures
    import tempfile
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with tempfile.TemporaryDirectory(prefix="lqr_build_") as tmpdir:
        odir = os.path.join(ROOT, "_build") if incremental else tmpdir
        os.makedirs(odir, exist_ok=True)
        objs = [os.path.join(odir, os.path.basename(s_) + ".o") for s_ in srcs]
        todo = [(s_, o) for s_, o in zip(srcs, objs) if not incremental or _stale(s_, o)]
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(lambda so: _compile(so[0], so[1], verbose), todo))
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(LIB)
