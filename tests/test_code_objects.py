"""Properties of the built gfx950 code objects (host only, no GPU).

The library's LDS budgets (the planner's 160 KiB per workgroup) count only
dynamic LDS, so no kernel may allocate static LDS: a kernel that did would
fail to launch at the largest planned footprints (a device-side helper such
as __syncthreads_or declares a static __shared__ word). The width-8
matrix-core variants, which faulted the GPU, must not be in the library.
Reads the kernel descriptors' metadata notes of the code objects that this
repository's build produced (offload bundles inside libmi355lqr.so).
"""

import os
import re
import struct
import subprocess

import pytest

import paper_1809_06360_amd as L

READELF = "/opt/rocm/llvm/bin/llvm-readelf"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def gfx950_objects(path):
    data = open(path, "rb").read()
    start = 0
    while True:
        i = data.find(MAGIC, start)
        if i < 0:
            return
        count = struct.unpack_from("<Q", data, i + len(MAGIC))[0]
        off = i + len(MAGIC) + 8
        for _ in range(count):
            o, size, idlen = struct.unpack_from("<QQQ", data, off)
            ident = data[off + 24:off + 24 + idlen]
            off += 24 + idlen
            if b"gfx950" in ident and size > 0:
                yield data[i + o:i + o + size]
        start = i + len(MAGIC)


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not os.path.exists(L.LIB_PATH) or not os.path.exists(READELF):
        pytest.skip("library or llvm-readelf missing")
    out = {}
    tmp = tmp_path_factory.mktemp("co")
    for k, blob in enumerate(gfx950_objects(L.LIB_PATH)):
        f = tmp / ("co%d.elf" % k)
        f.write_bytes(blob)
        notes = subprocess.run([READELF, "--notes", str(f)], capture_output=True, text=True,
                               check=True).stdout
        # one metadata map per kernel: group segment size precedes the name
        for m in re.finditer(r"\.group_segment_fixed_size:\s*(\d+)\s*\n(?:.*\n)*?\s*\.name:\s*(\S+)", notes):
            out[m.group(2)] = int(m.group(1))
    assert out, "no kernel metadata found"
    return out


def test_no_kernel_allocates_static_lds(kernels):
    static = {k: v for k, v in kernels.items() if v != 0}
    assert not static, static


def test_width8_matrix_core_variants_are_not_built(kernels):
    bad = [k for k in kernels if re.search(r"ILi8ELi[12]E", k)]
    assert not bad, bad
    assert any(re.search(r"k_phase1ILi8ELi0E", k) for k in kernels)
