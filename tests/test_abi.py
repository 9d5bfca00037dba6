"""The C-ABI library loads and exports every function include/psl.h
declares (no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psl.h")
LIB = os.path.join(ROOT, "paper_1302_1861_amd", "libpsl.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\([^;{]*\)\s*;", src,
                       flags=re.M)
    return sorted(set(n for n in names if not n.startswith("PSL_")))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for f in ("psl_build", "psl_sample", "transport_batch", "dose_tally"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsl.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.psl_version.restype = ctypes.c_int32
    assert lib.psl_version() == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsl.so not built")
def test_binding_lists_match_header():
    import paper_1302_1861_amd as P
    assert set(P.EXPORTS) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsl.so not built")
def test_struct_sizes_match_c():
    """ctypes mirrors of the header structs have the C sizes (compiled
    probe of the header with the host compiler)."""
    import subprocess
    import tempfile
    import paper_1302_1861_amd as P
    probe = r'''
#include <stdio.h>
#include "psl.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n",
    sizeof(psl_phsp), sizeof(psl_grid), sizeof(psl_field),
    sizeof(psl_sample_cfg), sizeof(psl_particles), sizeof(psl_queue),
    sizeof(psl_stats), sizeof(psl_phantom), sizeof(psl_physics),
    sizeof(psl_dose_acc), sizeof(psl_launch), sizeof(psl_tune_result),
    sizeof(psl_stream_cfg), sizeof(psl_flush), (size_t)PSL_QCOUNTS);
  return 0; }
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(probe)
        exe = os.path.join(d, "p")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c,
                               "-o", exe])
        got = list(map(int, subprocess.check_output([exe]).split()))
    want = [ctypes.sizeof(s) for s in (
        P.psl_phsp, P.psl_grid, P.psl_field, P.psl_sample_cfg,
        P.psl_particles, P.psl_queue, P.psl_stats, P.psl_phantom,
        P.psl_physics, P.psl_dose_acc, P.psl_launch, P.psl_tune_result,
        P.psl_stream_cfg, P.psl_flush)] + [P.PSL_QCOUNTS]
    assert got == want
