"""The transport kernels' random numbers: the library's Philox4x32-10
(Salmon, Moraes, Dror & Shaw, SC'11, ten rounds, multipliers 0xD2511F53
and 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85) against the
known-answer vectors published with the authors' Random123 library,
computed on the host from the same header the kernels compile."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# counter (4 words), key (2 words) -> output (4 words)
KAT = [
    ("00000000 00000000 00000000 00000000 00000000 00000000",
     "6627e8d5 e169c58d bc57ac4c 9b00dbd8"),
    ("ffffffff ffffffff ffffffff ffffffff ffffffff ffffffff",
     "408f276d 41c83b0e a20bc7c6 6d5451fd"),
    ("243f6a88 85a308d3 13198a2e 03707344 a4093822 299f31d0",
     "d16cfe09 94fdcceb 5001e420 24126ea1"),
]


@pytest.fixture(scope="module")
def kat_exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("kat") / "philox_kat")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-x", "hip",
                        os.path.join(HERE, "philox_kat.cpp"), "-o", out],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    yield out
    shutil.rmtree(os.path.dirname(out), ignore_errors=True)


@pytest.mark.parametrize("inp,want", KAT)
def test_philox4x32_10_known_answers(kat_exe, inp, want):
    r = subprocess.run([kat_exe, *inp.split()], capture_output=True,
                       text=True)
    assert r.returncode == 0
    assert r.stdout.split() == want.split()
