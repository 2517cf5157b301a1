"""Accuracy of the tracker's own FP64 sin/cos/exp routines (host build of
csrc/mbt_fastmath.h) against long-double libm.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1809_00391_amd", "csrc")

LIMITS = {  # name prefix: (max abs error, max rel error)
    "sincos_cw": (2.5e-16, 4e-16),
    "sincos_2pi": (3e-16, None),
    "exp_small": (None, 2.5e-16),
    "multiple_angle": (1.5e-15, None),
    "log_unit": (None, 4e-16),
}


def test_fastmath_accuracy(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "fastmath_check")
    subprocess.run([hipcc, "-O2", "-ffp-contract=off", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "fastmath_check.cpp")], check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    rows = [l.split() for l in out if l.strip()]
    assert len(rows) == 17
    for name, ea, er in rows:
        key = next(k for k in LIMITS if name.startswith(k))
        lim_a, lim_r = LIMITS[key]
        if lim_a is not None:
            assert float(ea) <= lim_a, (name, ea)
        if lim_r is not None:
            assert float(er) <= lim_r, (name, er)
