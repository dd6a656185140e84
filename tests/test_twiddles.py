"""The register FFTs' compile-time twiddles (csrc/fft_twiddles.h) are what
their generator writes, and each is cos or sin of 2 pi k / 128 to within half
an ulp of the long-double value (exact where the value is 0 or +-1)."""
import math
import os
import subprocess
import sys

import numpy as np

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2609_07172_amd", "csrc")


def _table(src, name):
    body = src[src.index(name):]
    body = body[body.index("{") + 1:body.index("}")]
    return [float.fromhex(v.strip()) for v in body.split(",") if v.strip()]


def test_header_is_the_generator_output():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_twiddles.py")], capture_output=True,
                         text=True, check=True).stdout
    with open(os.path.join(CSRC, "fft_twiddles.h")) as fh:
        assert fh.read() == out


def test_twiddles_are_rounded_cos_and_sin():
    with open(os.path.join(CSRC, "fft_twiddles.h")) as fh:
        src = fh.read()
    c, s = _table(src, "kFftCos"), _table(src, "kFftSin")
    assert len(c) == len(s) == 128
    pi = np.longdouble("3.14159265358979323846264338327950288")
    for k in range(128):
        a = 2 * pi * np.longdouble(k) / np.longdouble(128)
        for got, ref in ((c[k], np.cos(a)), (s[k], np.sin(a))):
            # within half an ulp of the double nearest the long-double value
            # (plus the long double's own rounding)
            ulp = math.ulp(float(ref)) if abs(float(ref)) > 1e-15 else 0.0
            assert abs(np.longdouble(got) - ref) <= 0.5 * ulp + 1e-18, (k, got, ref)
    for k in (0, 32, 64, 96):
        assert (c[k], s[k]) == ((1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0))[k // 32]
    # the symmetries the kernels use: a quarter turn swaps cos and sin
    for k in range(96):
        assert c[k + 32] == -s[k] and s[k + 32] == c[k]
