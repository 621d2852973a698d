"""The device atan2's first-octant polynomial is what its fitting script produces.

fit_atan2_poly.py (next to the device code) fits p(s) ~ atan(sqrt(s))/sqrt(s) on
[0, 1] with p(0) = 1; the coefficients in atan2_heading must be the script's
output rounded to FP32 (up to a few FP32 units of the least-squares solver's
last bits), and the FP32 Horner form must stay within 1.5 units in the last
place of atan in FP64 over [0, 1].
"""
import os
import re
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_10392_amd", "csrc")


def header_coefficients():
    src = open(os.path.join(CSRC, "traj_device.h")).read()
    body = src[src.index("float atan2_heading("):]
    body = body[:body.index("float r = a * p;")]
    vals = [float(v) for v in re.findall(r"p = (?:fmaf\(p, s, )?([-+0-9.e]+)f", body)]
    return vals  # highest degree first, constant 1 last


def test_header_polynomial_is_the_fit():
    sys.path.insert(0, CSRC)
    try:
        import fit_atan2_poly as F
    finally:
        sys.path.remove(CSRC)
    hdr = header_coefficients()
    assert len(hdr) == F.DEGREE + 1 and hdr[-1] == 1.0
    fit = [float(np.float32(v)) for v in F.lawson()][::-1]
    for h, f in zip(hdr, fit):
        assert abs(h - f) <= 4 * np.spacing(np.float32(abs(f))), (h, f)
    assert F.ulp_error(hdr[::-1]) <= 1.5
