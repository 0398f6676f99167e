"""The FP32 arctangent polynomial of the sweep kernel (csrc/fastmath.h) on
the CPU: its coefficients are the ones csrc/fit_atan.py computes, and their
relative error against atan over [0, 1] is within the stated bound."""
import os
import re
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_03038_amd", "csrc")


def _header_coefficients():
    text = open(os.path.join(CSRC, "fastmath.h")).read()
    body = text[text.index("float atan2(float y, float x)"):]
    body = body[:body.index("float r = t * p;")]
    first = re.search(r"float p = ([-0-9.e+]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, s, ([-0-9.e+]+)f\);", body)
    return [float(first)] + [float(v) for v in rest]


def test_atan_coefficients_are_the_committed_fit():
    sys.path.insert(0, CSRC)
    try:
        import fit_atan
    finally:
        sys.path.remove(CSRC)
    got = _header_coefficients()
    want = fit_atan.coefficients_f32()
    assert len(got) == 9 and got[-1] == 1.0
    np.testing.assert_allclose(got, want, rtol=2e-8, atol=0)


def test_atan_polynomial_error_bound():
    cf = _header_coefficients()
    t = np.linspace(0.0, 1.0, 400001)[1:]
    s = t * t
    p = np.zeros_like(s)
    for a in cf:
        p = p * s + a
    rel = np.abs(t * p - np.arctan(t)) / np.arctan(t)
    assert rel.max() <= 2.0e-8, rel.max()
