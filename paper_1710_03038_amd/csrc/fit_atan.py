"""Fit of the FP32 arctangent polynomial of fastmath.h (CPU only).

For t in [0, 1], atan(t) = t * P(t^2) with P(s) = 1 + s * Q(s), Q of degree
7.  Q minimises the maximum relative error of t * P(t^2) against atan(t):
weighted least squares on Chebyshev nodes in s, reweighted by Lawson's
iteration (C. L. Lawson, 1961) towards the minimax solution.  Prints the
coefficients rounded to float32 (highest power first, as the Horner chain
in fastmath.h takes them) and the maximum relative error of the rounded
coefficients evaluated in float64 over a dense grid of t.

    python paper_1710_03038_amd/csrc/fit_atan.py
"""
import numpy as np

DEG = 7          # degree of Q: P has degree 8 in s = t^2
N_NODES = 2000
LAWSON_STEPS = 200


def fit():
    k = np.arange(N_NODES)
    s = 0.5 - 0.5 * np.cos(np.pi * (k + 0.5) / N_NODES)   # Chebyshev nodes on [0, 1]
    t = np.sqrt(s)
    f = np.where(t > 0, np.arctan(t) / np.where(t > 0, t, 1.0), 1.0)
    # relative error of P: (1 + s Q(s) - f) / f; unknowns: the coefficients of Q
    A = (s[:, None] ** (np.arange(DEG + 1)[None, :] + 1)) / f[:, None]
    b = (f - 1.0) / f
    w = np.full(N_NODES, 1.0 / N_NODES)
    c = None
    for _ in range(LAWSON_STEPS):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], b * sw, rcond=None)
        r = np.abs(A @ c - b)
        w = w * r
        w = w / w.sum()
    return c  # c[j] multiplies s^(j + 1)


def coefficients_f32():
    """Coefficients of the Horner chain, highest power first, then 1."""
    c = fit()
    return [float(np.float32(v)) for v in c[::-1]] + [1.0]


def max_rel_error(coefs, n=200001):
    t = np.linspace(1e-6, 1.0, n)
    s = t * t
    p = np.zeros_like(s)
    for a in coefs:
        p = p * s + a
    return float(np.max(np.abs(t * p - np.arctan(t)) / np.arctan(t)))


if __name__ == "__main__":
    cf = coefficients_f32()
    for v in cf:
        print("%.8e" % v)
    print("max relative error (float64 evaluation):", "%.2e" % max_rel_error(cf))
