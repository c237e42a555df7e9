"""Fit of the scaled complementary error function used by the FP32 near-field kernel.

R(x) = erfc(x) exp(x^2) is smooth and bounded on [0, inf). With
t = 1 / (1 + x / 2) in (0, 1], R is fitted as a degree-9 polynomial in t
over x in [0, 8] by iteratively reweighted least squares on the relative
error. The kernel evaluates erfc(x) = exp(-x^2) R(x), sharing exp(-alpha r^2)
with the second term of G(r). Printed: the coefficients (lowest order first)
and the maximum relative error of an FP32 Horner evaluation.

Run: python fit_erfcx.py
"""
import numpy as np
from scipy.special import erfcx

P_SCALE = 0.5
DEGREE = 9


def fit():
    xs = np.linspace(0.0, 8.0, 200001)
    t = 1.0 / (1.0 + P_SCALE * xs)
    R = erfcx(xs)
    V = np.vander(t, DEGREE + 1, increasing=True)
    wt = np.ones_like(xs)
    for _ in range(30):
        c, *_ = np.linalg.lstsq(V * (wt / R)[:, None], wt, rcond=None)
        rel = (V @ c - R) / R
        wt = wt * (1.0 + np.abs(rel) / np.abs(rel).max())
    t32 = (np.float32(1.0) / (np.float32(1.0) + np.float32(P_SCALE) * xs.astype(np.float32))).astype(np.float32)
    acc = np.full_like(t32, np.float32(c[-1]))
    for k in range(DEGREE - 1, -1, -1):
        acc = (acc * t32 + np.float32(c[k])).astype(np.float32)
    err32 = np.abs(acc.astype(np.float64) - R) / R
    return c, np.abs(rel).max(), err32.max()


if __name__ == "__main__":
    c, e64, e32 = fit()
    print("coefficients:", ", ".join(f"{v:.9e}f" for v in c))
    print(f"max relative error: polynomial {e64:.2e}, FP32 evaluation {e32:.2e}")
