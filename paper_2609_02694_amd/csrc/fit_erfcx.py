"""Fits of the scaled complementary error function used by the near-field kernels.

R(x) = erfc(x) exp(x^2) is smooth and bounded on [0, inf). The kernels
evaluate erfc(x) = exp(-x^2) R(x), sharing exp(-alpha r^2) with the second
term of G(r), and need x = sqrt(alpha) r <= 8.

FP32 form: degree 9 in t = 1 / (1 + x / 2), fitted over [0, 8] by iteratively
reweighted least squares on the relative error.
FP64 form: degree 20 in s = 2 t - 1, weighted least squares on the relative
error against a 40-digit reference (mpmath), over [0, 8].

Printed: the coefficients (lowest order first) and the maximum relative error
of a Horner evaluation in the target precision.

Run: python fit_erfcx.py
"""
import numpy as np
from scipy.special import erfcx

X_MAX = 8.0


def fit_f32(degree=9, scale=0.5):
    xs = np.linspace(0.0, X_MAX, 200001)
    t = 1.0 / (1.0 + scale * xs)
    R = erfcx(xs)
    V = np.vander(t, degree + 1, increasing=True)
    wt = np.ones_like(xs)
    for _ in range(30):
        c, *_ = np.linalg.lstsq(V * (wt / R)[:, None], wt, rcond=None)
        rel = (V @ c - R) / R
        wt = wt * (1.0 + np.abs(rel) / np.abs(rel).max())
    t32 = (np.float32(1.0) / (np.float32(1.0) + np.float32(scale) * xs.astype(np.float32))).astype(np.float32)
    acc = np.full_like(t32, np.float32(c[-1]))
    for k in range(degree - 1, -1, -1):
        acc = (acc * t32 + np.float32(c[k])).astype(np.float32)
    return c, float((np.abs(acc.astype(np.float64) - R) / R).max())


def fit_f64(degree=20, scale=0.5):
    import mpmath

    mpmath.mp.dps = 40
    xs = np.linspace(0.0, X_MAX, 8001)
    ref_mp = [mpmath.erfc(mpmath.mpf(x)) * mpmath.exp(mpmath.mpf(x) ** 2) for x in xs]
    ref = np.array([float(v) for v in ref_mp])
    s = 2.0 / (1.0 + scale * xs) - 1.0
    V = np.vander(s, degree + 1, increasing=True)
    c, *_ = np.linalg.lstsq(V / ref[:, None], np.ones_like(ref), rcond=None)
    acc = np.full_like(s, c[-1])
    for k in range(degree - 1, -1, -1):
        acc = acc * s + c[k]
    err = max(float(abs(mpmath.mpf(a) / r - 1)) for a, r in zip(acc, ref_mp))
    return c, err


if __name__ == "__main__":
    c32, e32 = fit_f32()
    print("FP32 coefficients (t = 1/(1 + x/2)):", ", ".join(f"{v:.9e}f" for v in c32))
    print(f"FP32 max relative error {e32:.2e}")
    c64, e64 = fit_f64()
    print("FP64 coefficients (s = 2/(1 + x/2) - 1):", ", ".join(f"{v:.17e}" for v in c64))
    print(f"FP64 max relative error {e64:.2e}")
