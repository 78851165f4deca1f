"""Generates the erfcx coefficients of the regularised kernel factors in
dps_internal.h (kErfcx*): a degree-7 polynomial in s = 1/(1 + t/2) fitted by
least squares, with relative weighting, to erfcx(t) = exp(t^2) erfc(t) on
4000 Chebyshev nodes of [1, 4.5] (the part of the regularised range the
series does not cover).  Prints the coefficients and the fit's maximum
relative error (about 1e-9 in FP64; evaluated in FP32 the rounding of s and
of the Horner steps dominates, about 3e-7)."""
import numpy as np
import scipy.special as sp

A, B, N, DEG = 1.0, 4.5, 4000, 7


def fit():
    k = np.arange(N)
    t = 0.5 * (A + B) + 0.5 * (B - A) * np.cos(np.pi * (k + 0.5) / N)
    s = 1.0 / (1.0 + 0.5 * t)
    y = sp.erfcx(t)
    V = np.vander(s, DEG + 1, increasing=True)
    w = 1.0 / y
    c, *_ = np.linalg.lstsq(V * w[:, None], y * w, rcond=None)
    return c


if __name__ == "__main__":
    c = fit()
    tt = np.linspace(A, B, 200001)
    rel = np.max(np.abs(np.polyval(c[::-1], 1.0 / (1.0 + 0.5 * tt)) / sp.erfcx(tt) - 1.0))
    for i, v in enumerate(c.astype(np.float32)):
        print(f"kErfcx{i} = {float(v)!r}f")
    print(f"max relative error of the fit on [{A}, {B}]: {rel:.2e}")
