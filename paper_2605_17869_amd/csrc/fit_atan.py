"""Coefficients of the arctangent polynomial used by the gradient-orientation
code of the kernels: atan(a) ~= a * (c0 + c1 s + ... + c7 s^7), s = a^2, on
a in [0, 1].  Weighted least squares on Chebyshev nodes, reweighted toward
equal ripple (Lawson's iteration); prints the coefficients as fp32 literals
and the maximum error of the fp32 Horner evaluation (about 1.4e-7 rad).

    python paper_2605_17869_amd/csrc/fit_atan.py
"""
import numpy as np

DEG = 7
N = 4000


def fit():
    k = np.arange(N)
    a = 0.5 + 0.5 * np.cos(np.pi * (k + 0.5) / N)
    s = a * a
    y = np.arctan(a)
    V = np.stack([a * s ** j for j in range(DEG + 1)], axis=1)
    w = np.ones(N)
    for _ in range(60):
        c, *_ = np.linalg.lstsq(V * w[:, None], y * w, rcond=None)
        e = V @ c - y
        w = w * (np.abs(e) + 1e-30) ** 0.5
        w /= w.max()
    return c.astype(np.float32)


def fp32_error(c):
    a = np.linspace(0, 1, 200001).astype(np.float32)
    s = a * a
    r = c[-1]
    for j in range(DEG - 1, -1, -1):
        r = (r * s + c[j]).astype(np.float32)
    r = (r * a).astype(np.float32)
    return float(np.abs(r.astype(np.float64) - np.arctan(a.astype(np.float64))).max())


if __name__ == "__main__":
    c = fit()
    print(", ".join(f"{float(x):.9g}f" for x in c))
    print(f"max abs error of the fp32 evaluation: {fp32_error(c):.3g}")
