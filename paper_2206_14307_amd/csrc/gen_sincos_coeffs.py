"""Coefficients of the FP32 sine and cosine used by the theta epilogue.

After the argument is reduced by multiples of pi to r in [-pi/2, pi/2],
    sin r = r + r^3 P(r^2),  P of degree 3,
    cos r = 1 + r^2 Q(r^2),  Q of degree 4 (constant term -1/2 kept exact).
P and Q are near-minimax for the absolute error of sin and cos on that
interval: weighted least squares on Chebyshev points, with Lawson's weight
update (each iteration multiplies a point's weight by its current error),
which converges towards the equioscillating minimax solution.

Run: python gen_sincos_coeffs.py  -- prints the FP32 coefficients and the
approximation error of the rounded coefficients evaluated in FP64.
"""
import numpy as np


def fit(kind, n_coef, iters=60):
    r = np.cos(np.linspace(0.0, np.pi, 4001)) * (np.pi / 2)
    r = r[np.abs(r) > 1e-6]
    z = r * r
    if kind == "sin":
        target, scale = (np.sin(r) - r) / r**3, np.abs(r) ** 3
    else:
        target, scale = (np.cos(r) - 1.0) / z, z
    V = np.stack([z**d for d in range(n_coef)], axis=1)
    w = np.ones_like(r)
    for _ in range(iters):
        sw = np.sqrt(w) * scale
        c, *_ = np.linalg.lstsq(V * sw[:, None], target * sw, rcond=None)
        err = np.abs((V @ c - target) * scale)
        w = w * err
        w /= w.sum()
    if kind == "cos":
        c[0] = -0.5
    return np.float32(c)


def max_error(kind, c):
    r = np.linspace(-np.pi / 2, np.pi / 2, 2_000_001)
    z = r * r
    p = np.polyval(c[::-1].astype(np.float64), z)
    got = r + r**3 * p if kind == "sin" else 1.0 + z * p
    ref = np.sin(r) if kind == "sin" else np.cos(r)
    return float(np.abs(got - ref).max())


if __name__ == "__main__":
    for kind, n in (("sin", 4), ("cos", 5)):
        c = fit(kind, n)
        print(kind, ", ".join("%.9e" % float(v) for v in c), "max abs error %.2e" % max_error(kind, c))
