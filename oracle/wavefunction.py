"""RBM amplitude and its symmetry projection, in complex128.

Test infrastructure (see the package docstring).

* RBM (Sec. 3.1, Eq. (2)): psi(sigma) = exp(sum_i a_i sigma_i)
  prod_h 2 cosh(sum_j W_hj sigma_j + b_h), with sigma_j = +-1/2 literally
  (reading: the factor 2 is kept, so log psi_s contains M log 2).
* Projection (Sec. 3.1, Eqs. (4)-(6)): psi(sigma) = sum_k sum_g chi(g)
  psi_s^(k)(g sigma), evaluated as a complex log-sum-exp shifted by the
  largest real part; the imaginary part of the result lies in (-pi, pi].
"""
from __future__ import annotations

import numpy as np


def log2cosh(z):
    """log(2 cosh z) for complex z, without overflow: with z' = +-z chosen so
    that Re z' >= 0 (cosh is even), log 2cosh z = z' + log(1 + exp(-2 z'))."""
    z = np.asarray(z, dtype=np.complex128)
    zp = np.where(z.real < 0, -z, z)
    return zp + np.log1p(np.exp(-2.0 * zp))


def logpsi_s(X, W, a, b):
    """log of Eq. (2) for configurations X [..., N] with entries +-1/2."""
    X = np.asarray(X, dtype=np.float64)
    theta = X @ W.T + b
    return X @ a + log2cosh(theta).sum(axis=-1)


def images(model, spins):
    """Symmetry images of each configuration: [S, G, N] of +-1/2 values,
    (g sigma)[i] = sigma[perm_g[i]]."""
    X = np.asarray(spins, dtype=np.float64) * 0.5
    return X[:, model.lat.perms]


def _lse(terms, weights):
    """log sum_j weights_j exp(terms_j) along the last axis (complex)."""
    m = terms.real.max(axis=-1, keepdims=True)
    s = (weights * np.exp(terms - m)).sum(axis=-1)
    with np.errstate(divide="ignore"):
        return m[..., 0] + np.log(s)


def logpsi(model, params, spins, chunk=None):
    """Projected log-amplitude log psi(sigma) for int +-1 spins [S, N]."""
    spins = np.atleast_2d(np.asarray(spins))
    if chunk is None:   # bound the [chunk, G, K*M] complex intermediates to ~0.3 GB
        chunk = max(1, int(2e7 // (model.G * model.n_hidden * model.n_rbm)))
    rbms = model.split(params)
    out = np.empty(spins.shape[0], dtype=np.complex128)
    for s0 in range(0, spins.shape[0], chunk):
        Xg = images(model, spins[s0:s0 + chunk])          # [s, G, N]
        terms = np.concatenate([logpsi_s(Xg, W, a, b) for (W, a, b) in rbms], axis=-1)
        w = np.tile(model.chi, len(rbms))                 # chi(g) for each (k, g)
        out[s0:s0 + chunk] = _lse(terms, w)
    return out


def image_weights(model, params, spins):
    """w[s, k, g] = chi(g) psi_s^(k)(g sigma) / psi(sigma) and tanh(theta)[s,k,g,h].

    These are the per-image factors of the log-derivatives (Sec. 3.2,
    O_k = d psi / d theta_k / psi applied to Eq. (6))."""
    spins = np.atleast_2d(np.asarray(spins))
    Xg = images(model, spins)
    lp = logpsi(model, params, spins)
    ws, ts = [], []
    for (W, a, b) in model.split(params):
        theta = Xg @ W.T + b
        ls = Xg @ a + log2cosh(theta).sum(axis=-1)        # [S, G]
        ws.append(model.chi[None, :] * np.exp(ls - lp[:, None]))
        ts.append(np.tanh(theta))
    return np.stack(ws, axis=1), np.stack(ts, axis=1), Xg
