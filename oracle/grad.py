"""Log-derivatives O_k = (d psi / d theta_k) / psi (Sec. 3.2, below Eq. (12)).

Test infrastructure (see the package docstring).

For psi = sum_k sum_g chi(g) psi_s^(k)(g sigma) with psi_s of Eq. (2), and
w_{kg} = chi(g) psi_s^(k)(g sigma) / psi(sigma), t = tanh(theta):
    d log psi / d W^(k)_{hj} = sum_g w_{kg} t_{kgh} (g sigma)_j
    d log psi / d b^(k)_h    = sum_g w_{kg} t_{kgh}
    d log psi / d a^(k)_j    = sum_g w_{kg} (g sigma)_j
These are holomorphic derivatives (log psi is analytic in the complex
parameters); the parameter layout per RBM is [W (M x N) | a (N) | b (M)].
"""
from __future__ import annotations

import numpy as np

from .wavefunction import image_weights, logpsi


def logderiv(model, params, spins):
    """Analytic O [S, K * P_rbm] (complex128)."""
    w, t, Xg = image_weights(model, params, spins)        # w [S,K,G], t [S,K,G,M], Xg [S,G,N]
    S = Xg.shape[0]
    out = []
    for k in range(model.n_rbm):
        wt = w[:, k, :, None] * t[:, k]                    # [S, G, M]
        OW = np.einsum("sgh,sgj->shj", wt, Xg).reshape(S, -1)
        parts = [OW]
        if model.use_bias:
            parts.append(np.einsum("sg,sgj->sj", w[:, k], Xg))
            parts.append(wt.sum(axis=1))
        out.append(np.concatenate(parts, axis=1))
    return np.concatenate(out, axis=1)


def logderiv_fd(model, params, spins, step=1e-5, indices=None):
    """Central finite differences of log psi along the real direction of each
    parameter (the holomorphic derivative), columns restricted to ``indices``."""
    p0 = np.asarray(params, np.complex128).reshape(-1)
    idx = np.arange(p0.size) if indices is None else np.asarray(indices)
    out = np.empty((np.atleast_2d(spins).shape[0], len(idx)), np.complex128)
    for c, k in enumerate(idx):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += step
        pm[k] -= step
        d = logpsi(model, pp.reshape(model.n_rbm, -1), spins) - logpsi(model, pm.reshape(model.n_rbm, -1), spins)
        d = d.real + 1j * np.angle(np.exp(1j * d.imag))  # unwrap the branch of Im log psi
        out[:, c] = d / (2 * step)
    return out
