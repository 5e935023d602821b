"""Spin structure factor S(q) (Sec. 4, the equation defining S(q) in the
discussion of the 6x6 and 10x10 results; the tables display N S(q)).

Test infrastructure (see the package docstring).

    S(q) = (1/N^2) sum_{i,j} <sigma^z_i sigma^z_j> exp(i q.(r_i - r_j))

with sigma^z = +-1/2 (reading 1 of the readings: spins are +-1/2 literally)
and q = 2 pi (kx, ky) / L for the L x L torus.  The expectation is the
weighted mean over the given configurations: uniform for Monte-Carlo samples,
|psi|^2 (normalised) for an exact sum over the Sz = 0 sector.  The
correlation matrix <sigma_i sigma_j> is formed first and then transformed, as
the equation is written.
"""
from __future__ import annotations

import numpy as np


def momenta(L):
    """All lattice momenta q = 2 pi (kx, ky) / L, index kx + L ky: [N][2]."""
    k = np.array([(i % L, i // L) for i in range(L * L)], dtype=np.float64)
    return 2.0 * np.pi * k / L


def correlations(spins, weights=None):
    """<sigma^z_i sigma^z_j> over configurations: [N][N] (sigma = +-1/2)."""
    s = 0.5 * np.asarray(spins, dtype=np.float64)
    w = np.ones(len(s)) if weights is None else np.asarray(weights, dtype=np.float64)
    w = w / w.sum()
    return (s * w[:, None]).T @ s


def structure_factor(lat, spins, weights=None):
    """S(q) for every momentum of the lattice (index kx + L ky), real [N]."""
    C = correlations(spins, weights)
    q = momenta(lat.L)
    r = lat.coords.astype(np.float64)
    phase = np.exp(1j * (q @ r.T))                     # [q][i] = e^{i q.r_i}
    S = np.einsum("qi,ij,qj->q", phase, C, phase.conj()) / lat.N ** 2
    assert np.abs(S.imag).max() <= 1e-12 * max(1.0, np.abs(S.real).max())
    return S.real
