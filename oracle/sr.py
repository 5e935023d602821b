"""Stochastic reconfiguration step (Sec. 3.2, Eq. (12); ridge of Sec. 3.4).

Test infrastructure (see the package docstring).

With averages over the S samples (<.> = 1/S sum),
    S_kk' = <O_k^* O_k'> - <O_k^*><O_k'>,  F_k = <O_k^* E_loc> - <O_k^*><E_loc>,
    (S + lambda I) dtheta = -dtau F.
Reading: lambda = 1e-6 is an absolute diagonal shift.  With the centred,
1/sqrt(S)-scaled O_bar = (O - <O>)/sqrt(S) and eps = (E_loc - <E_loc>)/sqrt(S),
S = O_bar^H O_bar and F = O_bar^H eps, so the same step is also
dtheta = -dtau O_bar^H (O_bar O_bar^H + lambda I)^{-1} eps (push-through identity),
an S x S system instead of a P x P one.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _centre(O, eloc):
    O = np.asarray(O, np.complex128)
    e = np.asarray(eloc, np.complex128)
    S = O.shape[0]
    Ob = (O - O.mean(axis=0)) / np.sqrt(S)
    eps = (e - e.mean()) / np.sqrt(S)
    return Ob, eps


def sr_param_space(O, eloc, lam, dtau):
    """Solve the P x P system of Eq. (12) directly (dense Cholesky)."""
    Ob, eps = _centre(O, eloc)
    Smat = Ob.conj().T @ Ob
    F = Ob.conj().T @ eps
    A = Smat + lam * np.eye(Smat.shape[0])
    return -dtau * sla.cho_solve(sla.cho_factor(A, lower=True), F)


def sr_sample_space(O, eloc, lam, dtau):
    """The same step through the S x S Gram matrix O_bar O_bar^H + lambda I."""
    Ob, eps = _centre(O, eloc)
    T = Ob @ Ob.conj().T + lam * np.eye(Ob.shape[0])
    x = sla.cho_solve(sla.cho_factor(T, lower=True), eps)
    return -dtau * (Ob.conj().T @ x)
