"""Moments <H^n> and the p = 1 Lanczos energy (Sec. 3.3, Eqs. (13)-(18)).

Test infrastructure (see the package docstring).

Readings of the passage:
* The printed r = (<H^3> - 3<H^2><H> + 2<H>^3)/(<H^2>-<H>^2)^{3/2} is kept,
  but the printed alpha = r - sqrt(r^2 + 1) lacks a factor 1/2: the 2x2
  matrix of H in the basis (psi0, psi1) of Eq. (13) is <H> I + v [[0,1],[1,r]],
  whose lowest eigenvalue gives alpha = r/2 - sqrt(r^2/4 + 1).  For r > 0 the
  equivalent alpha = -1/(r/2 + sqrt(r^2/4 + 1)) avoids cancellation.
* Estimators: <H> = Re<e1>, <H^2> = <|e1|^2>, <H^3> = Re<conj(e1) e2>, with
  e1 = E_loc and e2 = (H^2 psi)/psi; the centred moments
  c2 = <|e1 - h1|^2> and c3 = Re<conj(e1 - h1)(e2 - 2 h1 e1 + h1^2)> are the
  ones that enter v and r (raw <H^2> - <H>^2 loses digits near eigenstates).
* v = 0 (an exact eigenstate): E_p1 = <H>, alpha = 0, flagged degenerate.
  "Zero" means c2 <= (8 eps max(|h1|, 1))^2 with eps the FP64 unit roundoff
  2^-53: below that the centred variance is rounding noise of h1 itself.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.linalg as sla


def _fsum_c(x, w):
    """Exactly rounded weighted mean sum(w x) / sum(w)."""
    x = np.asarray(x) * w
    sw = math.fsum(w)
    return complex(math.fsum(np.real(x)) / sw, math.fsum(np.imag(x)) / sw)


def _fsum_r(x, w):
    return math.fsum(np.asarray(x) * w) / math.fsum(w)


def moments(e1, e2=None, weights=None):
    """Two-pass FP64 moments with exactly rounded sums (math.fsum).

    weights: None for Monte-Carlo mode (uniform 1/S), else the exact Born
    weights p_sigma = |psi|^2 / sum |psi|^2 (Sec. 3.2, Eq. (9))."""
    e1 = np.asarray(e1, np.complex128)
    n = len(e1)
    w = np.ones(n) if weights is None else np.asarray(weights, np.float64)
    out = {"n": n}
    m1 = _fsum_c(e1, w)
    h1 = m1.real
    out["h1"], out["h1_im"] = h1, m1.imag
    d1 = e1 - h1
    out["h2"] = _fsum_r(np.abs(e1) ** 2, w)
    out["c2"] = _fsum_r(np.abs(d1) ** 2, w)
    if e2 is not None:
        e2 = np.asarray(e2, np.complex128)
        out["h2_alt"] = _fsum_c(e2, w).real
        out["h3"] = _fsum_c(np.conj(e1) * e2, w).real
        d2 = e2 - 2.0 * h1 * e1 + h1 * h1
        out["c3"] = _fsum_c(np.conj(d1) * d2, w).real
        out.update(lanczos_p1(h1, out["c2"], out["c3"]))
    return out


def lanczos_p1(h1, c2, c3):
    """Closed form of the lowest eigenpair of the 2x2 Lanczos matrix
    (Sec. 3.3, Eqs. (14), (16)-(18), with the reading stated above)."""
    if not (c2 > (8.0 * 2.0 ** -53 * max(abs(h1), 1.0)) ** 2):
        return {"v": 0.0, "r": 0.0, "alpha": 0.0, "e_p1": h1, "degenerate": True}
    v = math.sqrt(c2)
    r = c3 / (v ** 3)
    root = math.sqrt(0.25 * r * r + 1.0)
    alpha = 0.5 * r - root if r <= 0 else -1.0 / (0.5 * r + root)
    return {"v": v, "r": r, "alpha": alpha, "e_p1": h1 + v * alpha, "degenerate": False}


def lanczos_p1_explicit(H, psi):
    """Lowest Ritz value of H in span{psi, H psi} from explicit vectors: the
    generalised 2x2 problem A x = E B x with A_ij = <u_i|H|u_j>, B_ij = <u_i|u_j>,
    u = (psi, H psi).  Pins the closed form without sharing its algebra."""
    u = np.stack([psi, H @ psi], axis=1)
    Hu = np.stack([H @ u[:, 0], H @ u[:, 1]], axis=1)
    A = u.conj().T @ Hu
    B = u.conj().T @ u
    A = 0.5 * (A + A.conj().T)
    B = 0.5 * (B + B.conj().T)
    return float(sla.eigh(A, B, eigvals_only=True)[0])
