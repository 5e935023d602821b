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

p = 2 (Sec. 3.3, Eq. (19) with p = 2), readings:
* The coefficients beta_1, beta_2 of Psi_2 = (1 + beta_1 H + beta_2 H^2) psi are
  those of the lowest eigenvector of H restricted to the Krylov space
  span{psi, H psi, H^2 psi} (the p = 1 step is the same construction on
  span{psi, H psi}); E_p2 is its lowest Ritz value.
* In the basis u_i = ((H - h1)/v)^i psi the Gram and Hamiltonian matrices are
  Hankel in the centred moments mu_k = <(H - h1)^k>: B_ij = mu_{i+j}/v^{i+j},
  A_ij = mu_{i+j+1}/v^{i+j}, E_p2 = h1 + v lambda_min(A, B).  Each mu_k is
  estimated with the balanced split mu_k = Re<conj(d_{floor(k/2)}) d_{ceil(k/2)}>
  of the local values d_1 = e1 - h1, d_2 = e2 - 2 h1 e1 + h1^2,
  d_3 = e3 - 3 h1 e2 + 3 h1^2 e1 - h1^3 (so mu_2 = c2, mu_3 = c3 as for p = 1,
  mu_4 = <|d_2|^2>, mu_5 = Re<conj(d_2) d_3>); with exact weights every split
  gives the exact moment.
* The scaled Gram determinant is delta = mu_4/v^4 - r^2 - 1.  delta <=
  64 eps max(mu_4/v^4, 1) means the Krylov space has dimension 2 (psi spans
  two eigenvalues) or the Monte-Carlo Hankel matrix is not positive definite:
  E_p2 = E_p1, beta_2 = 0, flagged degenerate.
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


def moments(e1, e2=None, weights=None, e3=None):
    """Two-pass FP64 moments with exactly rounded sums (math.fsum).

    weights: None for Monte-Carlo mode (uniform 1/S), else the exact Born
    weights p_sigma = |psi|^2 / sum |psi|^2 (Sec. 3.2, Eq. (9)).
    e3 (with e2): adds h4, h5, mu4, mu5 and the p = 2 energy."""
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
        if e3 is not None:
            e3 = np.asarray(e3, np.complex128)
            d3 = e3 - 3.0 * h1 * e2 + 3.0 * h1 * h1 * e1 - h1 ** 3
            out["h4"] = _fsum_r(np.abs(e2) ** 2, w)
            out["h5"] = _fsum_c(np.conj(e2) * e3, w).real
            out["mu4"] = _fsum_r(np.abs(d2) ** 2, w)
            out["mu5"] = _fsum_c(np.conj(d2) * d3, w).real
            out.update(lanczos_p2(h1, out["c2"], out["c3"], out["mu4"], out["mu5"]))
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


def lanczos_p2(h1, mu2, mu3, mu4, mu5):
    """Lowest Ritz value of H in span{psi, H psi, H^2 psi} from the centred
    moments (Sec. 3.3, Eq. (19) with p = 2; readings above): the generalised
    3x3 Hankel eigenproblem solved with scipy's eigh, and the coefficients
    beta_1, beta_2 of Psi_2 = (1 + beta_1 H + beta_2 H^2) psi."""
    p1 = lanczos_p1(h1, mu2, mu3)
    out = {"e_p2": p1["e_p1"], "beta1": 0.0, "beta2": 0.0, "degenerate2": True}
    if p1["degenerate"]:
        return out
    v, alpha = p1["v"], p1["alpha"]
    # p = 1 fallback: Psi_1 = psi + alpha (H - h1) psi / v
    c0, c1 = 1.0 - alpha * h1 / v, alpha / v
    out["beta1"] = c1 / c0
    m = [1.0, 0.0, 1.0, mu3 / v ** 3, mu4 / v ** 4, mu5 / v ** 5]
    delta = m[4] - m[3] ** 2 - 1.0
    if not delta > 64.0 * 2.0 ** -53 * max(m[4], 1.0):
        return out
    B = np.array([[m[i + j] for j in range(3)] for i in range(3)])
    A = np.array([[m[i + j + 1] for j in range(3)] for i in range(3)])
    lam, X = sla.eigh(A, B)
    x = X[:, 0]
    # x0 + x1 K + x2 K^2 with K = (H - h1)/v, expanded in powers of H
    c0 = x[0] - x[1] * h1 / v + x[2] * h1 * h1 / (v * v)
    c1 = x[1] / v - 2.0 * x[2] * h1 / (v * v)
    c2 = x[2] / (v * v)
    return {"e_p2": h1 + v * float(lam[0]), "beta1": c1 / c0, "beta2": c2 / c0,
            "degenerate2": False}


def lanczos_p2_explicit(H, psi):
    """Lowest Ritz value of H in span{psi, H psi, H^2 psi} from explicit sector
    vectors, orthonormalised by QR (pins the moment route of lanczos_p2)."""
    u = np.stack([psi, H @ psi, H @ (H @ psi)], axis=1)
    Q, _ = np.linalg.qr(u)
    Hq = np.stack([H @ Q[:, k] for k in range(3)], axis=1)
    A = Q.conj().T @ Hq
    A = 0.5 * (A + A.conj().T)
    return float(np.linalg.eigvalsh(A)[0])
