"""Pins for the oracle's moments and p = 1 Lanczos energy.

* closed form vs the explicit generalised 2x2 eigenproblem in span{psi, H psi}
  built from sector vectors (no shared algebra);
* variational ordering E0 <= E_p1 <= <H> in exact mode;
* the exact eigenstate case (v = 0) is flagged degenerate;
* the reading of the printed alpha (the missing 1/2) is documented by showing
  that the printed form disagrees with the explicit eigenproblem.
"""
import math

import numpy as np
import pytest

import oracle as O


def _params(m, std, seed):
    rng = np.random.default_rng(seed)
    n = m.n_rbm * m.params_per_rbm
    return (rng.normal(0, std, n) + 1j * rng.normal(0, std, n)).reshape(m.n_rbm, -1)


@pytest.fixture(scope="module")
def exact_state():
    masks, spins = O.sector_basis(16)
    m = O.Model(L=4, J2=0.5, n_hidden=6)
    p = _params(m, 0.3, 2)
    lp = O.logpsi(m, p, spins)
    psi = np.exp(lp - lp.real.max())
    H = O.hamiltonian_sector(m, masks)
    return m, masks, psi, H


@pytest.mark.slow
def test_closed_form_equals_explicit_ritz_value(exact_state):
    m, masks, psi, H = exact_state
    e1 = (H @ psi) / psi
    e2 = (H @ (H @ psi)) / psi
    w = np.abs(psi) ** 2
    mo = O.moments(e1, e2, weights=w)
    ref = O.lanczos_p1_explicit(H, psi)
    assert abs(mo["e_p1"] - ref) < 1e-10 * abs(ref)
    e0 = O.ground_state(m)[0][0]
    assert e0 - 1e-10 <= mo["e_p1"] <= mo["h1"] + 1e-12
    # raw and centred estimators agree in exact mode
    assert abs(mo["h2"] - mo["h1"] ** 2 - mo["c2"]) < 1e-9 * mo["h2"]
    assert abs(mo["h2_alt"] - mo["h2"]) < 1e-9 * mo["h2"]
    h1, h2, h3 = mo["h1"], mo["h2"], mo["h3"]
    assert abs(mo["c3"] - (h3 - 3 * h1 * h2 + 2 * h1 ** 3)) < 1e-8 * abs(h3)


@pytest.mark.slow
def test_printed_alpha_needs_the_half(exact_state):
    m, masks, psi, H = exact_state
    e1 = (H @ psi) / psi
    e2 = (H @ (H @ psi)) / psi
    mo = O.moments(e1, e2, weights=np.abs(psi) ** 2)
    r = mo["r"]
    printed = mo["h1"] + mo["v"] * (r - math.sqrt(r * r + 1))
    ref = O.lanczos_p1_explicit(H, psi)
    assert abs(printed - ref) > 1e-3
    assert abs(mo["e_p1"] - ref) < 1e-10 * abs(ref)


def test_alpha_is_the_lowest_eigenvalue_of_the_unit_matrix():
    for r in (-5.0, -0.3, 0.0, 0.7, 40.0, 1e6):
        res = O.lanczos_p1(1.0, 4.0, r * 8.0)           # v = 2, c3 = r v^3
        lo = np.linalg.eigvalsh(np.array([[0.0, 1.0], [1.0, r]]))[0]
        assert abs(res["alpha"] - lo) < 1e-12 * max(1.0, abs(lo))
        assert abs(res["e_p1"] - (1.0 + 2.0 * lo)) < 1e-10


def test_eigenstate_is_degenerate():
    m = O.Model(L=4, J2=0.5, n_hidden=3)
    p = np.zeros((1, m.params_per_rbm), np.complex128)
    _, spins = O.sector_basis(16)
    e1 = O.eloc_direct(m, p, spins[:40])
    e2 = O.e2_direct(m, p, spins[:5])
    mo = O.moments(e1[:5], e2)
    assert mo["degenerate"] and mo["e_p1"] == mo["h1"] == 12.0 and mo["alpha"] == 0.0


def test_monte_carlo_mode_matches_plain_averages():
    rng = np.random.default_rng(0)
    e1 = rng.normal(-3, 0.5, 1000) + 1j * rng.normal(0, 0.1, 1000)
    e2 = rng.normal(10, 1, 1000) + 1j * rng.normal(0, 0.1, 1000)
    mo = O.moments(e1, e2)
    h1 = e1.real.mean()
    assert abs(mo["h1"] - h1) < 1e-13
    assert abs(mo["c2"] - np.mean(np.abs(e1 - h1) ** 2)) < 1e-12
    assert abs(mo["c3"] - np.mean(np.conj(e1 - h1) * (e2 - 2 * h1 * e1 + h1 ** 2)).real) < 1e-11
