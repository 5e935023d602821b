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


# ---------------------------------------------------------------- p = 2

def _krylov_moments(H, psi):
    e1 = (H @ psi) / psi
    h2v = H @ (H @ psi)
    e2 = h2v / psi
    e3 = (H @ h2v) / psi
    return e1, e2, e3


@pytest.mark.slow
def test_p2_moment_route_equals_explicit_krylov(exact_state):
    m, masks, psi, H = exact_state
    e1, e2, e3 = _krylov_moments(H, psi)
    w = np.abs(psi) ** 2
    mo = O.moments(e1, e2, weights=w, e3=e3)
    ref = O.lanczos_p2_explicit(H, psi)
    assert not mo["degenerate2"]
    assert abs(mo["e_p2"] - ref) < 1e-10 * abs(ref)
    e0 = O.ground_state(m)[0][0]
    assert e0 - 1e-10 <= mo["e_p2"] <= mo["e_p1"] + 1e-12
    assert mo["e_p1"] - mo["e_p2"] > 1e-6          # the third Krylov vector helps
    # centred moments against the binomial expansion of the raw ones
    h1, h2, h3, h4, h5 = mo["h1"], mo["h2"], mo["h3"], mo["h4"], mo["h5"]
    mu4 = h4 - 4 * h1 * h3 + 6 * h1 ** 2 * h2 - 3 * h1 ** 4
    mu5 = h5 - 5 * h1 * h4 + 10 * h1 ** 2 * h3 - 10 * h1 ** 3 * h2 + 4 * h1 ** 5
    assert abs(mo["mu4"] - mu4) < 1e-9 * h4
    assert abs(mo["mu5"] - mu5) < 1e-9 * abs(h5)
    # every split of <H^4> agrees in exact mode
    assert abs(h4 - (np.sum(w * np.conj(e1) * e3) / w.sum()).real) < 1e-9 * h4


@pytest.mark.slow
def test_p2_betas_build_the_ritz_vector(exact_state):
    m, masks, psi, H = exact_state
    e1, e2, e3 = _krylov_moments(H, psi)
    mo = O.moments(e1, e2, weights=np.abs(psi) ** 2, e3=e3)
    Hp = H @ psi
    phi = psi + mo["beta1"] * Hp + mo["beta2"] * (H @ Hp)
    rq = (np.vdot(phi, H @ phi) / np.vdot(phi, phi)).real
    assert abs(rq - mo["e_p2"]) < 1e-10 * abs(rq)


def test_e3_direct_matches_sector_vectors(exact_state):
    m, masks, psi, H = exact_state
    _, spins = O.sector_basis(16)
    p = _params(m, 0.3, 2)
    idx = np.array([0, 4321, 12869])
    got = O.e3_direct(m, p, spins[idx])
    h3 = H @ (H @ (H @ psi))
    want = h3[idx] / psi[idx]
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))


def test_p2_spectral_mixtures():
    """mu_k of a state spread over a few levels E_i with weights p_i: with three
    levels the 3-dimensional Krylov space is exact (E_p2 = min E_i); with two
    it collapses (degenerate, E_p2 = E_p1 = min E_i); with more, E_p2 is the
    explicit Ritz value of the diagonal matrix."""
    def mus(E, p):
        h = float(np.dot(p, E))
        return h, [float(np.dot(p, (E - h) ** k)) for k in (2, 3, 4, 5)]

    E3, p3 = np.array([-3.0, 0.5, 2.0]), np.array([0.6, 0.3, 0.1])
    h, mu = mus(E3, p3)
    res = O.lanczos_p2(h, *mu)
    assert not res["degenerate2"] and abs(res["e_p2"] + 3.0) < 1e-11
    E2, p2 = np.array([-1.0, 4.0]), np.array([0.7, 0.3])
    h, mu = mus(E2, p2)
    res = O.lanczos_p2(h, *mu)
    assert res["degenerate2"] and abs(res["e_p2"] + 1.0) < 1e-12
    rng = np.random.default_rng(5)
    E = np.sort(rng.normal(0, 2, 7))
    pr = rng.random(7)
    pr /= pr.sum()
    h, mu = mus(E, pr)
    res = O.lanczos_p2(h, *mu)
    ref = O.lanczos_p2_explicit(np.diag(E), np.sqrt(pr))
    assert abs(res["e_p2"] - ref) < 1e-11 * max(1.0, abs(ref))
    assert E[0] - 1e-12 <= res["e_p2"] <= O.lanczos_p1(h, mu[0], mu[1])["e_p1"] + 1e-12


def test_p2_monte_carlo_estimators():
    rng = np.random.default_rng(1)
    n = 500
    e1, e2, e3 = (rng.normal(c, s, n) + 1j * rng.normal(0, 0.1, n)
                  for c, s in ((-3, 0.5), (10, 1.0), (-30, 3.0)))
    mo = O.moments(e1, e2, e3=e3)
    h = e1.real.mean()
    d2 = e2 - 2 * h * e1 + h * h
    d3 = e3 - 3 * h * e2 + 3 * h * h * e1 - h ** 3
    assert abs(mo["mu4"] - np.mean(np.abs(d2) ** 2)) < 1e-10 * mo["mu4"]
    assert abs(mo["mu5"] - np.mean(np.conj(d2) * d3).real) < 1e-9 * max(1.0, abs(mo["mu5"]))
