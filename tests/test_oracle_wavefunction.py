"""Pins for the oracle's RBM amplitude and symmetry projection.

* the literal product of Eq. (2) and a 50-digit mpmath brute force;
* the special cases of Sec. 3.1 (a = b = 0 gives spin-flip symmetry; W = 0
  reduces to M log 2 + a.sigma);
* the defining property of the projection, psi(g sigma) = chi(g) psi(sigma),
  and orthogonality of different irreps over the whole Sz = 0 sector.
"""
import cmath

import mpmath
import numpy as np
import pytest

import oracle as O
from workloads import random_sz0_spins


def _model(L=4, **kw):
    return O.Model(L=L, **kw)


def _params(m, std, seed, complex_=True):
    rng = np.random.default_rng(seed)
    n = m.n_rbm * m.params_per_rbm
    p = rng.normal(0, std, n) + (1j * rng.normal(0, std, n) if complex_ else 0)
    return p.reshape(m.n_rbm, -1)


def test_log2cosh_matches_definition_and_survives_large_arguments():
    z = np.array([0.3 + 0.2j, -1.7 + 2.9j, 5 - 1j, -0.01 + 1.5j])
    assert np.allclose(O.log2cosh(z), np.log(2 * np.cosh(z)), atol=1e-14)
    big = np.array([800 + 0.3j, -900 - 2.0j])
    ref = [complex(mpmath.log(2 * mpmath.cosh(mpmath.mpc(v.real, v.imag)))) for v in big]
    got = O.log2cosh(big)
    # compare modulo 2 pi i in the imaginary part
    for g, r in zip(got, ref):
        assert abs(g.real - r.real) < 1e-9
        assert abs(cmath.exp(1j * (g.imag - r.imag)) - 1) < 1e-9


def test_rbm_matches_literal_product():
    rng = np.random.default_rng(3)
    N, M = 6, 5
    W = rng.normal(0, 0.4, (M, N)) + 1j * rng.normal(0, 0.4, (M, N))
    a = rng.normal(0, 0.4, N) + 1j * rng.normal(0, 0.4, N)
    b = rng.normal(0, 0.4, M) + 1j * rng.normal(0, 0.4, M)
    X = rng.choice([-0.5, 0.5], size=(7, N))
    lit = np.exp(X @ a) * np.prod(2 * np.cosh(X @ W.T + b), axis=1)
    assert np.allclose(np.exp(O.logpsi_s(X, W, a, b)), lit, rtol=1e-13)


def test_projected_amplitude_against_mpmath_brute_force():
    m = _model(irrep="B1", kx=2, ky=2, n_hidden=6, n_rbm=2)
    p = _params(m, 0.3, 7)
    spins = random_sz0_spins(16, 3, 11)
    got = O.logpsi(m, p, spins)
    mpmath.mp.dps = 50
    for s, lp in zip(spins, got):
        total = mpmath.mpc(0)
        for (W, a, b) in m.split(p):
            for g in range(m.G):
                x = [mpmath.mpf(int(v)) / 2 for v in s[m.lat.perms[g]]]
                amp = mpmath.exp(sum(mpmath.mpc(a[j].real, a[j].imag) * x[j] for j in range(16)))
                for h in range(m.n_hidden):
                    th = mpmath.mpc(b[h].real, b[h].imag) + sum(
                        mpmath.mpc(W[h, j].real, W[h, j].imag) * x[j] for j in range(16))
                    amp *= 2 * mpmath.cosh(th)
                total += complex(m.chi[g]).real * amp
        ref = complex(mpmath.log(total))
        assert abs(lp.real - ref.real) < 1e-12
        assert abs(cmath.exp(1j * (lp.imag - ref.imag)) - 1) < 1e-12


def test_bias_free_rbm_is_spin_flip_symmetric():
    m = _model(use_bias=False, n_hidden=8)
    p = _params(m, 0.3, 5)
    (W, a, b), = m.split(p)
    X = random_sz0_spins(16, 10, 2) * 0.5
    assert np.allclose(O.logpsi_s(X, W, a, b), O.logpsi_s(-X, W, a, b), atol=1e-13)


def test_zero_weights_reduce_to_bias_term():
    m = _model(n_hidden=8)
    p = _params(m, 0.3, 5)
    p[0, : 8 * 16] = 0.0
    (W, a, b), = m.split(p)
    X = random_sz0_spins(16, 10, 2) * 0.5
    ref = X @ a + np.log(2 * np.cosh(b)).sum()
    assert np.allclose(O.logpsi_s(X, W, a, b), ref, atol=1e-13)


@pytest.mark.parametrize("irrep,K", [("A1", (0, 0)), ("B1", (0, 0)), ("A1", (2, 2)), ("B1", (2, 2))])
def test_projection_transforms_with_its_character_4x4(irrep, K):
    m = _model(irrep=irrep, kx=K[0], ky=K[1], n_hidden=8)
    p = _params(m, 0.3, 13)
    spins = random_sz0_spins(16, 20, 3)
    lp = O.logpsi(m, p, spins)
    keep = lp.real > lp.real.max() - 20                 # skip configurations with psi ~ 0
    rng = np.random.default_rng(4)
    for h in rng.integers(0, m.G, 12):
        lph = O.logpsi(m, p, spins[:, m.lat.perms[h]])
        ratio = np.exp(lph - lp)[keep]
        assert np.allclose(ratio, m.chi[h], atol=1e-10)


@pytest.mark.parametrize("L,M", [(6, 12), (8, 4), (10, 2)])
def test_projection_transforms_with_its_character_larger(L, M):
    m = _model(L=L, irrep="A1", n_hidden=M)
    p = _params(m, 0.2, 17)
    spins = random_sz0_spins(L * L, 3, 5)
    lp = O.logpsi(m, p, spins)
    for h in (1, 9, 8 * L + 6, m.G - 1):
        lph = O.logpsi(m, p, spins[:, m.lat.perms[h]])
        assert np.allclose(np.exp(lph - lp), m.chi[h], atol=1e-10)


@pytest.mark.slow
def test_different_irreps_are_orthogonal_over_the_sector():
    masks, spins = O.sector_basis(16)
    ma = _model(irrep="A1", n_hidden=4)
    mb = _model(irrep="B1", n_hidden=4)
    p = _params(ma, 0.3, 21)
    la, lb = O.logpsi(ma, p, spins), O.logpsi(mb, p, spins)
    shift = max(la.real.max(), lb.real.max())
    pa, pb = np.exp(la - shift), np.exp(lb - shift)
    overlap = np.vdot(pa, pb) / np.sqrt(np.vdot(pa, pa).real * np.vdot(pb, pb).real)
    assert abs(overlap) < 1e-12
