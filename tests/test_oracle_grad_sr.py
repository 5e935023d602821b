"""Pins for the oracle's log-derivatives and SR step.

* analytic O_k vs central finite differences of log psi (FP64);
* Cauchy-Riemann: the derivative along Im(theta_k) is i times the one along
  Re(theta_k) (log psi is holomorphic in the parameters);
* the push-through identity: the P x P solve of Eq. (12) and the S x S
  sample-space solve agree, with S < P and S > P;
* a small SR step lowers the exact variational energy (imaginary-time
  descent, Sec. 3.2).
"""
import numpy as np
import pytest

import oracle as O
from workloads import random_sz0_spins


def _params(m, std, seed, complex_=True):
    rng = np.random.default_rng(seed)
    n = m.n_rbm * m.params_per_rbm
    p = rng.normal(0, std, n) + (1j * rng.normal(0, std, n) if complex_ else 0)
    return p.reshape(m.n_rbm, -1)


@pytest.mark.parametrize("n_rbm,irrep", [(1, "A1"), (2, "B1")])
def test_logderiv_matches_finite_differences(n_rbm, irrep):
    m = O.Model(L=4, n_rbm=n_rbm, n_hidden=4, irrep=irrep)
    p = _params(m, 0.3, 1)
    spins = random_sz0_spins(16, 8, 2)
    # drop configurations where psi vanishes by symmetry (B1: sigma fixed by a
    # mirror with character -1); there psi is rounding noise and O undefined
    w, _, _ = O.wavefunction.image_weights(m, p, spins)
    spins = spins[np.abs(w).sum(axis=(1, 2)) < 1e4][:3]
    assert len(spins) == 3
    Oa = O.logderiv(m, p, spins)
    idx = np.random.default_rng(3).choice(Oa.shape[1], 40, replace=False)
    Ofd = O.logderiv_fd(m, p, spins, step=1e-5, indices=idx)
    assert np.allclose(Oa[:, idx], Ofd, rtol=1e-7, atol=1e-8)


def test_logderiv_is_holomorphic():
    m = O.Model(L=4, n_hidden=3)
    p = _params(m, 0.3, 4)
    spins = random_sz0_spins(16, 2, 5)
    idx = np.arange(0, m.params_per_rbm, 7)
    fd_re = O.logderiv_fd(m, p, spins, indices=idx)
    # derivative along the imaginary direction
    p0 = p.reshape(-1)
    out = np.empty_like(fd_re)
    for c, k in enumerate(idx):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += 1e-5j
        pm[k] -= 1e-5j
        d = O.logpsi(m, pp.reshape(1, -1), spins) - O.logpsi(m, pm.reshape(1, -1), spins)
        out[:, c] = (d.real + 1j * np.angle(np.exp(1j * d.imag))) / 2e-5
    assert np.allclose(out, 1j * fd_re, rtol=1e-7, atol=1e-8)


def test_real_parameters_give_real_derivatives():
    m = O.Model(L=4, n_hidden=4)
    p = _params(m, 0.3, 6, complex_=False)
    Oa = O.logderiv(m, p, random_sz0_spins(16, 4, 7))
    assert np.abs(Oa.imag).max() < 1e-13


@pytest.mark.parametrize("S", [64, 512])
def test_sr_push_through_identity(S):
    m = O.Model(L=4, n_hidden=16)
    p = _params(m, 0.05, 8)
    spins = random_sz0_spins(16, S, 9)
    Od = O.logderiv(m, p, spins)
    el = O.eloc_direct(m, p, spins)
    d1 = O.sr_param_space(Od, el, 1e-6, 0.01)
    d2 = O.sr_sample_space(Od, el, 1e-6, 0.01)
    assert np.linalg.norm(d1 - d2) < 1e-8 * np.linalg.norm(d1)


@pytest.mark.slow
def test_sr_step_lowers_the_exact_energy():
    masks, spins = O.sector_basis(16)
    m = O.Model(L=4, J2=0.5, n_hidden=4)
    p = _params(m, 0.1, 10)
    H = O.hamiltonian_sector(m, masks)

    def energy(q):
        lp = O.logpsi(m, q, spins)
        psi = np.exp(lp - lp.real.max())
        return (np.vdot(psi, H @ psi) / np.vdot(psi, psi)).real, psi

    e0, psi = energy(p)
    prob = np.abs(psi) ** 2
    prob /= prob.sum()
    draw = np.random.default_rng(11).choice(len(masks), 3000, p=prob)
    Od = O.logderiv(m, p, spins[draw])
    el = O.eloc_direct(m, p, spins[draw])
    d = O.sr_sample_space(Od, el, 1e-3, 0.02)
    e1, _ = energy(p + d.reshape(p.shape))
    assert e1 < e0
