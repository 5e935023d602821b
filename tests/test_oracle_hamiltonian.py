"""Pins for the oracle's Hamiltonian, local energies and H^2 terms.

* the sector matrix equals the Kronecker-product construction of Eq. (1)
  restricted to Sz = 0 (an independent assembly from spin matrices);
* the 4x4 J2 = 0 ground-state energy equals the literature value
  (tests/golden/ed_4x4_heisenberg.json);
* SU(2): [H, S^2] = 0, the ground state is a singlet;
* closed form: W = a = b = 0 gives the Sz = 0 member of the fully polarised
  multiplet, E_loc = N (J1 + J2)/2 on every configuration, zero variance;
* the direct local energies (Eq. (10)) and H^2 terms agree with the vector
  forms (H psi)/psi and (H^2 psi)/psi over the whole 4x4 sector.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from workloads import random_sz0_spins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _params(m, std, seed):
    rng = np.random.default_rng(seed)
    n = m.n_rbm * m.params_per_rbm
    return (rng.normal(0, std, n) + 1j * rng.normal(0, std, n)).reshape(m.n_rbm, -1)


@pytest.fixture(scope="module")
def sector():
    return O.sector_basis(16)


@pytest.mark.slow
@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_sector_matrix_equals_kronecker_construction(sector, J2):
    masks, _ = sector
    m = O.Model(L=4, J2=J2)
    Hs = O.hamiltonian_sector(m, masks)
    Hk = O.hamiltonian_kron(m)[masks][:, masks]
    assert abs(Hk.imag).max() < 1e-15
    diff = (Hs - Hk.real).tocoo()
    assert diff.nnz == 0 or np.abs(diff.data).max() < 1e-14


def test_ground_state_energy_matches_literature():
    ref = json.load(open(os.path.join(GOLDEN, "ed_4x4_heisenberg.json")))
    m = O.Model(L=ref["L"], J1=ref["J1"], J2=ref["J2"])
    e0 = O.ground_state(m)[0][0] / m.N
    assert abs(e0 - ref["e0_per_site"]) < 0.6 * 10.0 ** (-ref["digits_quoted"])


def test_spin_rotation_symmetry(sector):
    masks, _ = sector
    m = O.Model(L=4, J2=0.5)
    H = O.hamiltonian_sector(m, masks)
    S2 = O.total_spin_sq_sector(m, masks)
    comm = (H @ S2 - S2 @ H)
    assert comm.nnz == 0 or np.abs(comm.data).max() < 1e-12
    vals, vecs, _, _ = O.ground_state(m)
    assert abs(vecs[:, 0] @ (S2 @ vecs[:, 0])) < 1e-9
    uni = np.ones(len(masks)) / np.sqrt(len(masks))
    assert abs(uni @ (S2 @ uni) - 8 * 9) < 1e-9       # S = N/2 = 8


@pytest.mark.parametrize("L", [4, 6])
def test_zero_parameters_give_the_polarised_closed_form(L):
    m = O.Model(L=L, J2=0.5, n_hidden=3)
    p = np.zeros((1, m.params_per_rbm), np.complex128)
    spins = random_sz0_spins(L * L, 6, 1)
    e1 = O.eloc_direct(m, p, spins)
    assert np.allclose(e1, m.N * (m.J1 + m.J2) / 2, atol=1e-13)


@pytest.mark.slow
def test_direct_local_energy_equals_sparse_vector_form(sector):
    masks, spins = sector
    m = O.Model(L=4, J2=0.5, irrep="A1", n_hidden=6)
    p = _params(m, 0.3, 3)
    lp = O.logpsi(m, p, spins)
    psi = np.exp(lp - lp.real.max())
    H = O.hamiltonian_sector(m, masks)
    idx = np.random.default_rng(0).choice(len(masks), 60, replace=False)
    e1_vec = (H @ psi)[idx] / psi[idx]
    e1 = O.eloc_direct(m, p, spins[idx])
    assert np.allclose(e1, e1_vec, rtol=1e-10, atol=1e-10)
    e2_vec = (H @ (H @ psi))[idx[:8]] / psi[idx[:8]]
    assert np.allclose(O.e2_direct(m, p, spins[idx[:8]]), e2_vec, rtol=1e-10, atol=1e-10)


@pytest.mark.slow
def test_eloc_of_exact_ground_state_is_constant(sector):
    masks, spins = sector
    m = O.Model(L=4, J2=0.5)
    vals, vecs, _, _ = O.ground_state(m)
    v = vecs[:, 0]
    amp = {int(k): x for k, x in zip(masks, v)}
    idx = np.nonzero(np.abs(v) > 1e-6)[0][:50]

    def lp_fn(s):
        mk = ((np.asarray(s) > 0) * (1 << np.arange(16))).sum(axis=1)
        return np.log(np.array([amp[int(k)] for k in mk], dtype=np.complex128))

    e1 = O.eloc_direct(m, None, spins[idx], logpsi_fn=lp_fn)
    assert np.allclose(e1, vals[0], atol=1e-8)


@pytest.mark.slow
def test_exact_second_moment_two_ways(sector):
    masks, spins = sector
    m = O.Model(L=4, J2=0.5, n_hidden=4)
    p = _params(m, 0.2, 9)
    lp = O.logpsi(m, p, spins)
    psi = np.exp(lp - lp.real.max())
    H = O.hamiltonian_sector(m, masks)
    e1 = (H @ psi) / psi
    e2 = (H @ (H @ psi)) / psi
    w = np.abs(psi) ** 2
    w /= w.sum()
    assert abs((w * e2).sum() - (w * np.abs(e1) ** 2).sum()) < 1e-10
    assert abs(((w * e1).sum()).imag) < 1e-12
    # and the expectation equals the Rayleigh quotient
    rq = np.vdot(psi, H @ psi).real / np.vdot(psi, psi).real
    assert abs((w * e1).sum().real - rq) < 1e-10
