"""Pins of the oracle's spin structure factor S(q) (Sec. 4, the S(q)
equation; sigma^z = +-1/2), against closed forms, a sum rule, and the exact
4x4 ground state through SU(2) symmetry and the literature energy."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ed_4x4_heisenberg.json")


def _index(L, kx, ky):
    return kx + L * ky


def _pattern(L, kind):
    x, y = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
    if kind == "neel":
        s = np.where((x + y) % 2 == 0, 1, -1)
    else:                                   # stripes: spins alternate along x
        s = np.where(x % 2 == 0, 1, -1)
    return s.astype(np.int8).reshape(1, -1)


@pytest.mark.parametrize("L", [4, 6, 10])
def test_neel_and_stripe_closed_forms(L):
    """Neel order: S(pi, pi) = (N/2)^2 / N^2 = 1/4, nothing at (pi, 0) or
    (0, pi); stripes along x: S(pi, 0) = 1/4 only."""
    lat = oracle.Lattice(L)
    h = L // 2
    S = oracle.structure_factor(lat, _pattern(L, "neel"))
    assert S[_index(L, h, h)] == pytest.approx(0.25, abs=1e-14)
    assert abs(S[_index(L, h, 0)]) < 1e-14 and abs(S[_index(L, 0, h)]) < 1e-14
    assert abs(S.sum() - 0.25) < 1e-14
    S = oracle.structure_factor(lat, _pattern(L, "stripe"))
    assert S[_index(L, h, 0)] == pytest.approx(0.25, abs=1e-14)
    assert abs(S[_index(L, 0, h)]) < 1e-14 and abs(S[_index(L, h, h)]) < 1e-14


def test_sum_rule_and_uniform_component():
    """sum_q S(q) = (1/N) sum_i <sigma_i^2> = 1/4 for any ensemble, and S(0) =
    (Sz / N)^2 = 0 on the Sz = 0 sector; S(q) >= 0 and S(q) = S(-q)."""
    lat = oracle.Lattice(6)
    rng = np.random.default_rng(5)
    half = np.r_[np.ones(18, np.int8), -np.ones(18, np.int8)]
    sp = rng.permuted(np.tile(half, (40, 1)), axis=1)
    w = rng.random(40)
    S = oracle.structure_factor(lat, sp, w)
    assert abs(S.sum() - 0.25) < 1e-13
    assert abs(S[0]) < 1e-15
    assert S.min() > -1e-15
    L = 6
    for kx in range(L):
        for ky in range(L):
            assert S[_index(L, kx, ky)] == pytest.approx(S[_index(L, -kx % L, -ky % L)], abs=1e-14)


def _sq_energy(L, S, J1, J2):
    """3 sum_q S(q) J(q): the energy per site of an SU(2) singlet from its
    S^z correlations (<S_i.S_j> = 3 <S^z_i S^z_j>), with N J1 bonds along x
    and y each and N J2 bonds along each diagonal."""
    q = oracle.momenta(L)
    Jq = J1 * (np.cos(q[:, 0]) + np.cos(q[:, 1])) + \
        J2 * (np.cos(q[:, 0] + q[:, 1]) + np.cos(q[:, 0] - q[:, 1]))
    return 3.0 * float((S * Jq).sum())


def test_exact_ground_state_energy_from_sq_j2_zero():
    """For the 4x4 Heisenberg ground state (a singlet), the S(q) of the exact
    wave function gives back the literature energy per site."""
    g = json.load(open(GOLDEN))
    lat = oracle.Lattice(4)
    model = oracle.Model(L=4, J1=1.0, J2=0.0)
    vals, vecs, masks, spins = oracle.ground_state(model)
    S = oracle.structure_factor(lat, spins, np.abs(vecs[:, 0]) ** 2)
    assert _sq_energy(4, S, 1.0, 0.0) == pytest.approx(g["e0_per_site"], abs=1e-6)
    h = 2
    assert S[_index(4, h, 0)] == pytest.approx(S[_index(4, 0, h)], abs=1e-12)
    assert S[_index(4, h, h)] > 4 * S[_index(4, h, 0)]      # antiferromagnetic peak


def test_exact_ground_state_energy_from_sq_frustrated():
    """Same identity at J2 = 0.5 against the oracle's own diagonalisation (the
    energy comes from the sparse Hamiltonian, S(q) from the eigenvector)."""
    lat = oracle.Lattice(4)
    model = oracle.Model(L=4, J1=1.0, J2=0.5)
    vals, vecs, masks, spins = oracle.ground_state(model)
    S = oracle.structure_factor(lat, spins, np.abs(vecs[:, 0]) ** 2)
    assert _sq_energy(4, S, 1.0, 0.5) == pytest.approx(vals[0] / lat.N, abs=1e-10)
