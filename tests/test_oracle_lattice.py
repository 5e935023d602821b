"""Pins for the oracle's lattice, bonds, space group and characters.

These check the tables against facts fixed by geometry and group theory
(bond counts and lengths, closure, faithfulness, class structure computed by
brute force, character orthogonality, the homomorphism property), not
against the oracle's own formulas.
"""
import itertools

import numpy as np
import pytest

from oracle.lattice import Lattice, POINT_OPS, POINT_CLASS, C4V_CHARACTERS, CLASS_SIZES


@pytest.mark.parametrize("L", [4, 6, 8, 10])
def test_bonds_are_the_plaquette_edges_and_diagonals(L):
    lat = Lattice(L)
    N = L * L
    assert len(lat.bonds) == 4 * N
    pairs = {frozenset(map(int, b)) for b in lat.bonds}
    assert len(pairs) == 4 * N                       # all distinct, no self bonds
    for (i, j), kind in zip(lat.bonds, lat.bond_kind):
        d = (lat.coords[j] - lat.coords[i]) % L
        d = np.where(d > L // 2, d - L, d)
        dist2 = int((d ** 2).sum())
        assert dist2 == (1 if kind == 0 else 2)      # J1: nearest; J2: diagonal
    # every site has 4 J1 and 4 J2 partners
    for kind in (0, 1):
        deg = np.bincount(lat.bonds[lat.bond_kind == kind].ravel(), minlength=N)
        assert (deg == 4).all()


@pytest.mark.parametrize("L", [4, 6])
def test_space_group_is_a_faithful_group_of_order_8N(L):
    lat = Lattice(L)
    P = lat.perms
    assert P.shape == (8 * L * L, L * L)
    assert all(sorted(p) == list(range(L * L)) for p in P)
    keys = {p.tobytes() for p in P}
    assert len(keys) == 8 * L * L                    # faithful
    ident = np.arange(L * L)
    assert ident.tobytes() in keys
    rng = np.random.default_rng(0)
    for _ in range(300):                             # closure under composition
        g, h = rng.integers(0, len(P), 2)
        assert P[g][P[h]].tobytes() in keys


@pytest.mark.parametrize("L", [4, 6])
def test_group_maps_bonds_to_bonds_of_the_same_kind(L):
    lat = Lattice(L)
    for kind in (0, 1):
        bset = {frozenset(map(int, b)) for b in lat.bonds[lat.bond_kind == kind]}
        for p in lat.perms:
            img = {frozenset((int(p[i]), int(p[j]))) for i, j in lat.bonds[lat.bond_kind == kind]}
            assert img == bset


def test_point_classes_by_brute_force_conjugation():
    mats = [m for m in POINT_OPS]
    idx = {m.tobytes(): k for k, m in enumerate(mats)}
    classes = []
    for k, m in enumerate(mats):
        cls = {idx[(g @ m @ np.round(np.linalg.inv(g)).astype(np.int64)).tobytes()] for g in mats}
        classes.append(frozenset(cls))
    for a, b in itertools.product(range(8), range(8)):
        assert (classes[a] == classes[b]) == (POINT_CLASS[a] == POINT_CLASS[b])
    assert sorted(len(c) for c in set(classes)) == [1, 1, 2, 2, 2]
    # the axial mirrors fix a coordinate axis, the diagonal ones swap x and y
    assert POINT_CLASS[4] == POINT_CLASS[5] and abs(POINT_OPS[4]).tolist() == [[1, 0], [0, 1]]
    assert POINT_CLASS[6] == POINT_CLASS[7] and abs(POINT_OPS[6]).tolist() == [[0, 1], [1, 0]]


def test_c4v_character_orthogonality():
    names = list(C4V_CHARACTERS)
    for a in names:
        for b in names:
            s = (CLASS_SIZES * C4V_CHARACTERS[a] * C4V_CHARACTERS[b]).sum()
            assert s == (8 if a == b else 0)
    assert sum(C4V_CHARACTERS[n][0] ** 2 for n in names) == 8


@pytest.mark.parametrize("irrep", ["A1", "A2", "B1", "B2"])
@pytest.mark.parametrize("K", [(0, 0), (2, 2)])
def test_characters_are_a_homomorphism(irrep, K):
    lat = Lattice(4)
    chi = lat.characters(K[0], K[1], irrep)
    key = {p.tobytes(): g for g, p in enumerate(lat.perms)}
    rng = np.random.default_rng(1)
    for _ in range(400):
        g, h = rng.integers(0, len(chi), 2)
        gh = key[lat.perms[g][lat.perms[h]].tobytes()]
        assert abs(chi[g] * chi[h] - chi[gh]) < 1e-12


def test_unsupported_momentum_is_rejected():
    with pytest.raises(ValueError):
        Lattice(4).characters(2, 0, "A1")          # (pi, 0) is not C4v invariant
    with pytest.raises(ValueError):
        Lattice(4).characters(0, 0, "E")
