"""J1-J2 Heisenberg Hamiltonian (Eq. (1)): local energies, H^2 terms, ED.

Test infrastructure (see the package docstring).

With S_i.S_j = S^z_i S^z_j + (S^+_i S^-_j + S^-_i S^+_j)/2 and sigma = +-1/2,
a bond b = (i, j) contributes J_b sigma_i sigma_j on the diagonal and, when
sigma_i != sigma_j, the matrix element J_b/2 to the configuration sigma^b in
which the two spins are exchanged.  The search is restricted to the Sz = 0
sector (Sec. 2.1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .wavefunction import logpsi


def diag_energy(model, spins):
    """H_{sigma sigma} = sum_b J_b sigma_i sigma_j with sigma = +-1/2."""
    s = np.atleast_2d(np.asarray(spins, dtype=np.float64)) * 0.5
    i, j = model.lat.bonds[:, 0], model.lat.bonds[:, 1]
    return (s[:, i] * s[:, j]) @ model.bond_J


def flip_bond(spins, i, j):
    out = np.array(spins, copy=True)
    out[..., [i, j]] = out[..., [j, i]]
    return out


def _connected(model, spins):
    """All (sample, bond) pairs with antiparallel spins and their sigma^b."""
    spins = np.atleast_2d(np.asarray(spins))
    i, j = model.lat.bonds[:, 0], model.lat.bonds[:, 1]
    anti = spins[:, i] != spins[:, j]                     # [S, 4N]
    s_idx, b_idx = np.nonzero(anti)
    conn = spins[s_idx].copy()
    bi, bj = i[b_idx], j[b_idx]
    r = np.arange(len(s_idx))
    conn[r, bi], conn[r, bj] = spins[s_idx, bj], spins[s_idx, bi]
    return s_idx, b_idx, conn


def eloc_direct(model, params, spins, logpsi_fn=None):
    """E_loc(sigma) = <sigma|H|psi>/<sigma|psi> (Sec. 3.2, Eq. (10)), with every
    psi(sigma^b) re-evaluated from scratch (no update identities)."""
    lp_fn = logpsi_fn or (lambda s: logpsi(model, params, s))
    spins = np.atleast_2d(np.asarray(spins))
    lp = lp_fn(spins)
    s_idx, b_idx, conn = _connected(model, spins)
    lp_conn = lp_fn(conn)
    terms = 0.5 * model.bond_J[b_idx] * np.exp(lp_conn - lp[s_idx])
    off = np.zeros(spins.shape[0], np.complex128)
    np.add.at(off, s_idx, terms)
    return diag_energy(model, spins) + off


def e2_direct(model, params, spins):
    """e2(sigma) = <sigma|H^2|psi>/<sigma|psi> by the direct double sum
    sum_{sigma'} H_{sigma sigma'} psi(sigma')/psi(sigma) E_loc(sigma'),
    every amplitude re-evaluated (needed for <H^2>, <H^3> of Sec. 3.3)."""
    spins = np.atleast_2d(np.asarray(spins))
    lp = logpsi(model, params, spins)
    e1 = eloc_direct(model, params, spins)
    s_idx, b_idx, conn = _connected(model, spins)
    lp_conn = logpsi(model, params, conn)
    e1_conn = eloc_direct(model, params, conn)
    terms = 0.5 * model.bond_J[b_idx] * np.exp(lp_conn - lp[s_idx]) * e1_conn
    off = np.zeros(spins.shape[0], np.complex128)
    np.add.at(off, s_idx, terms)
    return diag_energy(model, spins) * e1 + off


def e3_direct(model, params, spins):
    """e3(sigma) = <sigma|H^3|psi>/<sigma|psi>, one hop further than e2:
    H_{sigma sigma} e2(sigma) + sum_b (J_b/2) psi(sigma^b)/psi(sigma) e2(sigma^b),
    with e2 at every neighbour from e2_direct (the <H^4>, <H^5> of a p = 2
    Lanczos step, Sec. 3.3, need it)."""
    spins = np.atleast_2d(np.asarray(spins))
    lp = logpsi(model, params, spins)
    e2 = e2_direct(model, params, spins)
    s_idx, b_idx, conn = _connected(model, spins)
    lp_conn = logpsi(model, params, conn)
    e2_conn = e2_direct(model, params, conn)
    terms = 0.5 * model.bond_J[b_idx] * np.exp(lp_conn - lp[s_idx]) * e2_conn
    off = np.zeros(spins.shape[0], np.complex128)
    np.add.at(off, s_idx, terms)
    return diag_energy(model, spins) * e2 + off


# ---------------------------------------------------------------- the sector

def sector_basis(N):
    """All Sz = 0 configurations in colex order = increasing bit mask
    (bit i set <=> site i up); returns (masks int64 [D], spins int8 [D, N])."""
    masks = np.array([m for m in range(1 << N) if bin(m).count("1") == N // 2],
                     dtype=np.int64)
    spins = np.where((masks[:, None] >> np.arange(N)) & 1, 1, -1).astype(np.int8)
    return masks, spins


def _sector_matrix(N, bonds, J, masks):
    """Sparse sum_b J_b S_i.S_j on the Sz = 0 sector basis given by masks."""
    D = len(masks)
    bits = ((masks[:, None] >> np.arange(N)) & 1).astype(np.int8)
    s = bits.astype(np.float64) - 0.5
    diag = (s[:, bonds[:, 0]] * s[:, bonds[:, 1]]) @ J
    rows, cols, vals = [np.arange(D)], [np.arange(D)], [diag]
    for (i, j), Jb in zip(bonds, J):
        src = np.nonzero(bits[:, i] != bits[:, j])[0]
        dst = np.searchsorted(masks, masks[src] ^ ((1 << int(i)) | (1 << int(j))))
        rows.append(dst)
        cols.append(src)
        vals.append(np.full(len(src), 0.5 * Jb))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(D, D))


def hamiltonian_sector(model, masks=None):
    """Sparse H on the Sz = 0 sector basis (rows/cols in colex order)."""
    if masks is None:
        masks, _ = sector_basis(model.N)
    return _sector_matrix(model.N, model.lat.bonds, model.bond_J, masks)


def hamiltonian_kron(model):
    """Full 2^N Hamiltonian assembled from Kronecker products of spin-1/2
    matrices, S_i.S_j = sum_a S^a_i S^a_j, basis index sum_i bit_i 2^i with
    bit 1 = up.  An independent construction used to pin the sector matrix."""
    N = model.N
    sz = sp.csr_matrix(np.array([[-0.5, 0], [0, 0.5]]))
    sx = sp.csr_matrix(np.array([[0, 0.5], [0.5, 0]]))
    sy = sp.csr_matrix(np.array([[0, 0.5j], [-0.5j, 0]]))
    eye = sp.identity(2, format="csr")

    def site_op(op, i):
        out = sp.identity(1, format="csr")
        for k in range(N - 1, -1, -1):                    # site N-1 most significant
            out = sp.kron(out, op if k == i else eye, format="csr")
        return out

    ops = {a: [site_op(o, i) for i in range(N)] for a, o in (("x", sx), ("y", sy), ("z", sz))}
    H = sp.csr_matrix((1 << N, 1 << N), dtype=np.complex128)
    for (i, j), J in zip(model.lat.bonds, model.bond_J):
        for a in ("x", "y", "z"):
            H = H + J * (ops[a][i] @ ops[a][j])
    return H


def total_spin_sq_sector(model, masks=None):
    """S^2 = sum_{i,j} S_i.S_j = 3N/4 + 2 sum_{i<j} S_i.S_j on the sector."""
    N = model.N
    if masks is None:
        masks, _ = sector_basis(N)
    pairs = np.array([(i, j) for i in range(N) for j in range(i + 1, N)], dtype=np.int64)
    H = _sector_matrix(N, pairs, np.full(len(pairs), 2.0), masks)
    return H + 0.75 * N * sp.identity(len(masks), format="csr")


def ground_state(model, k=1):
    """Lowest eigenpair(s) of H on the Sz = 0 sector (exact diagonalisation,
    the reference the paper compares with in Sec. 4.1)."""
    masks, spins = sector_basis(model.N)
    H = hamiltonian_sector(model, masks)
    vals, vecs = spla.eigsh(H, k=k, which="SA", tol=1e-12)
    order = np.argsort(vals)
    return vals[order], vecs[:, order], masks, spins
