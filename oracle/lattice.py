"""Square L x L torus: sites, J1/J2 bonds, the space group and its characters.

Test infrastructure (see the package docstring).

* Sites i = x + L*y with periodic boundaries (Sec. 3.4: L x L lattices, L even).
* Bonds of Eq. (1): nearest neighbours <ij> and the next-nearest pairs
  <<ij>> along the plaquette diagonals (Sec. 2.1).  Each site emits the
  J1 bonds (i, i+x), (i, i+y) and the J2 bonds (i, i+x+y), (i, i+x-y), so
  there are 2N of each kind for L >= 4.
* Space group (Sec. 3.1, Eqs. (4)-(6)): translations T_R, R = m x + n y,
  times the eight operations of C4v.  Reading of the passage (the point-group
  table it refers to is not part of the text): the rotation centre is site 0,
  the axial mirrors (x->-x, y->-y) form the class sigma_v, the diagonal
  mirrors form sigma_d, and the characters are the textbook C4v table below.
* Action on configurations: (g sigma)[i] = sigma[perm_g[i]] with
  perm_g(i) = site(p . r_i + t) for g = (t, p).  Character
  chi(g) = exp(-i K.t) chi_I(p); it is a one-dimensional representation only
  for K invariant under C4v, i.e. K = (0,0) or (pi,pi), and only for the
  1-D irreps A1, A2, B1, B2.
"""
from __future__ import annotations

import numpy as np

# Point operations acting on the offset (x, y) from the rotation centre:
# identity, C4, C2, C4^3, the two axial mirrors, the two diagonal mirrors.
POINT_OPS = np.array([
    [[1, 0], [0, 1]],     # E       (x, y)
    [[0, -1], [1, 0]],    # C4      (-y, x)
    [[-1, 0], [0, -1]],   # C2      (-x, -y)
    [[0, 1], [-1, 0]],    # C4^3    (y, -x)
    [[-1, 0], [0, 1]],    # sigma_v (-x, y)
    [[1, 0], [0, -1]],    # sigma_v (x, -y)
    [[0, 1], [1, 0]],     # sigma_d (y, x)
    [[0, -1], [-1, 0]],   # sigma_d (-y, -x)
], dtype=np.int64)

# Conjugacy class of each point operation: 0 E, 1 C4, 2 C2, 3 sigma_v, 4 sigma_d.
POINT_CLASS = np.array([0, 1, 2, 1, 3, 3, 4, 4])

# Textbook C4v character table over the classes (E, 2C4, C2, 2sigma_v, 2sigma_d).
C4V_CHARACTERS = {
    "A1": np.array([1, 1, 1, 1, 1]),
    "A2": np.array([1, 1, 1, -1, -1]),
    "B1": np.array([1, -1, 1, 1, -1]),
    "B2": np.array([1, -1, 1, -1, 1]),
    "E": np.array([2, 0, -2, 0, 0]),
}
CLASS_SIZES = np.array([1, 2, 1, 2, 2])


class Lattice:
    """Geometry and symmetry tables of the L x L torus (built from scratch)."""

    def __init__(self, L: int):
        if L < 4 or L % 2:
            raise ValueError("L must be even and >= 4")
        self.L = L
        self.N = L * L
        self.coords = np.array([(i % L, i // L) for i in range(self.N)], dtype=np.int64)
        self.bonds, self.bond_kind = self._bonds()
        self.perms = self._perms()

    def site(self, x, y):
        L = self.L
        return (np.asarray(x) % L) + L * (np.asarray(y) % L)

    def _bonds(self):
        """4N bonds (i, j); kind 0 = J1 (+x, +y), kind 1 = J2 (+x+y, +x-y)."""
        bonds, kind = [], []
        for shift, k in (((1, 0), 0), ((0, 1), 0), ((1, 1), 1), ((1, -1), 1)):
            for i in range(self.N):
                x, y = self.coords[i]
                bonds.append((i, int(self.site(x + shift[0], y + shift[1]))))
                kind.append(k)
        return np.array(bonds, dtype=np.int64), np.array(kind, dtype=np.int64)

    def _perms(self):
        """perm[g, i] for g = (ty*L + tx)*8 + p."""
        L, N = self.L, self.N
        out = np.empty((8 * N, N), dtype=np.int64)
        for ty in range(L):
            for tx in range(L):
                for p in range(8):
                    r = self.coords @ POINT_OPS[p].T  # p . r_i
                    out[(ty * L + tx) * 8 + p] = self.site(r[:, 0] + tx, r[:, 1] + ty)
        return out

    def translation_of(self, g: int):
        t = g // 8
        return t % self.L, t // self.L

    def characters(self, kx: int, ky: int, irrep: str) -> np.ndarray:
        """chi(g) = exp(-i K.t) chi_I(p), K = 2 pi (kx, ky) / L (Sec. 3.1, Eq. (6))."""
        if irrep not in ("A1", "A2", "B1", "B2"):
            raise ValueError("only the one-dimensional irreps A1, A2, B1, B2")
        if (kx % self.L, ky % self.L) not in ((0, 0), (self.L // 2, self.L // 2)):
            raise ValueError("K must be (0,0) or (pi,pi) for a 1-D representation of C4v")
        chi_p = C4V_CHARACTERS[irrep][POINT_CLASS]
        g = np.arange(8 * self.N)
        t = g // 8
        tx, ty = t % self.L, t // self.L
        phase = np.exp(-2j * np.pi * (kx * tx + ky * ty) / self.L)
        return phase * chi_p[g % 8]
