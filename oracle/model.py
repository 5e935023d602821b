"""Model description for the oracle: Hamiltonian couplings + ansatz shape.

Test infrastructure (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

from .lattice import Lattice


@dataclass
class Model:
    """J1-J2 Heisenberg model (Eq. (1)) + projected linear combination of RBMs.

    The wave function (Sec. 3.1, Eq. (6), summed over ``n_rbm`` RBMs as the
    linear combination the paper introduces) is
        psi(sigma) = sum_k sum_g chi(g) psi_s^(k)(g sigma)
    with unit coefficients for the K RBMs (reading: the paper gives none).
    """
    L: int
    J1: float = 1.0
    J2: float = 0.5
    kx: int = 0
    ky: int = 0
    irrep: str = "A1"
    n_rbm: int = 1
    n_hidden: int = 16
    use_bias: bool = True
    lat: Lattice = field(init=False, repr=False)
    chi: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self.lat = Lattice(self.L)
        self.chi = self.lat.characters(self.kx, self.ky, self.irrep)

    @property
    def N(self):
        return self.lat.N

    @property
    def G(self):
        return 8 * self.lat.N

    @property
    def bond_J(self):
        return np.where(self.lat.bond_kind == 0, self.J1, self.J2)

    @property
    def params_per_rbm(self):
        M, N = self.n_hidden, self.N
        return M * N + (N + M if self.use_bias else 0)

    def split(self, params):
        """params [K, P_rbm] -> list of (W [M,N], a [N], b [M]) per RBM."""
        params = np.asarray(params, dtype=np.complex128).reshape(self.n_rbm, self.params_per_rbm)
        M, N = self.n_hidden, self.N
        out = []
        for k in range(self.n_rbm):
            W = params[k, : M * N].reshape(M, N)
            if self.use_bias:
                a = params[k, M * N: M * N + N]
                b = params[k, M * N + N:]
            else:
                a = np.zeros(N, np.complex128)
                b = np.zeros(M, np.complex128)
            out.append((W, a, b))
        return out

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(L=w.L, J1=w.J1, J2=w.J2, kx=w.kx, ky=w.ky, irrep=w.irrep,
                  n_rbm=w.n_rbm, n_hidden=w.n_hidden, use_bias=w.use_bias)
        kw.update(over)
        return cls(**kw)
