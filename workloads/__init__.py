"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module holds none of the method's arithmetic: it only describes the
workloads (lattice size, couplings, RBM shape, precision, sample counts) and
draws random numbers -- RBM parameters and uniformly random Sz=0 spin
configurations -- from ``numpy.random.default_rng(seed)``.  Both sides receive
exactly the same arrays, so random-number generation is never a parity issue.

Conventions
-----------
* Spin code: int8 +1 / -1 encodes sigma^z = +1/2 / -1/2 (Sec. 2.1; Sec. 3.1
  maps configurations of N values +-1/2 to amplitudes).  Site i = x + L*y.
* Parameters: complex array of shape [K, P_rbm] with the per-RBM layout
  [W (M x N, row-major) | a (N) | b (M)] when ``use_bias`` is set and [W]
  otherwise (the bias-free spin-flip-symmetric form of Sec. 3.1).
"""
from __future__ import annotations

from dataclasses import dataclass, asdict
import numpy as np

IRREPS = {"A1": 0, "A2": 1, "B1": 2, "B2": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x2": 2}


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: the model plus how many configurations it uses."""
    name: str
    L: int
    J1: float = 1.0
    J2: float = 0.5
    kx: int = 0          # K = 2*pi*(kx, ky)/L; only (0,0) and (L/2, L/2) are 1-D reps
    ky: int = 0
    irrep: str = "A1"
    n_rbm: int = 1
    n_hidden: int = 16
    is_complex: bool = True
    use_bias: bool = True
    precision: str = "fp32"
    param_std: float = 0.01
    seed: int = 1000
    n_chains: int = 0
    n_per_chain: int = 0
    n_samples: int = 0   # 0: full Sz=0 enumeration

    @property
    def N(self) -> int:
        return self.L * self.L

    @property
    def G(self) -> int:
        return 8 * self.N

    @property
    def params_per_rbm(self) -> int:
        M, N = self.n_hidden, self.N
        return M * N + (N + M if self.use_bias else 0)

    @property
    def n_params(self) -> int:
        return self.n_rbm * self.params_per_rbm

    def describe(self) -> dict:
        d = asdict(self)
        d.update(N=self.N, G=self.G, n_params=self.n_params)
        return d


# The five workloads: 4x4 exact enumeration (FP64, real), 6x6 FP32 complex
# logpsi+E_loc, 6x6 with the p=1 Lanczos step and the backward, 8x8 with a
# linear combination of four RBMs, 10x10 with M = 4N.
WORKLOADS = {
    "4x4_fp64_exact": Workload("4x4_fp64_exact", L=4, n_hidden=16, is_complex=False,
                               precision="fp64", seed=1001),
    "6x6_fp32_eloc": Workload("6x6_fp32_eloc", L=6, n_hidden=72, precision="fp32",
                              seed=1002, n_chains=4096, n_per_chain=64),
    "6x6_fp32_lanczos": Workload("6x6_fp32_lanczos", L=6, n_hidden=72, precision="fp32",
                                 seed=1003, n_chains=512, n_per_chain=16),
    "8x8_k4_m256": Workload("8x8_k4_m256", L=8, n_rbm=4, n_hidden=256, precision="bf16x2",
                            seed=1004, n_chains=1024, n_per_chain=16),
    "10x10_m400": Workload("10x10_m400", L=10, n_hidden=400, precision="bf16x2",
                           seed=1005, n_chains=1024, n_per_chain=32),
}


def draw_params(w: Workload, std: float | None = None, seed: int | None = None) -> np.ndarray:
    """Draw RBM parameters ~ N(0, std) independently for Re and Im.

    Order of draws: for each RBM k, W then a then b, each as all real parts
    followed by all imaginary parts.  FP32 and split-BF16 workloads round the
    draws to float32, so both sides see float32-representable values.
    Returns complex128 [K, params_per_rbm] (imaginary part 0 for real RBMs).
    """
    std = w.param_std if std is None else std
    rng = np.random.default_rng(w.seed if seed is None else seed)
    N, M = w.N, w.n_hidden
    sizes = [M * N] + ([N, M] if w.use_bias else [])
    out = np.zeros((w.n_rbm, w.params_per_rbm), dtype=np.complex128)
    for k in range(w.n_rbm):
        off = 0
        for n in sizes:
            re = rng.normal(0.0, std, n)
            im = rng.normal(0.0, std, n) if w.is_complex else np.zeros(n)
            out[k, off:off + n] = re + 1j * im
            off += n
    if w.precision != "fp64":
        out = out.astype(np.complex64).astype(np.complex128)
    return out


def random_sz0_spins(N: int, n: int, seed: int) -> np.ndarray:
    """n uniformly random Sz=0 configurations as int8 [n, N] of +-1."""
    rng = np.random.default_rng(seed)
    base = np.concatenate([np.ones(N // 2, np.int8), -np.ones(N // 2, np.int8)])
    out = np.empty((n, N), np.int8)
    for s in range(n):
        out[s] = rng.permutation(base)
    return out


def random_sz0_spins_fast(N: int, n: int, seed: int) -> np.ndarray:
    """Vectorised variant of random_sz0_spins for large n (different stream)."""
    rng = np.random.default_rng(seed)
    keys = rng.random((n, N))
    order = np.argsort(keys, axis=1)
    out = -np.ones((n, N), np.int8)
    np.put_along_axis(out, order[:, : N // 2], 1, axis=1)
    return out
