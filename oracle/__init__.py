"""FP64 reference implementation ("oracle") of the projected-RBM hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct CPU definition that the HIP path is checked against.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does and has no CPU fallback.  It shares no code
with the HIP library or its Python binding: it builds its own lattice,
symmetry tables and Hamiltonian from the paper.

Every function cites the passage of the paper it follows (section and
equation numbers of arXiv:2206.14307, "Systematic improvement of neural
network quantum states using a Lanczos recursion").  Readings of passages
that are silent, ambiguous or garbled are stated where they are used.
"""
from .lattice import Lattice, C4V_CHARACTERS, POINT_OPS, POINT_CLASS
from .model import Model
from .wavefunction import log2cosh, logpsi_s, logpsi, images, image_weights
from . import wavefunction, sampler
from .hamiltonian import (
    diag_energy, eloc_direct, e2_direct, e3_direct, sector_basis, hamiltonian_sector,
    hamiltonian_kron, ground_state, total_spin_sq_sector, flip_bond,
)
from .lanczos import moments, lanczos_p1, lanczos_p1_explicit, lanczos_p2, lanczos_p2_explicit
from .grad import logderiv, logderiv_fd
from .sr import sr_param_space, sr_sample_space
from .philox import philox4x64_10, uniform53
from .sampler import exchange_metropolis
from .observables import momenta, correlations, structure_factor

__all__ = [
    "Lattice", "C4V_CHARACTERS", "POINT_OPS", "POINT_CLASS", "Model",
    "log2cosh", "logpsi_s", "logpsi", "images",
    "diag_energy", "eloc_direct", "e2_direct", "e3_direct", "sector_basis", "hamiltonian_sector",
    "hamiltonian_kron", "ground_state", "total_spin_sq_sector", "flip_bond",
    "moments", "lanczos_p1", "lanczos_p1_explicit", "lanczos_p2", "lanczos_p2_explicit",
    "logderiv", "logderiv_fd", "sr_param_space", "sr_sample_space",
    "philox4x64_10", "uniform53", "exchange_metropolis",
    "momenta", "correlations", "structure_factor",
]
