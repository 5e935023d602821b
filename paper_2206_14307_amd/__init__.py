"""MI355X (gfx950) hot path of the symmetry-projected RBM + Lanczos method
(arXiv:2206.14307): batched log psi, local energies, two-hop H^2 terms with
FP64 Lanczos moments, log-derivatives, sample-space SR and exchange
Metropolis sampling, behind the C ABI of include/nqs.h (libnqs.so)."""
from .nqs import NQS, LogPsi, NQSError, load_library, LIB_PATH, EXPORTS, KERNELS  # noqa: F401
