"""Comparison helpers and tolerances shared by the GPU parity tests.

Tolerances (absolute on log psi = relative on psi; relative elsewhere):
FP64 1e-10, FP32 1e-5, split-BF16 theta 1e-4.  E_loc and e2 errors are
measured as |d| / max(1, |value|); O_k as ||dO_s|| / ||O_s|| per sample.
"""
import numpy as np

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x2": 1e-4}


def wrap_diff(a, b):
    """log-amplitude difference with the imaginary part wrapped to (-pi, pi]."""
    d = np.asarray(a) - np.asarray(b)
    return d.real + 1j * np.angle(np.exp(1j * d.imag))


def max_logpsi_err(a, b):
    return float(np.abs(wrap_diff(a, b)).max())


def max_rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float((np.abs(a - b) / np.maximum(1.0, np.abs(b))).max())


def max_row_rel_err(A, B):
    A, B = np.asarray(A), np.asarray(B)
    return float((np.linalg.norm(A - B, axis=1) / np.linalg.norm(B, axis=1)).max())


def stress_params(w, std, seed):
    rng = np.random.default_rng(seed)
    n = w.n_rbm * w.params_per_rbm
    p = rng.normal(0, std, n) + 1j * rng.normal(0, std, n)
    p = p.reshape(w.n_rbm, -1)
    if w.precision != "fp64":
        p = p.astype(np.complex64).astype(np.complex128)
    return p


def nonzero_rows(model, params, spins, cut=30.0):
    """Rows whose amplitude is not a symmetry zero (|psi| not at rounding level
    relative to its largest image term)."""
    import oracle
    w, _, _ = oracle.image_weights(model, params, spins)
    return np.abs(w).sum(axis=(1, 2)) < np.exp(cut)


def reciprocal_form_in_range(model, params, lg=96.0):
    """Whether the fused E_loc kernel may take the factors in the form
    T_h (t_h + s / T_h): with the hidden units of one RBM split into eight
    streams h = 8 j + r (j ascending), every suffix product of |tanh(D_h)|
    along a stream, D_h = W_h,p - W_h,q for a bond (p, q), must lie in
    [2^-lg, 2^lg].  Evaluated independently of the library to tell which form
    a test exercises."""
    M = model.n_hidden
    for W, _, _ in model.split(params):
        D = W[:, model.lat.bonds[:, 0]] - W[:, model.lat.bonds[:, 1]]      # [M, NB]
        with np.errstate(divide="ignore"):
            lg2 = np.log2(np.abs(np.tanh(D)))
        for r in range(8):
            suf = np.cumsum(lg2[r::8][::-1], axis=0)
            if not ((suf >= -lg) & (suf <= lg)).all():
                return False
    return True
