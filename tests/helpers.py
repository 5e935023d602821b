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


# ---------------------------------------------------------------- error model
#
# The tolerances bound the error relative to the size of what is summed, not
# to the size of the sum.  E_loc = H_ss + sum_b (J_b/2) psi(s^b)/psi(s), each
# psi(s^b) itself a sum over the images; when the terms are large and cancel
# (stress parameters, non-A1 irreps), rounding of the terms, not of the result,
# sets the attainable error.  The scale is therefore
#   kappa_E(s) = |H_ss| + sum_b |J_b/2| sum_{k,g} |psi_s^(k)(g s^b)| / |psi(s)|,
# and for a log-derivative row O_s (sums over images of w t x) the
# componentwise bound uses sum_{k,g} |w_kg| |t_kgh| |x_gj|.  Both equal |E_loc|
# and ||O_s|| when nothing cancels.

def eloc_error_scale(model, params, spins):
    """kappa_E per configuration (see above), from the oracle's per-image
    amplitudes of every exchange neighbour (no division by psi(s^b), which
    may vanish)."""
    import oracle
    spins = np.atleast_2d(np.asarray(spins))
    lp = oracle.logpsi(model, params, spins)
    diag = oracle.diag_energy(model, spins)
    bi, bj = model.lat.bonds[:, 0], model.lat.bonds[:, 1]
    out = np.empty(len(spins))
    for r, s in enumerate(spins):
        anti = np.nonzero(s[bi] != s[bj])[0]
        conn = np.repeat(s[None, :], len(anti), axis=0)
        rows = np.arange(len(anti))
        conn[rows, bi[anti]], conn[rows, bj[anti]] = s[bj[anti]], s[bi[anti]]
        Xg = oracle.images(model, conn)
        tot = np.zeros(len(anti))
        for (W, a, b) in model.split(params):
            ls = oracle.logpsi_s(Xg, W, a, b)
            tot += np.exp(ls.real - lp[r].real).sum(axis=1)
        out[r] = abs(diag[r]) + (0.5 * np.abs(model.bond_J[anti]) * tot).sum()
    return out


def max_scaled_eloc_err(got, ref, scale):
    """max_s |got - ref| / max(1, kappa_E(s))."""
    got, ref = np.asarray(got), np.asarray(ref)
    return float((np.abs(got - ref) / np.maximum(1.0, np.asarray(scale))).max())


def logpsi_error_scale(model, params, spins):
    """kappa_psi = sum_{k,g} |psi_s^(k)(g sigma)| / |psi(sigma)| per
    configuration: the size of log psi's terms relative to the sum (1 when
    the images add up without cancelling)."""
    import oracle
    w, _, _ = oracle.image_weights(model, params, spins)
    return np.abs(w).sum(axis=(1, 2))


def max_scaled_logpsi_err(a, b, kappa):
    """max |wrapped (a - b)| / kappa (log psi to the size of its terms)."""
    return float((np.abs(wrap_diff(np.asarray(a), np.asarray(b))) / np.asarray(kappa)).max())


def grad_error_scale(model, params, spins):
    """||sum_{k,g} |w_kg| |t_kgh| |x_gj| ||_2 per configuration, over the
    same [W | a | b] layout as the oracle's log-derivatives."""
    import oracle
    w, t, Xg = oracle.image_weights(model, params, spins)
    aw, at, ax = np.abs(w), np.abs(t), np.abs(Xg)
    S = Xg.shape[0]
    parts = []
    for k in range(model.n_rbm):
        wt = aw[:, k, :, None] * at[:, k]
        parts.append(np.einsum("sgh,sgj->shj", wt, ax).reshape(S, -1))
        if model.use_bias:
            parts.append(np.einsum("sg,sgj->sj", aw[:, k], ax))
            parts.append(wt.sum(axis=1))
    return np.linalg.norm(np.concatenate(parts, axis=1), axis=1)


def max_scaled_row_err(A, B, scale):
    """max_s ||A_s - B_s|| / max(||B_s||, scale_s)."""
    A, B = np.asarray(A), np.asarray(B)
    den = np.maximum(np.linalg.norm(B, axis=1), np.asarray(scale))
    return float((np.linalg.norm(A - B, axis=1) / den).max())
