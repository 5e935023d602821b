"""Log-derivatives O_k (nqs_grad) against the oracle, through the C ABI.

Models with K*M <= 128 in FP32 or split-BF16 theta take the fused gradient
kernel (theta, weights and the image contraction in one pass, nothing of
size S x G x K*M in HBM); wider FP32 / split-BF16 models take the wide
gradient kernel (image weights from a log-amplitude pass, theta recomputed
in-kernel); FP64 models the materialised path.  Each case
compares every O row with the oracle's gradient, per row ||dO|| / ||O||,
and the log psi that nqs_grad also returns.  Cases: drawn parameters and
stress parameters (std 0.3, complex, B1 at K = (pi, pi)), one and two RBMs,
with and without biases, ragged and degenerate sizes, and the full
262 144-configuration launch checked on sampled rows.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from helpers import (TOL, grad_error_scale, logpsi_error_scale, max_logpsi_err, max_rel_err,
                     max_row_rel_err, max_scaled_logpsi_err, max_scaled_row_err, nonzero_rows,
                     stress_params)
from workloads import WORKLOADS, draw_params, random_sz0_spins

pytestmark = pytest.mark.gpu


def make(w, params):
    from paper_2206_14307_amd import NQS
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(params.reshape(-1)))
    return m


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    # name: (workload, overrides, parameter std or None for the drawn ones)
    "6x6_m72_fp32": ("6x6_fp32_eloc", {}, None),
    "6x6_m72_bf16x2": ("6x6_fp32_eloc", {"precision": "bf16x2"}, None),
    "6x6_k2_m16_stress_b1": ("6x6_fp32_eloc", {"n_rbm": 2, "n_hidden": 16, "irrep": "B1",
                                                "kx": 3, "ky": 3}, 0.3),
    "6x6_m16_nobias": ("6x6_fp32_eloc", {"n_hidden": 16, "use_bias": False}, 0.1),
    "4x4_m16_fp32": ("4x4_fp64_exact", {"precision": "fp32", "is_complex": True}, 0.2),
    "4x4_k2_m8_nobias": ("4x4_fp64_exact", {"precision": "fp32", "is_complex": True,
                                            "n_rbm": 2, "n_hidden": 8, "use_bias": False}, 0.2),
    # K*M > 128: theta (log amplitudes only) + log-sum-exp, then the wide
    # gradient kernel with theta recomputed in-kernel
    "8x8_k4_m256_fp32": ("8x8_k4_m256", {"precision": "fp32"}, None),
    "8x8_k4_m256_bf16x2": ("8x8_k4_m256", {}, None),
    "10x10_m400_bf16x2_std0.05": ("10x10_m400", {}, 0.05),
    "10x10_m400_fp32": ("10x10_m400", {"precision": "fp32"}, None),
    "6x6_m144_b1_pi": ("6x6_fp32_eloc", {"n_hidden": 144, "irrep": "B1", "kx": 3, "ky": 3}, 0.1),
    "6x6_k2_m128_nobias_bf16x2": ("6x6_fp32_eloc", {"n_rbm": 2, "n_hidden": 128, "use_bias": False,
                                                    "precision": "bf16x2"}, 0.05),
}


@pytest.mark.parametrize("case", list(CASES))
def test_grad_vs_oracle(case):
    name, over, std = CASES[case]
    w = dataclasses.replace(WORKLOADS[name], **over)
    p = draw_params(w) if std is None else stress_params(w, std, 21)
    om = oracle.Model.from_workload(w)
    sp = random_sz0_spins(w.N, 60, 8)
    sp = sp[nonzero_rows(om, p, sp)][:37]              # ragged: not a multiple of 8 waves
    m = make(w, p)
    O, lp = m.grad(cuda(sp), want_logpsi=True)
    tol = TOL[w.precision]
    ref, lref = oracle.logderiv(om, p, sp), oracle.logpsi(om, p, sp)
    O, lp = O.cpu().numpy(), lp.cpu().numpy()
    # every case against the size of the terms (the error model of the
    # tolerances: sum_kg |w||t||x| for an O row, sum_kg |psi_s(g sigma)|/|psi|
    # for log psi); the drawn parameters, whose images do not cancel, also
    # row by row against ||O|| and absolutely on log psi
    err_o = max_scaled_row_err(O, ref, grad_error_scale(om, p, sp))
    err_l = max_scaled_logpsi_err(lp, lref, logpsi_error_scale(om, p, sp))
    print(f"{case}: O scaled {err_o:.3g} row-relative {max_row_rel_err(O, ref):.3g}; "
          f"log psi scaled {err_l:.3g} absolute {max_logpsi_err(lp, lref):.3g}")
    assert err_o < tol and err_l < tol
    if std is None:
        assert max_row_rel_err(O, ref) < tol
        assert max_logpsi_err(lp, lref) < tol


def test_grad_empty_and_single():
    w = WORKLOADS["6x6_fp32_eloc"]
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    sp = random_sz0_spins(w.N, 1, 3)
    m = make(w, p)
    assert m.grad(cuda(sp[:0])).numel() == 0
    O = m.grad(cuda(sp)).cpu().numpy()
    assert max_row_rel_err(O, oracle.logderiv(om, p, sp)) < TOL["fp32"]


def test_grad_full_size_sampled_rows():
    """All 262 144 configurations of the 6x6 workload in one call (the size
    the gradient leg of bench.py times); six rows are checked one by one."""
    w = WORKLOADS["6x6_fp32_eloc"]
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    S = w.n_chains * w.n_per_chain
    rng = np.random.default_rng(4)
    sp = rng.permuted(np.tile(np.r_[np.ones(18, np.int8), -np.ones(18, np.int8)], (S, 1)), axis=1)
    m = make(w, p)
    O, lp = m.grad(cuda(sp), want_logpsi=True)
    rows = np.r_[0, S - 1, rng.choice(S, 4, replace=False)]
    Os = O[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert max_row_rel_err(Os, oracle.logderiv(om, p, sp[rows])) < TOL["fp32"]
    assert max_logpsi_err(lp.cpu().numpy()[rows], oracle.logpsi(om, p, sp[rows])) < TOL["fp32"]
    del O


LOGPSI_CASES = {
    # name: (workload, overrides, parameter std or None for the drawn ones)
    "6x6_m16_fp32_complex": ("6x6_fp32_eloc", {"n_hidden": 16}, 0.1),
    "4x4_fp64_real": ("4x4_fp64_exact", {}, None),
}


@pytest.mark.parametrize("case", list(LOGPSI_CASES))
def test_logpsi_autograd_function(case):
    """LogPsi (torch.autograd.Function over nqs_logpsi / nqs_grad): the gradient
    of L = Re sum_s c_s log psi_s, for random complex c, equals
    conj(sum_s c_s O_sk) (its real part for a real RBM) with the oracle's
    log-derivatives, and central finite differences of the oracle's log psi
    along Re and Im of a few parameters; the forward equals the oracle's
    log psi and leaves the context's parameters unchanged."""
    from paper_2206_14307_amd import LogPsi
    name, over, std = LOGPSI_CASES[case]
    w = dataclasses.replace(WORKLOADS[name], **over)
    p = draw_params(w) if std is None else stress_params(w, std, 13)
    om = oracle.Model.from_workload(w)
    sp = random_sz0_spins(w.N, 9, 17)
    sp = sp[nonzero_rows(om, p, sp)]
    rng = np.random.default_rng(3)
    c = rng.normal(size=len(sp)) + 1j * rng.normal(size=len(sp))
    m = make(w, np.zeros_like(p))                       # the context holds other parameters
    before = m.get_params().cpu().numpy()
    pt = torch.from_numpy(p.reshape(-1) if w.is_complex else p.reshape(-1).real.copy())
    pt = pt.cuda().requires_grad_(True)
    lp = LogPsi.apply(pt, cuda(sp), m)
    assert np.array_equal(m.get_params().cpu().numpy(), before)
    tol = TOL[w.precision]
    assert max_logpsi_err(lp.detach().cpu().numpy(), oracle.logpsi(om, p, sp)) < tol
    L = (torch.from_numpy(c).cuda() * lp).real.sum()
    (g,) = torch.autograd.grad(L, pt)
    g = g.cpu().numpy()
    assert g.dtype == (np.complex128 if w.is_complex else np.float64)
    cO = (c[:, None] * oracle.logderiv(om, p, sp)).sum(axis=0)
    ref = np.conj(cO) if w.is_complex else cO.real
    assert np.linalg.norm(g - ref) < tol * np.linalg.norm(ref)
    # finite differences of the oracle along the real (and imaginary) direction
    idx = np.r_[0, 7, len(ref) // 2, len(ref) - 1]
    fd = (c[:, None] * oracle.logderiv_fd(om, p, sp, indices=idx)).sum(axis=0)
    fd_tol = max(tol, 1e-8)
    assert np.abs(g[idx].real - fd.real).max() < fd_tol * np.abs(ref).max()
    if w.is_complex:
        # d L / d Im p_k = Re sum_s c_s (i O_sk) = -Im sum_s c_s O_sk = Im g_k
        assert np.abs(g[idx].imag + fd.imag).max() < fd_tol * np.abs(ref).max()
    # no gradient wanted: log psi alone (no O formed), same values
    with torch.no_grad():
        lp2 = LogPsi.apply(pt.detach(), cuda(sp), m)
    assert max_logpsi_err(lp2.cpu().numpy(), lp.detach().cpu().numpy()) < tol


@pytest.mark.parametrize("name,over", [("6x6_fp32_eloc", {"n_hidden": 144}),
                                       ("6x6_fp32_eloc", {"n_rbm": 8, "n_hidden": 24})])
def test_eloc_grad_edges(name, over):
    """nqs_eloc_grad on a wide model sharing the log amplitudes (K = 1, M = 144)
    and on one beyond the shared path (K = 8 > 4 RBMs: nqs_eloc, then nqs_grad):
    no configurations, a single one against the oracle, a too-small workspace."""
    from paper_2206_14307_amd.nqs import NQSError, _ptr, _stream
    w = dataclasses.replace(WORKLOADS[name], **over)
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    m = make(w, p)
    sp = random_sz0_spins(w.N, 3, 9)
    lp, el, O = m.eloc_grad(cuda(sp[:0]))
    assert el.numel() == 0 and O.numel() == 0
    lp, el, O = m.eloc_grad(cuda(sp))
    tol = TOL[w.precision]
    assert max_rel_err(el.cpu().numpy(), oracle.eloc_direct(om, p, sp)) < tol
    assert max_row_rel_err(O.cpu().numpy(), oracle.logderiv(om, p, sp)) < tol
    lp2, el2 = m.eloc(cuda(sp))
    assert torch.equal(lp, lp2) and torch.equal(el, el2)
    need = int(m.lib.nqs_workspace_bytes(m._ctx, 10, 3))
    ws = torch.empty(max(need // 2, 1), dtype=torch.uint8, device="cuda")
    spt = cuda(sp)
    st = m.lib.nqs_eloc_grad(m._ctx, _ptr(spt), 3, None, _ptr(el), _ptr(O), _ptr(ws), ws.numel(),
                             _stream())
    with pytest.raises(NQSError, match="workspace too small"):
        m._check(st, "nqs_eloc_grad")
