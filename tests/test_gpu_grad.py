"""Log-derivatives O_k (nqs_grad) against the oracle, through the C ABI.

Models with K*M <= 128 in FP32 or split-BF16 theta take the fused gradient
kernel (theta, weights and the image contraction in one pass, nothing of
size S x G x K*M in HBM); the rest take the materialised path.  Each case
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
from helpers import TOL, max_logpsi_err, max_row_rel_err, nonzero_rows, stress_params
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
    assert max_row_rel_err(O.cpu().numpy(), oracle.logderiv(om, p, sp)) < tol
    assert max_logpsi_err(lp.cpu().numpy(), oracle.logpsi(om, p, sp)) < tol


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
