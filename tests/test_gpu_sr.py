"""Sample-space SR step (nqs_sr_solve) against the oracle.

Inputs O and E_loc come from the oracle, so the test isolates the Gram,
Cholesky and solves.  The oracle solves the P x P system of Eq. (12) and
the S x S sample-space form; by the push-through identity both equal the
GPU's dtheta.  FP64: 1e-9 relative (S < P and S > P, S not a multiple of the
32-row blocks).  FP32 (complex64 O, FP32 MFMA Gram, FP64 Cholesky): the
error budget is the FP32 Gram, so the ridge is chosen large enough that the
system is well conditioned and the relative error is gated at 1e-4.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from helpers import stress_params
from workloads import WORKLOADS, random_sz0_spins

pytestmark = pytest.mark.gpu


def make(w):
    from paper_2206_14307_amd import NQS
    return NQS.from_workload(w)


@pytest.fixture(scope="module")
def c1_inputs():
    w = WORKLOADS["4x4_fp64_exact"]
    w = dataclasses.replace(w, is_complex=True)
    p = stress_params(w, 0.1, 3)
    om = oracle.Model.from_workload(w)
    spins = random_sz0_spins(w.N, 400, 4)
    return w, om, p, spins, oracle.logderiv(om, p, spins), oracle.eloc_direct(om, p, spins)


@pytest.mark.parametrize("S", [40, 200, 400])
def test_sr_fp64_push_through(c1_inputs, S):
    w, om, p, spins, O, el = c1_inputs
    O, el = O[:S], el[:S]
    m = make(w)
    got = m.sr_solve(torch.from_numpy(O).cuda(), torch.from_numpy(el).cuda(), lam=1e-6,
                     dtau=0.02).cpu().numpy()
    ref_p = oracle.sr_param_space(O, el, 1e-6, 0.02)
    ref_s = oracle.sr_sample_space(O, el, 1e-6, 0.02)
    assert np.linalg.norm(ref_p - ref_s) < 1e-8 * np.linalg.norm(ref_s)
    assert np.linalg.norm(got - ref_s) < 1e-9 * np.linalg.norm(ref_s)


@pytest.mark.parametrize("S", [150, 300])
def test_sr_fp32_6x6(S):
    """FP32 Gram on 128 x 128 tiles: S = 150 and 300 give 2 and 3 tile rows,
    off-diagonal tiles and a partial last tile; P = 628 ends in a partial
    8-column stage."""
    w = dataclasses.replace(WORKLOADS["6x6_fp32_lanczos"], n_hidden=16)
    p = stress_params(w, 0.05, 5)
    om = oracle.Model.from_workload(w)
    spins = random_sz0_spins(w.N, S, 6)
    O = oracle.logderiv(om, p, spins).astype(np.complex64)
    el = oracle.eloc_direct(om, p, spins)
    m = make(w)
    lam = 1e-3
    got = m.sr_solve(torch.from_numpy(O).cuda(), torch.from_numpy(el).cuda(), lam=lam,
                     dtau=0.01).cpu().numpy()
    ref = oracle.sr_sample_space(O.astype(np.complex128), el, lam, 0.01)
    assert np.linalg.norm(got - ref) < 1e-4 * np.linalg.norm(ref)


def test_sr_not_positive_definite(c1_inputs):
    from paper_2206_14307_amd import NQSError
    w, om, p, spins, O, el = c1_inputs
    m = make(w)
    with pytest.raises(NQSError) as ei:
        # one sample: the centred O is zero, so with lambda = 0 the Gram matrix is 0
        m.sr_solve(torch.from_numpy(O[:1]).cuda(), torch.from_numpy(el[:1]).cuda(), lam=0.0)
    assert ei.value.status == 6
