"""Spin structure factor (nqs_structure_factor) against the oracle's S(q),
through the C ABI.  FP64 arithmetic on both sides: tolerance 1e-10 relative
to max S(q) (only the summation order differs)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from workloads import WORKLOADS, draw_params, random_sz0_spins

pytestmark = pytest.mark.gpu
TOL = 1e-10


def make(name, **over):
    from paper_2206_14307_amd import NQS
    w = dataclasses.replace(WORKLOADS[name], **over)
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    return w, m


def close(got, ref):
    return np.abs(np.asarray(got) - ref).max() <= TOL * max(1.0, np.abs(ref).max())


def test_exact_sector_with_born_weights():
    """4x4: the whole Sz = 0 sector (nqs_enumerate_sz0) weighted by |psi|^2
    from nqs_logpsi, against the oracle's S(q) of its own |psi|^2."""
    w, m = make("4x4_fp64_exact")
    sp = m.enumerate_sz0()
    lp = m.logpsi(sp)
    wts = torch.exp(2.0 * (lp.real - lp.real.max()))
    got = m.structure_factor(sp, wts).cpu().numpy()
    om = oracle.Model.from_workload(w)
    spn = sp.cpu().numpy()
    lpo = oracle.logpsi(om, draw_params(w), spn)
    ref = oracle.structure_factor(om.lat, spn, np.exp(2.0 * (lpo.real - lpo.real.max())))
    assert close(got, ref)


@pytest.mark.parametrize("name,S", [("6x6_fp32_eloc", 517), ("10x10_m400", 300)])
def test_samples_uniform_and_weighted(name, S):
    """Random Sz = 0 configurations (more than one wavefront's worth per
    block, a ragged count), uniform and random weights; 10x10 takes two
    momenta per lane."""
    w, m = make(name)
    lat = oracle.Lattice(w.L)
    sp = random_sz0_spins(w.N, S, 7)
    got = m.structure_factor(torch.from_numpy(sp).cuda()).cpu().numpy()
    assert close(got, oracle.structure_factor(lat, sp))
    wts = np.random.default_rng(8).random(S)
    wts[::5] = 0.0
    got = m.structure_factor(torch.from_numpy(sp).cuda(), torch.from_numpy(wts)).cpu().numpy()
    assert close(got, oracle.structure_factor(lat, sp, wts))


def test_full_size_launch():
    """All 262 144 configurations of the 6x6 benchmark size in one call."""
    w, m = make("6x6_fp32_eloc")
    lat = oracle.Lattice(w.L)
    rng = np.random.default_rng(4)
    S = w.n_chains * w.n_per_chain
    sp = rng.permuted(np.tile(np.r_[np.ones(18, np.int8), -np.ones(18, np.int8)], (S, 1)), axis=1)
    got = m.structure_factor(torch.from_numpy(sp).cuda()).cpu().numpy()
    assert close(got, oracle.structure_factor(lat, sp))
    assert abs(got.sum() - 0.25) < 1e-12 and abs(got[0]) < 1e-15


@pytest.mark.parametrize("L", [4, 6, 8, 10])
def test_neel_stripe_and_single_sample(L):
    name = {4: "4x4_fp64_exact", 6: "6x6_fp32_eloc", 8: "8x8_k4_m256", 10: "10x10_m400"}[L]
    w, m = make(name)
    x, y = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
    neel = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8).reshape(1, -1)
    stripe = np.where(x % 2 == 0, 1, -1).astype(np.int8).reshape(1, -1)
    h = L // 2
    S = m.structure_factor(torch.from_numpy(neel).cuda()).cpu().numpy()
    assert abs(S[h + L * h] - 0.25) < 1e-15 and abs(S.sum() - 0.25) < 1e-14
    S = m.structure_factor(torch.from_numpy(stripe).cuda()).cpu().numpy()
    assert abs(S[h] - 0.25) < 1e-15 and abs(S[L * h]) < 1e-15


def test_errors():
    from paper_2206_14307_amd import NQSError
    w, m = make("6x6_fp32_eloc")
    with pytest.raises(NQSError):
        m.structure_factor(torch.zeros((0, 36), dtype=torch.int8, device="cuda"))
