"""nqs_eloc_noalloc (the allocation-free variant of nqs_eloc, for callers that
cannot allocate) through the C ABI, against nqs_eloc on the same inputs: two
calls in a row on the same device array, the second with fewer
configurations, for a fused (6x6 M = 72 FP32, 4x4 FP64) and a wide (10x10
M = 400 split BF16) model; then the size limit and an unsupported model,
both rejected before any launch."""
import ctypes as C
import dataclasses

import numpy as np
import pytest
import torch

from helpers import TOL, max_logpsi_err, max_rel_err
from workloads import WORKLOADS, draw_params, random_sz0_spins

pytestmark = pytest.mark.gpu


def _noalloc(m, sp, lp, el):
    from paper_2206_14307_amd.nqs import _ptr, _stream
    return m.lib.nqs_eloc_noalloc(m._ctx, _ptr(sp), sp.shape[0], _ptr(lp), _ptr(el), _stream())


@pytest.mark.parametrize("name", ["6x6_fp32_eloc", "4x4_fp64_exact", "10x10_m400"])
def test_noalloc_matches_eloc_on_consecutive_calls(name):
    from paper_2206_14307_amd import NQS
    w = WORKLOADS[name]
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    tol = TOL[w.precision]
    for S, seed in ((300, 1), (37, 2)):                 # the second call is smaller
        sp = torch.from_numpy(random_sz0_spins(w.N, S, seed)).cuda()
        lp_ref, el_ref = m.eloc(sp)
        lp = torch.full((S,), complex("nan"), dtype=torch.complex128, device="cuda")
        el = torch.full((S,), complex("nan"), dtype=torch.complex128, device="cuda")
        assert _noalloc(m, sp, lp, el) == 0, m.lib.nqs_last_error(m._ctx)
        torch.cuda.synchronize()
        assert max_logpsi_err(lp.cpu().numpy(), lp_ref.cpu().numpy()) < tol
        assert max_rel_err(el.cpu().numpy(), el_ref.cpu().numpy()) < tol
        # without log psi
        el2 = torch.empty_like(el)
        from paper_2206_14307_amd.nqs import _ptr, _stream
        assert m.lib.nqs_eloc_noalloc(m._ctx, _ptr(sp), S, None, _ptr(el2), _stream()) == 0
        assert max_rel_err(el2.cpu().numpy(), el_ref.cpu().numpy()) < tol


def test_noalloc_rejects_what_it_cannot_hold():
    from paper_2206_14307_amd import NQS
    from paper_2206_14307_amd.nqs import NQS_ERR_ARG, _ptr, _stream
    w = WORKLOADS["10x10_m400"]
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    sp = torch.from_numpy(random_sz0_spins(w.N, 1, 3)).cuda()
    el = torch.zeros(1, dtype=torch.complex128, device="cuda")
    # S beyond floor(2^26 / (24 N)) = 27962: rejected before anything is launched
    assert m.lib.nqs_eloc_noalloc(m._ctx, _ptr(sp), 27963, None, _ptr(el), _stream()) == NQS_ERR_ARG
    assert b"scratch" in m.lib.nqs_last_error(m._ctx)
    assert torch.count_nonzero(el).item() == 0
    # an FP64 model beyond the fused sizes has no fused / wide kernel
    w8 = dataclasses.replace(WORKLOADS["8x8_k4_m256"], precision="fp64", n_rbm=1, n_hidden=64)
    m8 = NQS.from_workload(w8)
    sp8 = torch.from_numpy(random_sz0_spins(w8.N, 2, 3)).cuda()
    el8 = torch.zeros(2, dtype=torch.complex128, device="cuda")
    assert m8.lib.nqs_eloc_noalloc(m8._ctx, _ptr(sp8), 2, None, _ptr(el8), _stream()) == NQS_ERR_ARG
    assert m.lib.nqs_eloc_noalloc(m._ctx, _ptr(sp), 0, None, None, _stream()) == 0
