"""The error scales behind the tolerances of the stress cases (each is the
size of the terms of a sum, so the triangle inequality bounds the sum by it):
kappa_psi >= 1 with equality when the images do not cancel, kappa_E >= |E_loc|,
and the O row scale >= ||O||.  CPU only; the oracle supplies every value."""
import dataclasses

import numpy as np

import oracle
from helpers import eloc_error_scale, grad_error_scale, logpsi_error_scale, stress_params
from workloads import WORKLOADS, draw_params, random_sz0_spins


def _model(over, std):
    w = dataclasses.replace(WORKLOADS["4x4_fp64_exact"], **over)
    p = draw_params(w) if std is None else stress_params(w, std, 21)
    return oracle.Model.from_workload(w), p


def test_scales_bound_their_sums():
    om, p = _model({"is_complex": True, "irrep": "B1", "kx": 2, "ky": 2}, 0.3)
    sp = random_sz0_spins(om.N, 24, 5)
    kpsi = logpsi_error_scale(om, p, sp)
    assert (kpsi >= 1.0 - 1e-12).all()
    assert kpsi.max() > 1.5                       # the B1 images do cancel
    kE = eloc_error_scale(om, p, sp)
    assert (kE >= np.abs(oracle.eloc_direct(om, p, sp)) * (1 - 1e-12)).all()
    kO = grad_error_scale(om, p, sp)
    assert (kO >= np.linalg.norm(oracle.logderiv(om, p, sp), axis=1) * (1 - 1e-12)).all()


def test_no_cancellation_gives_unit_kappa():
    # real A1 RBM with small drawn weights: every image term is positive
    om, p = _model({}, None)
    sp = random_sz0_spins(om.N, 16, 6)
    np.testing.assert_allclose(logpsi_error_scale(om, p, sp), 1.0, rtol=1e-12)
