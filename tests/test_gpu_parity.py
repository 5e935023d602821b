"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case compares element by element on the same seeded inputs: the full
4x4 Sz = 0 sector in FP64 (exact mode), seeded 6x6 / 8x8 / 10x10 subsets in
FP32 and split-BF16, stress parameters (std 0.3, complex, B1 and K = (pi,pi))
and ragged / degenerate sizes.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from helpers import (TOL, eloc_error_scale, grad_error_scale, max_logpsi_err, max_rel_err,
                     max_row_rel_err, max_scaled_eloc_err, max_scaled_row_err, nonzero_rows,
                     reciprocal_form_in_range, stress_params)
from workloads import WORKLOADS, draw_params, random_sz0_spins

pytestmark = pytest.mark.gpu


def make(w, params, direct=False):
    from paper_2206_14307_amd import NQS
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(params.reshape(-1)))
    m.set_factor_form(direct)          # direct: the plain product forms of the factors
    return m


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def sector16():
    return oracle.sector_basis(16)


# ------------------------------------------------------------------ 4x4 FP64

@pytest.fixture(scope="module")
def c1_case(sector16):
    w = WORKLOADS["4x4_fp64_exact"]
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    masks, spins = sector16
    lp = oracle.logpsi(om, p, spins)
    psi = np.exp(lp - lp.real.max())
    H = oracle.hamiltonian_sector(om, masks)
    e1 = (H @ psi) / psi
    e2 = (H @ (H @ psi)) / psi
    return w, p, om, spins, lp, e1, e2


def test_logpsi_full_sector_fp64(c1_case):
    w, p, om, spins, lp, e1, e2 = c1_case
    m = make(w, p)
    got = m.logpsi(cuda(spins)).cpu().numpy()
    assert max_logpsi_err(got, lp) < TOL["fp64"]


def test_eloc_full_sector_fp64(c1_case):
    w, p, om, spins, lp, e1, e2 = c1_case
    m = make(w, p)
    glp, gel = m.eloc(cuda(spins))
    assert max_logpsi_err(glp.cpu().numpy(), lp) < TOL["fp64"]
    assert max_rel_err(gel.cpu().numpy(), e1) < TOL["fp64"]


@pytest.mark.parametrize("direct", [False, True])
def test_exact_moments_fp64(c1_case, direct):
    w, p, om, spins, lp, e1, e2 = c1_case
    m = make(w, p, direct)
    res, e12 = m.lanczos_moments(cuda(spins), exact=True)
    e12 = e12.cpu().numpy()
    assert max_rel_err(e12[:, 0], e1) < TOL["fp64"]
    assert max_rel_err(e12[:, 1], e2) < TOL["fp64"]
    ref = oracle.moments(e1, e2, weights=np.abs(np.exp(lp - lp.real.max())) ** 2)
    assert res["n"] == len(spins)
    for key in ("h1", "h2", "h2_alt", "h3"):
        assert abs(res[key] - ref[key]) <= TOL["fp64"] * abs(ref[key]), key
    assert abs(res["e_p1"] - ref["e_p1"]) <= TOL["fp64"] * abs(ref["h1"])
    # c2 ~ 2e-7 h1^2 here: compare on the scale of h2, the raw second moment
    assert abs(res["c2"] - ref["c2"]) <= TOL["fp64"] * ref["h2"]


def test_grad_fp64(c1_case):
    w, p, om, spins, lp, e1, e2 = c1_case
    idx = np.random.default_rng(0).choice(len(spins), 48, replace=False)
    m = make(w, p)
    O = m.grad(cuda(spins[idx])).cpu().numpy()
    ref = oracle.logderiv(om, p, spins[idx])
    assert max_row_rel_err(O, ref) < TOL["fp64"]


@pytest.mark.parametrize("irrep,k", [("A1", 0), ("B1", 0), ("A1", 2), ("B2", 2)])
def test_stress_fp64(irrep, k, sector16):
    w = dataclasses.replace(WORKLOADS["4x4_fp64_exact"], irrep=irrep, kx=k, ky=k, n_rbm=2,
                            n_hidden=8, is_complex=True)
    p = stress_params(w, 0.3, 5)
    om = oracle.Model.from_workload(w)
    _, spins = sector16
    sp = spins[np.random.default_rng(1).choice(len(spins), 200, replace=False)]
    keep = nonzero_rows(om, p, sp)
    sp = sp[keep][:60]
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    assert max_logpsi_err(glp.cpu().numpy(), oracle.logpsi(om, p, sp)) < TOL["fp64"]
    # std-0.3 parameters: the exchange terms and image sums cancel, so the
    # errors are gated against the size of the terms (helpers' error model)
    kE = eloc_error_scale(om, p, sp)
    assert max_scaled_eloc_err(gel.cpu().numpy(), oracle.eloc_direct(om, p, sp), kE) < TOL["fp64"]
    O = m.grad(cuda(sp[:12])).cpu().numpy()
    kO = grad_error_scale(om, p, sp[:12])
    assert max_scaled_row_err(O, oracle.logderiv(om, p, sp[:12]), kO) < TOL["fp64"]


# ------------------------------------------------------------------ 6x6 FP32

@pytest.fixture(scope="module")
def c2_case():
    w = WORKLOADS["6x6_fp32_eloc"]
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    spins = random_sz0_spins(w.N, 37, 2002)             # ragged: not a tile multiple
    return w, p, om, spins


@pytest.mark.parametrize("direct", [False, True])
def test_logpsi_eloc_fp32(c2_case, direct):
    w, p, om, spins = c2_case
    m = make(w, p, direct)
    glp, gel = m.eloc(cuda(spins))
    assert max_logpsi_err(glp.cpu().numpy(), oracle.logpsi(om, p, spins)) < TOL["fp32"]
    assert max_rel_err(gel.cpu().numpy(), oracle.eloc_direct(om, p, spins)) < TOL["fp32"]
    lp_only = m.logpsi(cuda(spins)).cpu().numpy()      # separate (unfused) kernel path
    assert max_logpsi_err(lp_only, oracle.logpsi(om, p, spins)) < TOL["fp32"]


def test_grad_fp32(c2_case):
    w, p, om, spins = c2_case
    m = make(w, p)
    O = m.grad(cuda(spins[:9])).cpu().numpy()
    assert max_row_rel_err(O, oracle.logderiv(om, p, spins[:9])) < TOL["fp32"]


def test_stress_fp32_b1_pi():
    w = dataclasses.replace(WORKLOADS["6x6_fp32_eloc"], irrep="B1", kx=3, ky=3, n_rbm=2,
                            n_hidden=16)
    p = stress_params(w, 0.3, 9)
    om = oracle.Model.from_workload(w)
    sp = random_sz0_spins(w.N, 24, 3)
    sp = sp[nonzero_rows(om, p, sp)][:12]
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    assert max_logpsi_err(glp.cpu().numpy(), oracle.logpsi(om, p, sp)) < TOL["fp32"]
    kE = eloc_error_scale(om, p, sp)
    assert max_scaled_eloc_err(gel.cpu().numpy(), oracle.eloc_direct(om, p, sp), kE) < TOL["fp32"]
    O = m.grad(cuda(sp)).cpu().numpy()
    kO = grad_error_scale(om, p, sp)
    assert max_scaled_row_err(O, oracle.logderiv(om, p, sp), kO) < TOL["fp32"]


@pytest.mark.parametrize("direct", [False, True])
def test_twohop_fp32(direct):
    w = WORKLOADS["6x6_fp32_lanczos"]
    p = stress_params(w, 0.05, 4)
    om = oracle.Model.from_workload(w)
    sp = random_sz0_spins(w.N, 2, 11)
    m = make(w, p, direct)
    res, e12 = m.lanczos_moments(cuda(sp), exact=False)
    e12 = e12.cpu().numpy()
    e1 = oracle.eloc_direct(om, p, sp)
    e2 = oracle.e2_direct(om, p, sp)
    assert max_rel_err(e12[:, 0], e1) < TOL["fp32"]
    assert max_rel_err(e12[:, 1], e2) < TOL["fp32"]
    ref = oracle.moments(e1, e2)
    assert abs(res["h1"] - ref["h1"]) < TOL["fp32"] * abs(ref["h1"])
    assert abs(res["e_p1"] - ref["e_p1"]) < TOL["fp32"] * abs(ref["h1"])


@pytest.mark.parametrize("direct", [False, True])
def test_twohop_fp32_4x4_exact_mode(sector16, direct):
    w = dataclasses.replace(WORKLOADS["4x4_fp64_exact"], precision="fp32", is_complex=True,
                            n_hidden=16)
    p = stress_params(w, 0.1, 6)
    om = oracle.Model.from_workload(w)
    masks, spins = sector16
    lp = oracle.logpsi(om, p, spins)
    psi = np.exp(lp - lp.real.max())
    H = oracle.hamiltonian_sector(om, masks)
    e1 = (H @ psi) / psi
    e2 = (H @ (H @ psi)) / psi
    m = make(w, p, direct)
    res, e12 = m.lanczos_moments(cuda(spins), exact=True)
    e12 = e12.cpu().numpy()
    assert max_rel_err(e12[:, 0], e1) < TOL["fp32"]
    assert max_rel_err(e12[:, 1], e2) < TOL["fp32"]
    ref = oracle.moments(e1, e2, weights=np.abs(psi) ** 2)
    assert abs(res["e_p1"] - ref["e_p1"]) < TOL["fp32"] * abs(ref["h1"])
    assert abs(res["h2"] - ref["h2"]) < TOL["fp32"] * ref["h2"]


# ------------------------------------------------------- split BF16, 8x8, 10x10

@pytest.mark.parametrize("name", ["6x6_fp32_eloc", "8x8_k4_m256", "10x10_m400"])
@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
def test_larger_lattices(name, prec):
    w = dataclasses.replace(WORKLOADS[name], precision=prec)
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    sp = random_sz0_spins(w.N, 3, 5)
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    lref = oracle.logpsi(om, p, sp)
    assert max_logpsi_err(glp.cpu().numpy(), lref) < TOL[prec]
    assert max_rel_err(gel.cpu().numpy(), oracle.eloc_direct(om, p, sp)) < TOL[prec]
    # nqs_logpsi alone: the theta kernel (FP32 models: site-grouped three-term
    # BF16 theta) and the log-sum-exp over the images
    assert max_logpsi_err(m.logpsi(cuda(sp)).cpu().numpy(), lref) < TOL[prec]


# ----------------------------------------------------------- sizes and edges

def test_empty_and_single(c2_case):
    w, p, om, spins = c2_case
    m = make(w, p)
    assert m.logpsi(cuda(spins[:0])).numel() == 0
    lp, el = m.eloc(cuda(spins[:1]))
    assert max_rel_err(el.cpu().numpy(), oracle.eloc_direct(om, p, spins[:1])) < TOL["fp32"]


def test_zero_params_closed_form():
    w = WORKLOADS["6x6_fp32_eloc"]
    p = np.zeros((1, w.params_per_rbm), np.complex128)
    m = make(w, p)
    sp = random_sz0_spins(w.N, 50, 1)
    el = m.eloc(cuda(sp), want_logpsi=False).cpu().numpy()
    assert np.abs(el - w.N * (w.J1 + w.J2) / 2).max() < 1e-5


def test_symmetry_invariance_at_full_size():
    """E_loc(g sigma) = E_loc(sigma) and psi(g sigma) = chi(g) psi(sigma) hold at
    any size, checked on the 262144-configuration launch."""
    w = WORKLOADS["6x6_fp32_eloc"]
    p = draw_params(w)
    om = oracle.Model.from_workload(w)
    S = w.n_chains * w.n_per_chain
    sp = cuda(np.random.default_rng(0).permuted(
        np.tile(np.r_[np.ones(18, np.int8), -np.ones(18, np.int8)], (S, 1)), axis=1))
    m = make(w, p)
    lp, el = m.eloc(sp)
    h = 8 * 7 + 5
    perm = torch.from_numpy(om.lat.perms[h]).cuda()
    lp2, el2 = m.eloc(sp[:, perm])
    assert max_rel_err(el2.cpu().numpy(), el.cpu().numpy()) < 1e-5
    assert max_logpsi_err(lp2.cpu().numpy(), lp.cpu().numpy()) < 1e-5
    rows = np.random.default_rng(1).choice(S, 6, replace=False)
    spn = sp[rows].cpu().numpy()
    assert max_rel_err(el.cpu().numpy()[rows], oracle.eloc_direct(om, p, spn)) < TOL["fp32"]


# ------------------------------------------- both forms of the exchange factor

def _flat_column(p, w, h):
    """hidden unit h of every RBM gets W_h,p equal over sites: tanh(D_h) = 0
    on every bond, so the reciprocal form is out of range"""
    q = p.copy().reshape(w.n_rbm, -1)
    for k in range(w.n_rbm):
        q[k, h * w.N:(h + 1) * w.N] = q[k, h * w.N]
    return q


@pytest.mark.parametrize("case", ["drawn", "std1e-3", "std1e-4", "flat_column"])
@pytest.mark.parametrize("name", ["4x4_fp64_exact", "6x6_fp32_eloc"])
def test_eloc_both_factor_forms(name, case):
    """The fused kernel takes the exchange factors as s + t T (direct) or as
    T (t + s / T) (reciprocal, when every partial product stays in range);
    both agree with the oracle, including parameters close to the range limit
    (std 1e-3: suffix products near 2^-80 at M = 72) and just past it."""
    w = WORKLOADS[name]
    om = oracle.Model.from_workload(w)
    if case == "drawn":
        p = draw_params(w)
    elif case == "flat_column":
        p = _flat_column(draw_params(w), w, 3)
    else:
        p = stress_params(w, float(case[3:]), 12)
    expect = {"drawn": True, "std1e-3": True, "std1e-4": w.n_hidden < 32, "flat_column": False}
    lg = 900.0 if w.precision == "fp64" else 96.0
    assert reciprocal_form_in_range(om, p, lg) == expect[case]
    sp = random_sz0_spins(w.N, 21, 5)
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    tol = TOL[w.precision]
    assert max_logpsi_err(glp.cpu().numpy(), oracle.logpsi(om, p, sp)) < tol
    assert max_rel_err(gel.cpu().numpy(), oracle.eloc_direct(om, p, sp)) < tol


@pytest.mark.parametrize("case", ["std2e-3", "flat_column"])
@pytest.mark.parametrize("name,over", [("8x8_k4_m256", {"precision": "fp32"}),
                                       ("10x10_m400", {})])
def test_wide_eloc_small_and_vanishing_exchange_factors(name, over, case):
    """The wide kernel's products s + t T at |T| ~ 3e-3 (std 2e-3: every chunk
    of 8 units multiplies factors within 1e-5 of s) and with one hidden unit
    whose W column is flat (T = 0 on every bond), against the oracle."""
    w = dataclasses.replace(WORKLOADS[name], **over)
    om = oracle.Model.from_workload(w)
    p = _flat_column(draw_params(w), w, 5) if case == "flat_column" else \
        stress_params(w, float(case[3:]), 12)
    sp = random_sz0_spins(w.N, 7, 5)
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    tol = TOL[w.precision]
    assert max_logpsi_err(glp.cpu().numpy(), oracle.logpsi(om, p, sp)) < tol
    assert max_rel_err(gel.cpu().numpy(), oracle.eloc_direct(om, p, sp)) < tol


# ----------------------------------------------- wide hidden layers (K*M > 128)

def _neel_and_stripe(L):
    x, y = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
    neel = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8).reshape(-1)
    stripe = np.where(x % 2 == 0, 1, -1).astype(np.int8).reshape(-1)
    return np.stack([neel, stripe])


@pytest.mark.parametrize("name,over,std", [
    ("8x8_k4_m256", {"precision": "fp32"}, None),
    ("10x10_m400", {}, None),
    ("6x6_fp32_eloc", {"n_hidden": 144, "irrep": "B1", "kx": 3, "ky": 3}, 0.1),
])
def test_wide_models_many_samples_and_bond_passes(name, over, std):
    """Models with K*M > 128 take the wide kernel: one workgroup per sample,
    hidden units in chunks, 18 bonds per lane and pass (16 at N = 36).  300 configurations
    (more than one per workgroup) with the Neel and stripe states first (2N and
    3N antiparallel bonds: several bond passes); rows checked one by one."""
    w = dataclasses.replace(WORKLOADS[name], **over)
    p = draw_params(w) if std is None else stress_params(w, std, 31)
    om = oracle.Model.from_workload(w)
    sp = np.concatenate([_neel_and_stripe(w.L), random_sz0_spins(w.N, 298, 12)])
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    rows = np.r_[0, 1, 299]                  # Neel, stripe, a later sample of a workgroup
    sub = sp[rows]
    keep = nonzero_rows(om, p, sub)
    rows, sub = rows[keep], sub[keep]
    tol = TOL[w.precision]
    assert max_logpsi_err(glp.cpu().numpy()[rows], oracle.logpsi(om, p, sub)) < tol
    assert max_rel_err(gel.cpu().numpy()[rows], oracle.eloc_direct(om, p, sub)) < tol


def _anti_count(om, s):
    """Antiparallel coupled bonds of configuration s."""
    b = om.lat.bonds[om.bond_J != 0]
    return int(np.sum(s[b[:, 0]] != s[b[:, 1]]))


def _with_anti_count(om, target, seed):
    """An Sz = 0 configuration with exactly `target` antiparallel coupled
    bonds: random exchanges of an up and a down spin from a random start, kept
    when they do not move the count away from the target."""
    rng = np.random.default_rng(seed)
    s = random_sz0_spins(om.N, 1, seed)[0].copy()
    n = _anti_count(om, s)
    for _ in range(50000):
        if n == target:
            return s
        i = rng.choice(np.flatnonzero(s > 0))
        j = rng.choice(np.flatnonzero(s < 0))
        s[i], s[j] = s[j], s[i]
        n2 = _anti_count(om, s)
        if abs(n2 - target) <= abs(n - target):
            n = n2
        else:
            s[i], s[j] = s[j], s[i]
    raise AssertionError(f"no configuration with {target} antiparallel bonds")


@pytest.mark.parametrize("name,over,std,counts", [
    ("8x8_k4_m256", {"precision": "fp32"}, None, (72, 74, 78, 144)),
    ("10x10_m400", {}, None, (216, 218, 222)),
    ("6x6_fp32_eloc", {"n_hidden": 144, "irrep": "B1", "kx": 3, "ky": 3}, 0.1, (64, 66, 70)),
])
def test_wide_models_bond_pass_boundaries(name, over, std, counts):
    """The wide kernel takes 4 x 18 bonds per pass at N >= 64 (4 x 16 at
    N = 36) and skips the empty slot pairs of a partly filled last pass with a
    bound taken from lane group 0 (bond i of a pass goes to lane group i mod 4).
    Configurations whose antiparallel-bond count fills the passes exactly, or
    carries 2, 4 or 6 bonds into a further pass (one more in some lane groups
    than in others), checked row by row against the oracle's direct E_loc.  The
    count is always even: every site has an even number of coupled bonds, and
    the antiparallel ones are the bonds between the down spins and the rest."""
    w = dataclasses.replace(WORKLOADS[name], **over)
    p = draw_params(w) if std is None else stress_params(w, std, 31)
    om = oracle.Model.from_workload(w)
    sub = np.stack([_with_anti_count(om, n, 40 + k) for k, n in enumerate(counts)])
    assert [_anti_count(om, s) for s in sub] == list(counts)
    sp = np.concatenate([sub, random_sz0_spins(w.N, 5, 13)])
    m = make(w, p)
    glp, gel = m.eloc(cuda(sp))
    rows = np.flatnonzero(nonzero_rows(om, p, sub))
    assert len(rows) >= len(counts) - 1
    tol = TOL[w.precision]
    assert max_logpsi_err(glp.cpu().numpy()[rows], oracle.logpsi(om, p, sub[rows])) < tol
    assert max_rel_err(gel.cpu().numpy()[rows], oracle.eloc_direct(om, p, sub[rows])) < tol


# ------------------------------------------------------------ Sz = 0 sector

def test_enumerate_sz0_matches_oracle_basis(sector16):
    """nqs_enumerate_sz0 is integer work: bit-exact against the oracle's
    increasing-mask (colex) basis of the 4x4 sector."""
    from paper_2206_14307_amd import NQS
    m = NQS.from_workload(WORKLOADS["4x4_fp64_exact"])
    assert m.sector_size() == 12870
    got = m.enumerate_sz0().cpu().numpy()
    assert np.array_equal(got, sector16[1])


def test_enumerate_sz0_limits():
    import ctypes as C
    from paper_2206_14307_amd import NQS, NQSError
    from paper_2206_14307_amd.nqs import _stream
    m4 = NQS.from_workload(WORKLOADS["4x4_fp64_exact"])
    buf = torch.empty((100, 16), dtype=torch.int8, device="cuda")
    n = C.c_int64(0)
    st = m4.lib.nqs_enumerate_sz0(m4._ctx, C.c_void_p(buf.data_ptr()), 100, C.byref(n), _stream())
    assert st == 1 and n.value == 12870                  # cap too small: NQS_ERR_ARG
    m6 = NQS.from_workload(WORKLOADS["6x6_fp32_eloc"])
    assert m6.sector_size() == 9075135300                # counted, too large to enumerate
    st = m6.lib.nqs_enumerate_sz0(m6._ctx, C.c_void_p(buf.data_ptr()), 1 << 40, C.byref(n),
                                  _stream())
    assert st == 1 and n.value == 9075135300
    m10 = NQS.from_workload(WORKLOADS["10x10_m400"])
    with pytest.raises(NQSError):                        # C(100, 50) overflows int64
        m10.sector_size()


# ------------------------------------------- two-hop terms at any lattice size

def _bonds_and_J(w):
    om = oracle.Model.from_workload(w)
    return om.lat.bonds, np.asarray(om.bond_J, dtype=np.float64)


@pytest.mark.parametrize("name,over", [
    ("6x6_fp32_lanczos", {}),
    ("8x8_k4_m256", {"precision": "fp32"}),
])
def test_twohop_composes_from_one_hop_calls(name, over):
    """e2(s) = diag(s) e1(s) + sum_b (J_b/2) psi(s^b)/psi(s) e1(s^b) holds at any
    size: the moments kernel's e2 is rebuilt from nqs_logpsi / nqs_eloc on the
    exchanged configurations (each of those oracle-checked elsewhere).  Covers
    the 8x8 K=4 M=256 model, whose direct oracle e2 is out of reach."""
    w = dataclasses.replace(WORKLOADS[name], **over)
    p = draw_params(w)
    bonds, J = _bonds_and_J(w)
    sp = random_sz0_spins(w.N, 2, 21)
    m = make(w, p)
    res, e12 = m.lanczos_moments(cuda(sp), exact=False)
    e12 = e12.cpu().numpy()
    for r in range(len(sp)):
        s = sp[r]
        anti = np.nonzero(s[bonds[:, 0]] != s[bonds[:, 1]])[0]
        nb = np.repeat(s[None, :], len(anti), axis=0)
        for k, b in enumerate(anti):
            i, j = bonds[b]
            nb[k, i], nb[k, j] = s[j], s[i]
        lp0 = m.logpsi(cuda(s[None, :])).cpu().numpy()[0]
        lpn, eln = m.eloc(cuda(nb))
        lpn, eln = lpn.cpu().numpy(), eln.cpu().numpy()
        diag = 0.25 * float((J * s[bonds[:, 0]] * s[bonds[:, 1]]).sum())
        e2 = diag * e12[r, 0] + (0.5 * J[anti] * np.exp(lpn - lp0) * eln).sum()
        assert abs(e12[r, 1] - e2) <= 1e-5 * max(1.0, abs(e2)), (r, e12[r, 1], e2)
