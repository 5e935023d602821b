"""Pins for the oracle's Philox generator and exchange Metropolis sampler.

* Philox4x64-10 equals the known-answer vector of its authors for counter 0,
  key 0, and numpy's independent implementation (whose first block uses
  counter 1) over many counters and keys;
* the sampler conserves Sz, and the distribution of a binned observable
  matches the exact |psi|^2 of the whole 4x4 sector (chi-square test);
* auto N_skip follows 5/r in exact integer arithmetic.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle.philox import index_below
from oracle.sampler import auto_nskip


def test_philox_known_answer():
    got = O.philox4x64_10((0, 0, 0, 0), (0, 0))
    assert got == (0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B)


@pytest.mark.parametrize("key", [(0, 0), (12345, 7), (2**64 - 1, 2**63 + 5)])
def test_philox_matches_numpy(key):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64))
    raw = bg.random_raw(4 * 50).reshape(50, 4)
    for n in range(50):
        assert O.philox4x64_10((n + 1, 0, 0, 0), key) == tuple(int(v) for v in raw[n])


def test_index_below_is_floor_of_uniform_times_n():
    rng = np.random.default_rng(0)
    for r in rng.integers(0, 2**63, 200, dtype=np.int64):
        r = int(r) * 2 + 1
        for n in (1, 8, 18, 50):
            k = index_below(r, n)
            assert 0 <= k < n
            assert k == int((r >> 11) * n // (1 << 53))


def test_auto_nskip():
    assert auto_nskip(100, 100) == 5
    assert auto_nskip(10, 100) == 50
    assert auto_nskip(3, 100) == 167
    assert auto_nskip(0, 100) == O.sampler.NSKIP_MAX


@pytest.mark.slow
def test_sampler_reproduces_exact_distribution():
    m = O.Model(L=4, J2=0.5, n_hidden=4)
    rng = np.random.default_rng(1)
    n = m.params_per_rbm
    p = (rng.normal(0, 0.25, n) + 1j * rng.normal(0, 0.25, n)).reshape(1, -1)
    masks, spins = O.sector_basis(16)
    lp = O.logpsi(m, p, spins)
    prob = np.exp(2 * (lp.real - lp.real.max()))
    prob /= prob.sum()
    # observable: the diagonal energy, binned by value
    diag = O.diag_energy(m, spins)
    init = spins[rng.choice(len(spins), 6)]
    samples, acc, final, ctr, nskip, _ = O.exchange_metropolis(
        m, p, init, seed=77, n_per_chain=400, n_skip=4, n_burn=50)
    assert (samples.sum(axis=1) == 0).all()
    assert (ctr == 50 + 400 * 4).all()
    vals = np.unique(np.round(diag, 9))
    exp_p = np.array([prob[np.isclose(diag, v)].sum() for v in vals])
    sd = O.diag_energy(m, samples)
    obs = np.array([np.isclose(sd, v).sum() for v in vals])
    keep = exp_p * len(samples) >= 5
    f_exp, f_obs = exp_p[keep] * len(samples), obs[keep]
    if (~keep).any():                                   # pool the rare bins
        f_exp = np.append(f_exp, exp_p[~keep].sum() * len(samples))
        f_obs = np.append(f_obs, obs[~keep].sum())
    # samples are correlated (N_skip = 4): use a conservative threshold
    chi2 = ((f_obs - f_exp) ** 2 / f_exp).sum()
    assert chi2 < stats.chi2.ppf(0.9999, len(f_obs) - 1) * 3
