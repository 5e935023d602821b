"""Exchange Metropolis sampling of |psi|^2 (Sec. 3.2; schedule of Sec. 3.4).

Test infrastructure (see the package docstring).

The paper samples by exchanging randomly chosen anti-aligned spin pairs and
accepting with |psi(new)|^2 / |psi(old)|^2.  Readings where it is silent:
* proposal n of chain c draws (r0, r1, r2, r3) = Philox4x64-10 with counter
  (n, 0, 0, 0) and key (seed, c); the up site is the k-th up spin in
  ascending site order with k = floor(U(r0) * N/2), the down site likewise
  from r1, and the move is accepted iff U(r2) < |psi'/psi|^2, where
  U(r) = (r >> 11) / 2^53 (the index draws use exact integer arithmetic).
  The pair is global, not restricted to bonds; the proposal is symmetric.
* N_skip counts proposals between kept samples; N_skip = 5/r is taken as
  max(1, ceil(5 P / A)) from the A accepted of P burn-in proposals over all
  chains (exact integer arithmetic), capped at ``NSKIP_MAX``.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x64_10, index_below, uniform53
from .wavefunction import logpsi

NSKIP_MAX = 1000


def auto_nskip(accepted, proposed):
    if accepted <= 0:
        return NSKIP_MAX
    return int(max(1, min(NSKIP_MAX, -(-5 * proposed // accepted))))


def propose(spins, n, seed, chain):
    """Apply proposal n of chain ``chain`` to spins (+-1 int array); returns
    (new spins, acceptance uniform)."""
    r0, r1, r2, _ = philox4x64_10((n, 0, 0, 0), (seed, chain))
    up = np.nonzero(spins > 0)[0]
    dn = np.nonzero(spins < 0)[0]
    i = up[index_below(r0, len(up))]
    j = dn[index_below(r1, len(dn))]
    new = spins.copy()
    new[i], new[j] = -1, 1
    return new, uniform53(r2)


def exchange_metropolis(model, params, init_spins, seed, n_per_chain, n_skip, n_burn,
                        counters=None, chain_ids=None, record=False):
    """Run every chain; returns (samples [C*n_per_chain, N], acc_rate [C],
    final spins [C, N], final counters [C], n_skip used, log of decisions).

    The decision log (if ``record``) holds, per proposal, the uniform u and
    the FP64 ratio, so a replay can locate near-ties."""
    init_spins = np.atleast_2d(np.asarray(init_spins, np.int8))
    C, N = init_spins.shape
    counters = np.zeros(C, np.int64) if counters is None else np.asarray(counters, np.int64).copy()
    chain_ids = np.arange(C) if chain_ids is None else np.asarray(chain_ids)
    state = init_spins.copy()
    lp = logpsi(model, params, state)
    log = [[] for _ in range(C)]

    def step(c):
        nonlocal lp
        new, u = propose(state[c], counters[c], seed, chain_ids[c])
        lpn = logpsi(model, params, new[None])[0]
        ratio = float(np.exp(2.0 * (lpn - lp[c]).real))
        acc = u < ratio
        if record:
            log[c].append((int(counters[c]), u, ratio, bool(acc)))
        counters[c] += 1
        if acc:
            state[c] = new
            lp[c] = lpn
        return acc

    burn_acc = 0
    for c in range(C):
        for _ in range(n_burn):
            burn_acc += step(c)
    if n_skip == 0:
        n_skip = auto_nskip(burn_acc, C * n_burn)
    samples = np.empty((C, n_per_chain, N), np.int8)
    acc = np.zeros(C)
    for c in range(C):
        a = 0
        for m in range(n_per_chain):
            for _ in range(n_skip):
                a += step(c)
            samples[c, m] = state[c]
        acc[c] = a / max(1, n_per_chain * n_skip)
    return samples.reshape(C * n_per_chain, N), acc, state, counters, n_skip, log
