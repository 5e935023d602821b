"""Variational Monte-Carlo training by stochastic reconfiguration (Sec. 3.2,
Eq. (12); the training procedure of Sec. 3.4).

Every numerical step runs in the library: configurations come from
nqs_sample (exchange Metropolis chains that persist across steps), and each
training step is one nqs_vmc_step call (E_loc, their FP64 statistics, O_k,
the sample-space SR solve and the update theta <- theta + dtheta).  This
module is the host-side control around it, following Sec. 3.4:

* N_skip = 5 / r, r the acceptance rate of the previous training step
  (the first step measures r during a burn-in of n_burn proposals);
* the learning rate dtau is halved once the variational energy stops
  decreasing.  Reading of "not decreasing": the mean energy of the latest
  window of `window` steps is not below the mean of the window before it
  (windows do not overlap); dtau is not halved below `dtau_min`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch


def nskip_from_acceptance(r: float, cap: int = 1000) -> int:
    """N_skip = 5 / r proposals between kept samples (Sec. 3.4), at least 1."""
    if not (r > 0.0):
        return cap
    return int(min(cap, max(1, math.ceil(5.0 / r))))


@dataclass
class DtauSchedule:
    """dtau, halved when a window's mean energy is not below the previous one's."""
    dtau: float
    window: int = 10
    dtau_min: float = 5e-4
    _energies: list = field(default_factory=list)
    _prev_mean: float | None = None

    def update(self, energy: float) -> float:
        self._energies.append(float(energy))
        if len(self._energies) % self.window == 0:
            mean = sum(self._energies[-self.window:]) / self.window
            if self._prev_mean is not None and not (mean < self._prev_mean):
                self.dtau = max(self.dtau_min, 0.5 * self.dtau)
            self._prev_mean = mean
        return self.dtau


def train(model, init_spins, steps, n_per_chain, dtau=0.02, lam=1e-6, seed=0, n_burn=None,
          real_params=False, window=10, dtau_min=5e-4, solver="cholesky", callback=None):
    """Run `steps` SR steps with len(init_spins) chains and n_per_chain
    samples per chain and step.  Returns the per-step records (energy
    statistics before each update, N_skip, acceptance, dtau)."""
    state = model.chain_init(init_spins)
    if n_burn is None:
        n_burn = 20 * model.N
    sched = DtauSchedule(dtau, window, dtau_min)
    nskip, history = 0, []
    for step in range(steps):
        sp, acc, ns = model.sample(state, n_per_chain, n_skip=nskip,
                                   n_burn=n_burn if step == 0 else 0, seed=seed)
        used = int(ns.item()) if nskip == 0 else nskip
        r = float(acc.cpu().double().mean())
        stats = model.vmc_step(sp, lam=lam, dtau=sched.dtau, real_params=real_params,
                               solver=solver)
        rec = dict(stats, step=step, n_skip=used, acceptance=r, dtau=sched.dtau)
        history.append(rec)
        if callback is not None:
            callback(rec)
        nskip = nskip_from_acceptance(r)
        sched.update(stats["energy"])
    return history
