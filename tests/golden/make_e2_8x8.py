"""Writes the oracle's log psi, e1 = E_loc and e2 = (H^2 psi)/psi for the 8x8
linear combination of four RBMs (M = 256 each), for the Lanczos-moment
parity tests of that model (the oracle's direct double sum re-evaluates
psi at ~17 000 configurations per row, about ten minutes each: too long
inside a GPU test).  Calls only the oracle and the seeded input generators.

e2_8x8_k4_m256.json holds three rows:
* rows 0, 1: the 8x8 K = 4 workload's N(0, 0.01) parameters (FP32-representable,
  so they serve the FP32 and the split-BF16 theta models alike) on the first two
  configurations of random_sz0_spins(64, 2, 21);
* row 2: the same model shape with std-0.05 complex parameters
  (stress_params(w, 0.05, 8)) on random_sz0_spins(64, 1, 22), where the
  exchange ratios depart further from 1.
Each row records which parameter set it uses ("params": "workload" or
"stress_0.05_seed8").
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle                                                       # noqa: E402
from helpers import stress_params                                   # noqa: E402
from workloads import WORKLOADS, draw_params, random_sz0_spins      # noqa: E402

NAME = "8x8_k4_m256"


def rows():
    w = WORKLOADS[NAME]
    a = random_sz0_spins(w.N, 2, 21)
    b = random_sz0_spins(w.N, 1, 22)
    return [("workload", a[0]), ("workload", a[1]), ("stress_0.05_seed8", b[0])]


def params_of(tag):
    w = WORKLOADS[NAME]
    return draw_params(w) if tag == "workload" else stress_params(w, 0.05, 8)


def one(task):
    tag, s = task
    from threadpoolctl import threadpool_limits
    om = oracle.Model.from_workload(WORKLOADS[NAME])
    p = params_of(tag)
    sp = s[None, :]
    with threadpool_limits(2):
        lp = oracle.logpsi(om, p, sp)[0]
        e1 = oracle.eloc_direct(om, p, sp)[0]
        e2 = oracle.e2_direct(om, p, sp)[0]
    return {"params": tag, "spins": s.tolist(), "logpsi": [lp.real, lp.imag],
            "e1": [e1.real, e1.imag], "e2": [e2.real, e2.imag]}


def main():
    tasks = rows()
    with mp.get_context("fork").Pool(len(tasks)) as pool:
        out = pool.map(one, tasks)
    doc = {"description": "8x8 J1-J2 (J2 = 0.5), K = (0,0), A1, four RBMs of 256 hidden units "
                          "with biases; oracle log psi, e1, e2 per row.  Written by "
                          "make_e2_8x8.py from the oracle.",
           "rows": out}
    with open(os.path.join(HERE, "e2_8x8_k4_m256.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
