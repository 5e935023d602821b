"""Writes the oracle's log psi and E_loc on 256 seeded configurations of the
8x8 (four RBMs, M = 256) and 10x10 (M = 400) workloads, so that the
benchmark can state the FP32-theta and split-BF16-theta errors of those
models on 256 checked rows without running the oracle for minutes inside the
timed job (the oracle needs several seconds per configuration at these sizes).
Calls only the oracle and the seeded input generators.

oracle_rows_<workload>.json: the workload's N(0, 0.01) parameters (they are
FP32-representable, so both theta precisions use the same values), the
configurations random_sz0_spins_fast(N, 256, 4004) (stored as the recipe plus
a SHA-256 of the int8 array, which the benchmark checks), log psi and E_loc.
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                                          # noqa: E402
from workloads import WORKLOADS, draw_params, random_sz0_spins_fast    # noqa: E402

N_ROWS, SEED = 256, 4004


def spins_of(name):
    w = WORKLOADS[name]
    return random_sz0_spins_fast(w.N, N_ROWS, SEED)


def one(task):
    name, lo, hi = task
    from threadpoolctl import threadpool_limits
    w = WORKLOADS[name]
    om = oracle.Model.from_workload(w)
    p = draw_params(w)
    sp = spins_of(name)[lo:hi]
    with threadpool_limits(1):
        return oracle.logpsi(om, p, sp), oracle.eloc_direct(om, p, sp)


def write(name, procs):
    sp = spins_of(name)
    step = max(1, N_ROWS // (4 * procs))
    tasks = [(name, lo, min(N_ROWS, lo + step)) for lo in range(0, N_ROWS, step)]
    with mp.get_context("fork").Pool(procs) as pool:
        out = pool.map(one, tasks)
    lp = np.concatenate([o[0] for o in out])
    el = np.concatenate([o[1] for o in out])
    doc = {"description": f"oracle log psi and E_loc of the {name} workload (its N(0, 0.01) "
                          f"parameters) on random_sz0_spins_fast(N, {N_ROWS}, {SEED}); written "
                          "by make_oracle_rows.py from the oracle",
           "workload": name, "rows": N_ROWS, "seed": SEED,
           "spins_sha256": hashlib.sha256(np.ascontiguousarray(sp).tobytes()).hexdigest(),
           "logpsi": [[z.real, z.imag] for z in lp], "eloc": [[z.real, z.imag] for z in el]}
    with open(os.path.join(HERE, f"oracle_rows_{name}.json"), "w") as f:
        json.dump(doc, f)


def main(names=("8x8_k4_m256", "10x10_m400")):
    procs = len(os.sched_getaffinity(0))
    for name in names:
        write(name, procs)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("8x8_k4_m256", "10x10_m400"))
