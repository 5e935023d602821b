"""Writes e3_6x6_striped.json: e1, e2, e3 = (H^k psi)/psi (k = 1, 2, 3) of the
oracle on two striped 6x6 configurations, for the p = 2 Lanczos parity test
(the oracle needs about a minute per configuration, too long inside a GPU
test).  Calls only the oracle and the seeded input generators.

Model: the 6x6 J1-J2 (J2 = 0.5) projected RBM, K = (0, 0), A1, one RBM with
8 hidden units, FP32-representable complex parameters of std 0.05 (seed 4).
Configurations: rows 0-2 up and rows 3-5 down, and its transpose (columns).
"""
import dataclasses
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle                                   # noqa: E402
from helpers import stress_params               # noqa: E402
from workloads import WORKLOADS                 # noqa: E402


def workload():
    return dataclasses.replace(WORKLOADS["6x6_fp32_lanczos"], n_hidden=8)


def configs():
    a = np.where(np.arange(36) < 18, 1, -1).astype(np.int8)          # site i = x + 6 y
    b = np.where(np.arange(36) % 6 < 3, 1, -1).astype(np.int8)
    return np.stack([a, b])


def main():
    w = workload()
    p = stress_params(w, 0.05, 4)
    om = oracle.Model.from_workload(w)
    sp = configs()
    out = {
        "description": __doc__.strip(),
        "spins": sp.tolist(),
        "logpsi": [[z.real, z.imag] for z in oracle.logpsi(om, p, sp)],
        "e1": [[z.real, z.imag] for z in oracle.eloc_direct(om, p, sp)],
        "e2": [[z.real, z.imag] for z in oracle.e2_direct(om, p, sp)],
        "e3": [[z.real, z.imag] for z in oracle.e3_direct(om, p, sp)],
    }
    with open(os.path.join(HERE, "e3_6x6_striped.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
