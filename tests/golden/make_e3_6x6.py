"""Writes the oracle's e1, e2, e3 = (H^k psi)/psi (k = 1, 2, 3) on striped 6x6
configurations for the p = 2 Lanczos parity tests (the oracle needs one to
three minutes per configuration, too long inside a GPU test).  Calls only the
oracle and the seeded input generators.

e3_6x6_striped.json: the 6x6 J1-J2 (J2 = 0.5) projected RBM, K = (0, 0), A1,
one RBM with 8 hidden units, FP32-representable complex parameters of std
0.05 (seed 4); rows 0-2 up and rows 3-5 down, and its transpose (columns).
e3_6x6_m72_striped.json: the 6x6 Lanczos workload's model (72 hidden units,
its N(0, 0.01) parameters), the first of those configurations.
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
from workloads import WORKLOADS, draw_params    # noqa: E402


def workload():
    return dataclasses.replace(WORKLOADS["6x6_fp32_lanczos"], n_hidden=8)


def configs():
    a = np.where(np.arange(36) < 18, 1, -1).astype(np.int8)          # site i = x + 6 y
    b = np.where(np.arange(36) % 6 < 3, 1, -1).astype(np.int8)
    return np.stack([a, b])


def write(name, w, p, sp, doc):
    om = oracle.Model.from_workload(w)
    out = {
        "description": doc,
        "spins": sp.tolist(),
        "logpsi": [[z.real, z.imag] for z in oracle.logpsi(om, p, sp)],
        "e1": [[z.real, z.imag] for z in oracle.eloc_direct(om, p, sp)],
        "e2": [[z.real, z.imag] for z in oracle.e2_direct(om, p, sp)],
        "e3": [[z.real, z.imag] for z in oracle.e3_direct(om, p, sp)],
    }
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)


def main(which=("m8", "m72")):
    if "m8" in which:
        w = workload()
        write("e3_6x6_striped.json", w, stress_params(w, 0.05, 4), configs(),
              "6x6, 8 hidden units, std-0.05 complex parameters (seed 4); two striped "
              "configurations.  Written by make_e3_6x6.py from the oracle.")
    if "m72" in which:
        w = WORKLOADS["6x6_fp32_lanczos"]
        write("e3_6x6_m72_striped.json", w, draw_params(w), configs()[:1],
              "6x6 Lanczos workload model (72 hidden units, its N(0, 0.01) parameters); "
              "rows 0-2 up.  Written by make_e3_6x6.py from the oracle.")


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("m8", "m72"))
