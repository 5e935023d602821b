#!/usr/bin/env python3
"""Benchmark: configs*sym-images/s for log psi + E_loc on one MI355X.

Workload (default): the 6x6 J1-J2 lattice (J2/J1 = 0.5), one complex RBM with
M = 72 (alpha = 2) in FP32, projected on the 288 space-group images,
4096 chains x 64 samples = 262144 configurations resident in HBM.  A step is
one nqs_eloc call (theta GEMM + log 2cosh/LSE epilogue + bond-exchange
products) over the whole batch; value = S * K * G / step time.

Printed as ONE JSON line, with
  roofline     -- the dominant kernel (eloc_bonds), achieved algorithmic
                  TFLOP/s (13 real flops per exchange factor) against the
                  FP32 vector peak, from HIP events recorded live around each
                  launch on the call's stream;
  cpu_baseline -- the FP64 oracle timed on this host's cores on a bounded
                  sample of the same configurations;
  errors       -- log psi / E_loc errors of the GPU path vs the oracle on the
                  CPU-baseline sample (the only leg that runs the oracle);
  legs         -- the other rows of the hot path (sampling, backward, log psi
                  alone, two-hop Lanczos moments, split-BF16 vs FP32 at 8x8,
                  SR at 10x10), timed, each with its roofline where one binds.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6          # MI355X published FP64 vector (and MFMA) peak
FLOPS_PER_FACTOR = 13             # P <- P (1 + t T): complex mul, +1, complex mul


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def n_antiparallel(spins, bonds):
    return (spins[:, bonds[:, 0]] != spins[:, bonds[:, 1]]).sum(axis=1)


COUNTER_JSON = os.path.join(ROOT, "profiles", "eloc_fused_6x6_m72_hbm_counters.json")
COUNTER_SOURCES = ["k_eloc_fused.hip", "fused_theta.h", "theta_common.h", "device_common.h",
                   "nqs_internal.h", "lds_layout.cpp"]


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2206_14307_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def write_counters(fetch_csv, write_csv, kernel="eloc_fused_kernel", copy_bytes=1 << 30):
    """Summarise two rocprofv3 --pmc runs of `bench.py --copy-probe` (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch) into the committed counter JSON: the
    kernel's mean per launch, scaled by what the counter reads for the 1 GiB
    device copy the same run makes."""
    import csv

    def per_kernel(path, counter):
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    kname = next(k for k in f if kernel in k)
    copy = next(k for k in f if "copyBuffer" in k)
    kib = copy_bytes / 1024.0
    cf, cw = max(f[copy]), max(w[copy])
    fk, wk = float(np.mean(f[kname])), float(np.mean(w[kname]))
    d = {
        "kernel": kname.replace("void ", "").replace("nqs::(anonymous namespace)::", "").split("(")[0],
        "workload": "6x6 M=72 FP32, 262144 configurations, one launch",
        "fetch_kib": fk, "write_kib": wk,
        "copy_probe_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": kib / cf, "write_scale": kib / cw,
        "traffic_bytes_per_launch": 1024.0 * (fk * kib / cf + wk * kib / cw),
        "kernel_source_sha256_16": source_hash(COUNTER_SOURCES),
        "kernel_sources": COUNTER_SOURCES,
    }
    with open(COUNTER_JSON, "w") as fh:
        json.dump(d, fh, indent=1)
    return d


def counted_traffic(path=COUNTER_JSON):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (copy-calibrated), or None when the kernel's
    sources have changed since the counters were taken."""
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if source_hash(d["kernel_sources"]) != d["kernel_source_sha256_16"]:
        return None
    return d["traffic_bytes_per_launch"]


# ------------------------------------------------------------- CPU baseline

def _oracle_chunk(args):
    name, params, spins = args
    from threadpoolctl import threadpool_limits
    import oracle
    from workloads import WORKLOADS
    om = oracle.Model.from_workload(WORKLOADS[name])
    with threadpool_limits(1):          # one BLAS thread per worker process
        lp = oracle.logpsi(om, params, spins)
        el = oracle.eloc_direct(om, params, spins)
    return lp, el


def cpu_baseline(name, params, spins, budget_s=20.0, extra=()):
    """Time the oracle's log psi + E_loc on a bounded sample on all host cores.
    Returns the baseline record and the oracle's outputs: for the timed sample
    (indices into spins, log psi, E_loc) and for each (name, params, spins) of
    `extra` (evaluated in the same pool), so the GPU path's errors can be
    stated against the oracle on the same configurations."""
    from workloads import WORKLOADS
    w = WORKLOADS[name]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    # calibrate on two configurations (after a warm-up), then size the sample to ~budget_s
    _oracle_chunk((name, params, spins[:1]))
    t0 = time.perf_counter()
    _oracle_chunk((name, params, spins[:2]))
    per = (time.perf_counter() - t0) / 2
    n = int(max(cores, min(len(spins), 0.7 * budget_s * cores / max(per, 1e-3))))
    n = max(cores, (n // cores) * cores)
    log(f"cpu baseline: {per * 1e3:.1f} ms per configuration on one core; "
        f"timing {n} configurations on {cores} worker processes")
    idx = [np.arange(len(spins))[i::cores][: n // cores] for i in range(cores)]
    chunks = [(name, params, spins[ix]) for ix in idx]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        outs = pool.map(_oracle_chunk, chunks)
    dt = time.perf_counter() - t0
    refs = {"idx": np.concatenate(idx), "logpsi": np.concatenate([o[0] for o in outs]),
            "eloc": np.concatenate([o[1] for o in outs]), "extra": []}
    if extra:
        tasks = [(n_, p_, sp_[i:i + 1]) for (n_, p_, sp_) in extra for i in range(len(sp_))]
        with ctx.Pool(min(cores, len(tasks))) as pool:
            res = pool.map(_oracle_chunk, tasks)
        k = 0
        for (_, _, sp_) in extra:
            part = res[k:k + len(sp_)]
            k += len(sp_)
            refs["extra"].append((np.concatenate([r[0] for r in part]),
                                  np.concatenate([r[1] for r in part])))
    return ({"value": n * w.n_rbm * w.G / dt, "unit": "configs*sym-images/s", "cores": cores,
             "kind": "oracle", "cpu": cpu_model(),
             "sample": f"{n} Sz = 0 configurations of the benchmark's size, FP64 NumPy log psi + "
                       f"E_loc by direct re-evaluation, {cores} worker processes, {dt:.1f} s"},
            refs)


def errors_of(lp_gpu, el_gpu, lp_ref, el_ref):
    """log psi / E_loc errors of GPU outputs against oracle outputs (same rows)."""
    d = lp_gpu - lp_ref
    d = d.real + 1j * np.angle(np.exp(1j * d.imag))
    return {"checked": int(len(lp_ref)),
            "max_abs_dlogpsi": float(np.abs(d).max()),
            "max_rel_deloc": float((np.abs(el_gpu - el_ref) / np.maximum(1, np.abs(el_ref))).max()),
            "rel_err_mean_eloc": float(abs(el_gpu.mean() - el_ref.mean()) / abs(el_ref.mean()))}


def square_bonds(L):
    """The 4N bonds of the L x L torus: (i, i+x), (i, i+y) (J1), (i, i+x+y), (i, i+x-y) (J2)."""
    out = []
    for dx, dy in ((1, 0), (0, 1), (1, 1), (1, -1)):
        for i in range(L * L):
            x, y = i % L, i // L
            out.append((i, (x + dx) % L + L * ((y + dy) % L)))
    return np.array(out, dtype=np.int64)


# ------------------------------------------------------------------- GPU legs

def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def twohop_hops(spins, bonds):
    """Exchange-factor products (per image and hidden unit) that e1 + e2 of a
    set of configurations evaluate: the n_c(s) first hops, and for each first
    hop b1 the second hops b2 antiparallel in s^{b1}, b2 != b1 (the exchange
    back is closed-form), bonds disjoint from b1 once per unordered pair."""
    NB = len(bonds)
    idx = np.arange(NB)
    shared = ((bonds[:, None, 0] == bonds[None, :, 0]) | (bonds[:, None, 0] == bonds[None, :, 1]) |
              (bonds[:, None, 1] == bonds[None, :, 0]) | (bonds[:, None, 1] == bonds[None, :, 1]))
    hops = 0
    for s0 in range(0, len(spins), 512):
        x = spins[s0:s0 + 512].astype(np.int16)
        anti = x[:, bonds[:, 0]] != x[:, bonds[:, 1]]
        hops += int(anti.sum())
        for b, (i, j) in enumerate(bonds):
            rows = np.nonzero(anti[:, b])[0]
            if rows.size:
                y = x[rows].copy()
                y[:, [i, j]] = -y[:, [i, j]]
                keep = (idx != b) & (shared[b] | (idx > b))
                hops += int(((y[:, bonds[:, 0]] != y[:, bonds[:, 1]]) & keep).sum())
    return hops


def neighbours(spins, bonds):
    """All exchange neighbours s^b (antiparallel bonds b) of the configurations."""
    out = []
    for i, j in bonds:
        rows = np.nonzero(spins[:, i] != spins[:, j])[0]
        y = spins[rows].copy()
        y[:, [i, j]] = y[:, [j, i]]
        out.append(y)
    return np.concatenate(out)


def leg_lanczos(steps=2):
    """Two-hop e2 + FP64 moments on the 6x6 Lanczos workload (8192 samples)."""
    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    w = WORKLOADS["6x6_fp32_lanczos"]
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    S = w.n_chains * w.n_per_chain
    sp = torch.from_numpy(random_sz0_spins_fast(w.N, S, 3003)).cuda()
    res = {}
    ms = timed(lambda: res.update(m.lanczos_moments(sp, exact=False, want_e1e2=False)[0]), steps, 1)
    # exact factor count: one-hop n_c(s) plus two-hop sum_{b1} n_c(s^{b1}), times G K M
    bonds = square_bonds(w.L)
    hops = twohop_hops(sp.cpu().numpy(), bonds)
    factors = float(hops) * w.G * w.n_rbm * w.n_hidden
    flops = 13.0 * factors
    out = {"workload": w.name, "S": S, "ms": ms,
           "configs_per_s": S / (ms / 1e3), "h1_per_site": res["h1"] / w.N,
           "e_p1_per_site": res["e_p1"] / w.N, "factors": factors,
           "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12, "peak": 157.3,
                        "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / 1e12 / 157.3,
                        "flops_per_factor": 13}}
    # the wide models' e2, on a small sample of their workloads
    out["wide_models"] = {}
    for name, Sw in (("8x8_k4_m256", 64), ("10x10_m400", 16)):
        ww = WORKLOADS[name]
        mw = NQS.from_workload(ww)
        mw.set_params(torch.from_numpy(draw_params(ww).reshape(-1)))
        spw = torch.from_numpy(random_sz0_spins_fast(ww.N, Sw, 3003)).cuda()
        msw = timed(lambda: mw.lanczos_moments(spw, exact=False, want_e1e2=False), 1, 1)
        # e2 from the exchange neighbours through the wide E_loc kernel, each
        # with its parent's unordered-pair bond list: the same factor products
        # as the two-hop kernels evaluate
        fw = float(twohop_hops(spw.cpu().numpy(), square_bonds(ww.L))) * ww.G * ww.n_rbm * ww.n_hidden
        out["wide_models"][name] = {"S": Sw, "ms": msw, "ms_per_config": msw / Sw, "factors": fw,
                                    "factors_per_s": fw / (msw / 1e3),
                                    "frac": 13.0 * fw / (msw / 1e3) / 1e12 / 157.3}
        del mw
    return out


def leg_lanczos2(S=256, steps=1):
    """p = 2 Lanczos (e1, e2, e3 + fifth-order moments + 3x3 Krylov solve) on
    the first S configurations of the 6x6 Lanczos workload's random set."""
    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    w = WORKLOADS["6x6_fp32_lanczos"]
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    spins = random_sz0_spins_fast(w.N, w.n_chains * w.n_per_chain, 3003)[:S]
    sp = torch.from_numpy(spins).cuda()
    res = {}
    ms = timed(lambda: res.update(m.lanczos_moments_p2(sp, exact=False, want_e123=False)[0]),
               steps, 1)
    # one more call with per-kernel events: where the time goes
    names = ("theta", "lse", "eloc_bonds", "eloc_finish", "twohop", "twohop_finish", "hop3")
    m.profile(True)
    for k in names:
        m.profile_read(k, reset=True)
    m.lanczos_moments_p2(sp, exact=False, want_e123=False)
    split = {k: round(m.profile_read(k, reset=True)[0], 3) for k in names}
    m.profile(False)
    bonds = square_bonds(w.L)
    nb = neighbours(spins, bonds)
    hops = twohop_hops(spins, bonds) + twohop_hops(nb, bonds)
    factors = float(hops) * w.G * w.n_rbm * w.n_hidden
    flops = 13.0 * factors
    return {"workload": w.name, "S": S, "neighbour_configs": int(len(nb)), "ms": ms,
            "configs_per_s": S / (ms / 1e3), "h1_per_site": res["h1"] / w.N,
            "e_p1_per_site": res["e_p1"] / w.N, "e_p2_per_site": res["e_p2"] / w.N,
            "degenerate": res["degenerate"], "factors": factors,
            "kernel_ms": split,
            "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12, "peak": 157.3,
                         "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / 1e12 / 157.3,
                         "flops_per_factor": 13}}


def leg_logpsi(m, sp, S, w, steps=3):
    """nqs_logpsi alone (theta GEMM + log 2cosh + LSE): 4N useful MFMA flops per
    complex theta; the log 2cosh epilogue runs on the VALU beside it."""
    import torch
    out = torch.empty(S, dtype=torch.complex128, device="cuda")
    ms = timed(lambda: out.copy_(m.logpsi(sp)), steps, 1)
    flops = 4.0 * w.N * S * w.G * w.n_rbm * w.n_hidden
    peak = {"fp64": 78.6, "fp32": 157.3, "bf16x2": 2500.0}[w.precision]
    # the dominant kernel's own launch time (library HIP events), as for the headline
    m.profile(True)
    for k in ("theta", "lse"):
        m.profile_read(k, reset=True)
    for _ in range(steps):
        m.logpsi(sp)
    kms = {k: m.profile_read(k, reset=True) for k in ("theta", "lse")}
    m.profile(False)
    t_ms = kms["theta"][0] / max(1, kms["theta"][1])
    return {"S": S, "ms": ms, "configs_sym_images_per_s": S * w.n_rbm * w.G / (ms / 1e3),
            "call_frac": flops / (ms / 1e3) / 1e12 / peak,
            "kernel_ms": {"theta": t_ms, "lse": kms["lse"][0] / max(1, kms["lse"][1])},
            "roofline": {"kernel": "theta_kernel", "bound": "mfma",
                         "achieved": flops / (t_ms / 1e3) / 1e12, "peak": peak,
                         "unit": "TFLOP/s", "frac": flops / (t_ms / 1e3) / 1e12 / peak,
                         "flops": flops}}


def leg_sq(m, sp, S, w, steps=5):
    """nqs_structure_factor over the benchmark's configurations (uniform
    weights): per configuration and momentum q, N real-times-complex FMAs
    (4 FP64 flops each) and |F(q)|^2; timed on the library's own events."""
    m.structure_factor(sp)
    import torch
    torch.cuda.synchronize()
    m.profile(True)
    m.profile_read("sq", reset=True)
    for _ in range(steps):
        m.structure_factor(sp)
    ms, n = m.profile_read("sq", reset=True)
    m.profile(False)
    ms /= max(n, 1)
    flops = (4.0 * w.N + 3.0) * w.N * S
    nbytes = S * (w.N + 8)
    return {"S": S, "ms": ms, "configs_per_s": S / (ms / 1e3),
            "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12,
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / (ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, "flops": flops,
                         "hbm_GBps": nbytes / (ms / 1e3) / 1e9}}


def leg_vmc(steps=3):
    """SR training at the paper's step size (10 000 samples per step, Sec. 3.4)
    on the 6x6 M = 72 FP32 model: time of nqs_sample (1000 chains x 10 samples,
    N_skip = 5/r from the previous step) and of nqs_vmc_step (E_loc, statistics,
    O_k, the 10 000 x 10 000 sample-space SR solve, update).  Then the 4x4
    complex M = 16 model trained for 200 steps of 2048 samples from
    N(0, 0.01): its exact energy against exact diagonalisation of the
    4 x 4 lattice is computed on the GPU over the whole Sz = 0 sector."""
    import dataclasses
    import torch
    from paper_2206_14307_amd import NQS
    from paper_2206_14307_amd.vmc import nskip_from_acceptance, train
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    w = WORKLOADS["6x6_fp32_eloc"]
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    state = m.chain_init(torch.from_numpy(random_sz0_spins_fast(w.N, 1000, 77)).cuda())
    nskip, t_s, t_v, t_c, rec, iters = 0, [], [], [], None, []
    for step in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp, acc, ns = m.sample(state, 10, n_skip=nskip, n_burn=20 * w.N if step == 0 else 0,
                               seed=77)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # the same step with both solvers of Eq. (12), from the same parameters
        p_before = m.get_params()
        rec = m.vmc_step(sp, lam=1e-6, dtau=0.01, solver="cholesky")
        t2 = time.perf_counter()
        m.set_params(p_before)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rc = m.vmc_step(sp, lam=1e-6, dtau=0.01, solver="cg")
        t4 = time.perf_counter()
        if step > 0:                                   # the first step carries the burn-in
            t_s.append(t1 - t0)
            t_v.append(t2 - t1)
            t_c.append(t4 - t3)
            iters.append(rc["solver_iters"])
        nskip = nskip_from_acceptance(float(acc.cpu().double().mean()))
    out = {"workload": "6x6_fp32_eloc", "samples_per_step": 10000, "n_skip": nskip,
           "ms_sample": 1e3 * sum(t_s) / len(t_s),
           "ms_vmc_step_cholesky": 1e3 * sum(t_v) / len(t_v),
           "ms_vmc_step_cg": 1e3 * sum(t_c) / len(t_c), "cg_iterations": iters,
           "energy_per_site": rec["energy"] / w.N}
    out["ms_per_training_step"] = out["ms_sample"] + min(out["ms_vmc_step_cholesky"],
                                                          out["ms_vmc_step_cg"])
    w4 = dataclasses.replace(WORKLOADS["4x4_fp64_exact"], is_complex=True, J2=0.0)
    m4 = NQS.from_workload(w4)
    m4.set_params(torch.from_numpy(draw_params(w4).reshape(-1)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(m4, torch.from_numpy(random_sz0_spins_fast(w4.N, 256, 3)).cuda(), steps=200,
                 n_per_chain=8, dtau=0.05)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res, _ = m4.lanczos_moments_p2(m4.enumerate_sz0(), exact=True, want_e123=False)
    e0 = -0.701780 * w4.N          # 4x4 Heisenberg ground state (exact diagonalisation, 6 digits)
    out["train_4x4_j2_0"] = {"steps": len(hist), "seconds": t_train,
                             "exact_energy": res["h1"], "e_p1": res["e_p1"], "e_p2": res["e_p2"],
                             "e0_ed_6_digits": e0,
                             "rel_err": abs(res["h1"] - e0) / abs(e0),
                             "rel_err_p1": abs(res["e_p1"] - e0) / abs(e0),
                             "e_p1_minus_e_p2": res["e_p1"] - res["e_p2"]}
    return out


def leg_grad(m, sp, S, G, K, steps=3):
    import torch
    O = torch.empty((S, m.P), dtype=m.o_dtype, device="cuda")
    ws = m.workspace("grad", S)
    import ctypes as C
    from paper_2206_14307_amd.nqs import _ptr, _stream

    def run():
        m._check(m.lib.nqs_grad(m._ctx, _ptr(sp), S, _ptr(O), None, _ptr(ws), ws.numel(),
                                _stream()), "nqs_grad")
    ms = timed(run, steps, 1)
    del O
    # algorithmic work: 8 N flops per (configuration, image, hidden unit),
    # theta recompute included, on MFMA; the O write on HBM
    N = int(sp.shape[1])
    flops = 8.0 * N * S * G * m.n_rbm * m.n_hidden
    o_bytes = S * m.P * (16 if m.precision == "fp64" else 8)
    peak = 78.6 if m.precision == "fp64" else 157.3
    return {"S": S, "ms": ms, "configs_sym_images_per_s": S * K * G / (ms / 1e3),
            "O_bytes": o_bytes,
            "roofline": {"bound": "mfma", "achieved": flops / (ms / 1e3) / 1e12, "peak": peak,
                         "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / 1e12 / peak,
                         "flops": flops, "hbm_GBps_O_write": o_bytes / (ms / 1e3) / 1e9}}


PRECISION_LEG_SEED = 4004


def precision_leg_refs(name):
    """(name, params, spins) of the two configurations whose oracle values the
    precision leg states its errors against (computed in the CPU-baseline leg)."""
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    w = WORKLOADS[name]
    S = w.n_chains * w.n_per_chain
    return (name, draw_params(w), random_sz0_spins_fast(w.N, S, PRECISION_LEG_SEED)[:2])


def leg_precision(name, refs=None, steps=2):
    """split-BF16 vs FP32 theta on the same spins (the workload's sample count),
    each with its errors against the oracle on two of them when the CPU-baseline
    leg computed those (refs = (log psi, E_loc))."""
    import dataclasses
    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    out = {}
    base = WORKLOADS[name]
    S = base.n_chains * base.n_per_chain
    spins = random_sz0_spins_fast(base.N, S, PRECISION_LEG_SEED)
    sp = torch.from_numpy(spins).cuda()
    for prec in ("fp32", "bf16x2"):
        w = dataclasses.replace(base, precision=prec)
        p = draw_params(w)
        m = NQS.from_workload(w)
        m.set_params(torch.from_numpy(p.reshape(-1)))
        holder = {}
        ms = timed(lambda: holder.update(r=m.eloc(sp)), steps, 1)
        lp, el = holder["r"]
        err = (errors_of(lp[:2].cpu().numpy(), el[:2].cpu().numpy(), *refs) if refs is not None
               else {"checked": 0})
        out[prec] = {"ms": ms, "configs_sym_images_per_s": S * w.n_rbm * w.G / (ms / 1e3), **err}
    out["workload"] = name
    out["S"] = S
    return out


def leg_sr(name="10x10_m400", S=32768, steps=1):
    """logpsi + E_loc + O_k for S configurations (the 10x10 workload's sample
    count), then the sample-space SR step; the Gram matrix and the Cholesky
    factorisation + solves are timed with the library's HIP events."""
    import ctypes as C
    import torch
    from paper_2206_14307_amd import NQS
    from paper_2206_14307_amd.nqs import KERNELS
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    w = WORKLOADS[name]
    m = NQS.from_workload(w)
    p = draw_params(w)
    m.set_params(torch.from_numpy(p.reshape(-1)))
    sp = torch.from_numpy(random_sz0_spins_fast(w.N, S, 5005)).cuda()
    holder = {}
    ms_e = timed(lambda: holder.update(e=m.eloc(sp, want_logpsi=False)), steps, 0)
    ms_g = timed(lambda: holder.update(O=m.grad(sp)), steps, 0)
    m.profile(True)
    ms_sr = timed(lambda: holder.update(d=m.sr_solve(holder["O"], holder["e"], 1e-6, 0.01)),
                  steps, 0)
    part = {}
    for k in ("gram", "cholesky"):
        ms, n = C.c_double(0), C.c_int64(0)
        m.lib.nqs_profile_read(m._ctx, KERNELS[k], C.byref(ms), C.byref(n), 1)
        part[k] = ms.value / max(n.value, 1)
    # the same system by matrix-free CG in parameter space (two passes over O
    # per iteration: HBM-bound)
    m.profile_read("cg", reset=True)
    cg_out = m.sr_solve_cg(holder["O"], holder["e"], 1e-6, 0.01, tol=1e-8, max_iter=200)
    ms_cg, _ = m.profile_read("cg", reset=True)
    m.profile(False)
    d_cg, iters, resid = cg_out
    o_bytes = holder["O"].numel() * holder["O"].element_size()
    cg_rel = float((torch.linalg.norm(d_cg - holder["d"]) / torch.linalg.norm(holder["d"])).item())
    cg = {"ms": ms_cg, "iterations": iters, "rel_residual": resid,
          "ms_per_iteration": ms_cg / max(iters, 1),
          "rel_diff_vs_sample_space": cg_rel, "bound": "hbm",
          "achieved": 2.0 * o_bytes * iters / (ms_cg / 1e3) / 1e9, "peak": PEAK_HBM_GBS,
          "unit": "GB/s", "frac": 2.0 * o_bytes * iters / (ms_cg / 1e3) / 1e9 / PEAK_HBM_GBS,
          "bytes_per_iteration": 2.0 * o_bytes}
    flops_gram = 8.0 * S * S * m.P / 2
    # complex Cholesky: S^3/6 complex multiply-adds = (4/3) S^3 real flops, plus
    # the two triangular solves (S^2/2 complex multiply-adds each)
    flops_chol = 4.0 * S ** 3 / 3 + 8.0 * S * S
    pk_gram = 78.6 if w.precision == "fp64" else 157.3
    return {"workload": name, "S": S, "P": m.P, "precision": w.precision,
            "ms_eloc": ms_e, "ms_grad": ms_g, "ms_sr": ms_sr,
            "gram": {"ms": part["gram"], "flops_lower_half": flops_gram, "bound": "mfma",
                     "achieved": flops_gram / part["gram"] / 1e9, "peak": pk_gram,
                     "unit": "TFLOP/s", "frac": flops_gram / part["gram"] / 1e9 / pk_gram},
            "cholesky_and_solves": {"ms": part["cholesky"], "flops": flops_chol, "bound": "mfma",
                                    "achieved": flops_chol / part["cholesky"] / 1e9,
                                    "peak": 78.6, "unit": "TFLOP/s",
                                    "frac": flops_chol / part["cholesky"] / 1e9 / 78.6},
            "cg_parameter_space": cg,
            "dtheta_norm": float(holder["d"].abs().pow(2).sum().sqrt().item())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="6x6_fp32_eloc")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--legs", default="grad,logpsi,sq,vmc,lanczos,lanczos2,precision,sr",
                    help="comma-separated subset of the extra legs to run")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--write-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 counter CSVs into the committed JSON and exit")
    args = ap.parse_args()
    if args.write_counters:
        print(json.dumps(write_counters(*args.write_counters), indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the hot path is measured at "
                                   "--gpus 1 only (the multi-GPU sharding is a design, "
                                   "not an implementation)"}))
        sys.exit(2)

    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast

    w = WORKLOADS[args.workload]
    S = w.n_chains * w.n_per_chain
    params = draw_params(w)
    spins_np = random_sz0_spins_fast(w.N, S, 2002)
    # the CPU baseline runs first, in worker processes forked before any GPU use
    # (on uniformly random Sz = 0 configurations: at these near-uniform amplitudes
    # they follow the distribution the sampler produces)
    cpu, refs = None, None
    if not args.no_cpu_baseline:
        want_prec = not args.no_legs and "precision" in args.legs.split(",")
        extra = (precision_leg_refs("8x8_k4_m256"),) if want_prec else ()
        cpu, refs = cpu_baseline(args.workload, params, spins_np, extra=extra)
        log(f"cpu baseline done: {cpu['value']:.3g} {cpu['unit']} on {cpu['cores']} cores")
    spins_random = spins_np
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(params.reshape(-1)))
    # the benchmark's configurations come from the sampler: n_chains x n_per_chain
    # samples, automatic N_skip, burn-in 20 N proposals per chain
    init = torch.from_numpy(spins_np[: w.n_chains]).cuda()
    state = m.chain_init(init)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp, acc_rate, nskip = m.sample(state, w.n_per_chain, n_skip=0, n_burn=20 * w.N, seed=2002)
    torch.cuda.synchronize()
    t_sample = time.perf_counter() - t0
    nskip = int(nskip.item())
    props = w.n_chains * (20 * w.N + w.n_per_chain * nskip)
    acc = float(acc_rate.mean().item())
    # per proposal: G K M exchange factors (13 flops each, as for E_loc) and, if
    # accepted, the tanh addition (t - T)/(1 - t T) of every (g, h): ~20 flops
    fl_s = props * w.G * w.n_rbm * w.n_hidden * (13.0 + 20.0 * acc)
    sample_leg = {"chains": w.n_chains, "per_chain": w.n_per_chain, "burn_in": 20 * w.N,
                  "n_skip": nskip, "acceptance": acc, "seconds": t_sample,
                  "proposals_per_s": props / t_sample,
                  "roofline": {"bound": "alu", "achieved": fl_s / t_sample / 1e12, "peak": 157.3,
                               "unit": "TFLOP/s", "frac": fl_s / t_sample / 1e12 / 157.3,
                               "flops_per_factor": "13 + 20 x acceptance"}}
    log(f"sampled {S} configurations in {t_sample:.2f} s (N_skip {nskip})")
    spins_np = sp.cpu().numpy()
    lp = torch.empty(S, dtype=torch.complex128, device="cuda")
    el = torch.empty(S, dtype=torch.complex128, device="cuda")
    ws = m.workspace("eloc", S)
    from paper_2206_14307_amd.nqs import _ptr, _stream

    def step():
        m._check(m.lib.nqs_eloc(m._ctx, _ptr(sp), S, _ptr(lp), _ptr(el), _ptr(ws), ws.numel(),
                                _stream()), "nqs_eloc")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    m.profile(True)
    for k in ("theta", "lse", "eloc_bonds", "eloc_finish"):
        m.profile_read(k, reset=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step")
    kern = {k: m.profile_read(k, reset=True) for k in ("theta", "lse", "eloc_bonds", "eloc_finish")}
    m.profile(False)

    nc = n_antiparallel(spins_np, square_bonds(w.L)).astype(np.int64)
    factors_per_step = int(nc.sum()) * w.G * w.n_rbm * w.n_hidden
    ms_bonds, n_bonds = kern["eloc_bonds"]
    launches_per_step = n_bonds / args.steps
    flops_per_launch = FLOPS_PER_FACTOR * factors_per_step / launches_per_step
    avg_ms = ms_bonds / n_bonds
    achieved = flops_per_launch / (avg_ms / 1e3) / 1e12
    roofline = {"kernel": "eloc_fused_kernel", "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                "traffic": counted_traffic() if args.workload == "6x6_fp32_eloc" else None,
                "avg_launch_ms": avg_ms, "launches_per_step": launches_per_step,
                "flops_per_launch": flops_per_launch,
                "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kern.items()}}

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    errs = None
    if refs is not None:
        # the oracle's values come from the CPU-baseline leg: evaluate the same
        # configurations on the GPU path and compare
        chk = torch.from_numpy(spins_random[refs["idx"]]).cuda()
        glp, gel = m.eloc(chk)
        errs = errors_of(glp.cpu().numpy(), gel.cpu().numpy(), refs["logpsi"], refs["eloc"])
        errs["configurations"] = "the CPU-baseline sample (uniform Sz = 0)"
        log(f"errors vs oracle: {errs}")
    result = {
        "metric": "configs*sym-images/s for logpsi+E_loc, 1 GPU, at stated energy error",
        "value": S * w.n_rbm * w.G / (ms_step / 1e3),
        "unit": "configs*sym-images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "lattice": f"{w.L}x{w.L}", "J2": w.J2,
                   "n_rbm": w.n_rbm, "n_hidden": w.n_hidden, "sym_images": w.G,
                   "configs": S, "params": "N(0,0.01) complex, seed %d" % w.seed,
                   "spins": "exchange Metropolis samples (nqs_sample), seed 2002"},
        "roofline": roofline,
        "errors": errs,
    }
    legs = {"sample": sample_leg}
    which = set() if args.no_legs else set(args.legs.split(","))
    if "grad" in which:
        legs["grad"] = leg_grad(m, sp, S, w.G, w.n_rbm)
        log(f"grad leg: {legs['grad']['ms']:.2f} ms")
    if "logpsi" in which:
        legs["logpsi"] = leg_logpsi(m, sp, S, w)
        log(f"logpsi leg: {legs['logpsi']['ms']:.2f} ms")
    if "sq" in which:
        legs["structure_factor"] = leg_sq(m, sp, S, w)
        log(f"structure factor leg: {legs['structure_factor']['ms']:.3f} ms")
    if "vmc" in which:
        legs["vmc_training"] = leg_vmc()
        log(f"vmc leg: {legs['vmc_training']['ms_per_training_step']:.1f} ms per 6x6 step")
    if "lanczos" in which:
        legs["lanczos_two_hop"] = leg_lanczos()
        log(f"lanczos leg: {legs['lanczos_two_hop']['ms']:.2f} ms")
    if "lanczos2" in which:
        legs["lanczos_p2"] = leg_lanczos2()
        log(f"lanczos p=2 leg: {legs['lanczos_p2']['ms']:.1f} ms")
    if "precision" in which:
        legs["bf16x2_vs_fp32_8x8"] = leg_precision(
            "8x8_k4_m256", None if refs is None or not refs["extra"] else refs["extra"][0])
        log("precision leg done")
    if "sr" in which:
        legs["sr_10x10"] = leg_sr()
        log(f"sr leg: {legs['sr_10x10']['ms_sr']:.1f} ms")
    result["legs"] = legs
    del ws
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
