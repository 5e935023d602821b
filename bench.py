#!/usr/bin/env python3
"""Benchmark: configs*sym-images/s for log psi + E_loc + d log psi on one MI355X.

Workload (default): the 10x10 J1-J2 lattice (J2/J1 = 0.5), one complex RBM
with M = 400 (alpha = 4), theta on split hi+lo BF16 MFMA with FP32
accumulation, projected on the 800 space-group images; 1024 exchange-
Metropolis chains x 32 samples = 32 768 configurations drawn by nqs_sample
and resident in HBM.  A step is one nqs_eloc_grad call over the whole batch:
log psi, E_loc and O_k = d log psi / d theta_k for W, a, b (the gradient's
image weights from the log amplitudes of the E_loc pass); value =
S * K * G / step time.

Printed as ONE JSON line, with
  roofline     -- the dominant kernel (the wide E_loc kernel): achieved
                  algorithmic TFLOP/s, 10 real flops per exchange factor
                  (configuration x antiparallel bond x image x hidden unit),
                  over its average launch time from HIP events recorded live
                  around each launch on the call's stream, against the FP32
                  vector peak; HBM traffic from committed rocprofv3 counters;
  cpu_baseline -- the FP64 oracle (log psi, E_loc, O_k) timed on this host's
                  cores on a bounded sample of the timed configurations, and
                  its one-core rate;
  errors       -- log psi / E_loc / O errors of the timed step's outputs vs
                  the oracle on that sample;
  legs         -- the FP32-theta step beside the split-BF16 one, the
                  backward's MFMA fraction, sampling, theta alone, the 6x6
                  fused E_loc workload, split-BF16 vs FP32 on 256 stored
                  oracle rows, two-hop Lanczos moments, p = 2, S(q), SR at
                  10x10 on the step's O, VMC training.
"""
from __future__ import annotations

import argparse
import hashlib
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
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6          # MI355X published FP64 vector (and MFMA) peak
FLOPS_PER_FACTOR = 10            # one exchange factor P <- P (1 + s t T), counted as 10 flops
CPU_SHARE = 16                   # host cores per GPU on the MI355X hosts measured (one GPU's share)


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


def square_bonds(L):
    """The 4N bonds of the L x L torus: (i, i+x), (i, i+y) (J1), (i, i+x+y), (i, i+x-y) (J2)."""
    out = []
    for dx, dy in ((1, 0), (0, 1), (1, 1), (1, -1)):
        for i in range(L * L):
            x, y = i % L, i // L
            out.append((i, (x + dx) % L + L * ((y + dy) % L)))
    return np.array(out, dtype=np.int64)


def n_antiparallel(spins, bonds):
    return (spins[:, bonds[:, 0]] != spins[:, bonds[:, 1]]).sum(axis=1)


# ------------------------------------------------------------ HBM counters

COUNTERS = {
    "10x10_m400": {
        "json": os.path.join(ROOT, "profiles", "eloc_wide_10x10_m400_hbm_counters.json"),
        "kernel": "eloc_wide_kernel",
        "sources": ["k_eloc_wide.hip", "theta_common.h", "device_common.h", "nqs_internal.h",
                    "hops.h", "lds_layout.cpp"],
        "workload": "10x10 M=400 split-BF16 theta, 32768 sampled configurations, one launch"},
    "6x6_fp32_eloc": {
        "json": os.path.join(ROOT, "profiles", "eloc_fused_6x6_m72_hbm_counters.json"),
        "kernel": "eloc_fused_kernel",
        "sources": ["k_eloc_fused.hip", "fused_theta.h", "theta_common.h", "device_common.h",
                    "nqs_internal.h", "lds_layout.cpp"],
        "workload": "6x6 M=72 FP32, 262144 configurations, one launch"},
}


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2206_14307_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def write_counters(workload, fetch_csv, write_csv, copy_bytes=1 << 30):
    """Summarise two rocprofv3 --pmc runs of `bench.py --copy-probe` (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch) into the committed counter JSON: the
    kernel's mean per launch, scaled by what the counter reads for the 1 GiB
    device copy the same run makes."""
    import csv
    spec = COUNTERS[workload]

    def per_kernel(path, counter):
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    kname = next(k for k in f if spec["kernel"] in k)
    copy = next(k for k in f if "copyBuffer" in k)
    kib = copy_bytes / 1024.0
    cf, cw = max(f[copy]), max(w[copy])
    fk, wk = float(np.mean(f[kname])), float(np.mean(w[kname]))
    d = {
        "kernel": kname.replace("void ", "").replace("nqs::(anonymous namespace)::", "").split("(")[0],
        "workload": spec["workload"],
        "fetch_kib": fk, "write_kib": wk,
        "copy_probe_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": kib / cf, "write_scale": kib / cw,
        "traffic_bytes_per_launch": 1024.0 * (fk * kib / cf + wk * kib / cw),
        "kernel_source_sha256_16": source_hash(spec["sources"]),
        "kernel_sources": spec["sources"],
    }
    with open(spec["json"], "w") as fh:
        json.dump(d, fh, indent=1)
    return d


def counted_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (copy-calibrated), or None when the kernel's
    sources have changed since the counters were taken."""
    spec = COUNTERS.get(workload)
    if spec is None:
        return None
    try:
        d = json.load(open(spec["json"]))
    except (OSError, ValueError):
        return None
    if source_hash(d["kernel_sources"]) != d["kernel_source_sha256_16"]:
        return None
    return d["traffic_bytes_per_launch"]


# ------------------------------------------------------------- CPU baseline

def _oracle_rows(args):
    """Oracle log psi, E_loc and O_k of some configurations, one BLAS thread."""
    name, params, spins = args
    from threadpoolctl import threadpool_limits
    import oracle
    from workloads import WORKLOADS
    om = oracle.Model.from_workload(WORKLOADS[name])
    with threadpool_limits(1):
        lp = oracle.logpsi(om, params, spins)
        el = oracle.eloc_direct(om, params, spins)
        O = oracle.logderiv(om, params, spins)
    return lp, el, O


def cpu_baseline(name, params, spins, budget_s=25.0):
    """Time the oracle's log psi + E_loc + O_k on a bounded sample of the timed
    configurations on this host's cores (spawned worker processes: the parent
    already uses the GPU).  Returns the baseline record and the oracle's
    outputs on the sample (row indices, log psi, E_loc, O)."""
    from workloads import WORKLOADS
    w = WORKLOADS[name]
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(affinity, CPU_SHARE))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        # one-core rate: two configurations in one worker (after an import warm-up)
        pool.map(_oracle_rows, [(name, params, spins[:1])] * cores)
        t0 = time.perf_counter()
        pool.map(_oracle_rows, [(name, params, spins[:2])])
        per = (time.perf_counter() - t0) / 2
        n = int(max(cores, min(len(spins), 0.8 * budget_s * cores / max(per, 1e-3))))
        n = max(cores, (n // cores) * cores)
        log(f"cpu baseline: {per:.2f} s per configuration on one core; timing {n} "
            f"configurations on {cores} worker processes ({affinity} cores in the affinity mask)")
        idx = np.unique(np.linspace(0, len(spins) - 1, n).astype(np.int64))
        chunks = [(name, params, spins[idx[i::cores]]) for i in range(cores)]
        t0 = time.perf_counter()
        outs = pool.map(_oracle_rows, chunks)
        dt = time.perf_counter() - t0
    order = np.concatenate([idx[i::cores] for i in range(cores)])
    refs = {"idx": order, "logpsi": np.concatenate([o[0] for o in outs]),
            "eloc": np.concatenate([o[1] for o in outs]),
            "O": np.concatenate([o[2] for o in outs])}
    rate = len(idx) * w.n_rbm * w.G / dt
    return ({"value": rate, "unit": "configs*sym-images/s", "cores": cores,
             "kind": "oracle", "cpu": cpu_model(), "affinity_cores": affinity,
             "value_1core": w.n_rbm * w.G / per,
             "sample": f"{len(idx)} of the timed (sampled) configurations, evenly spaced; FP64 "
                       f"NumPy log psi + E_loc by direct re-evaluation + O_k, {cores} worker "
                       f"processes with one BLAS thread each, {dt:.1f} s"},
            refs)


def errors_of(lp_gpu, el_gpu, lp_ref, el_ref, O_gpu=None, O_ref=None):
    """log psi / E_loc (/ O) errors of GPU outputs against oracle outputs (same rows)."""
    d = lp_gpu - lp_ref
    d = d.real + 1j * np.angle(np.exp(1j * d.imag))
    out = {"checked": int(len(lp_ref)),
           "max_abs_dlogpsi": float(np.abs(d).max()),
           "max_rel_deloc": float((np.abs(el_gpu - el_ref) / np.maximum(1, np.abs(el_ref))).max()),
           "rel_err_mean_eloc": float(abs(el_gpu.mean() - el_ref.mean()) / abs(el_ref.mean())),
           "mean_eloc_per_site_oracle": None}
    if O_gpu is not None:
        out["max_row_rel_dO"] = float((np.linalg.norm(O_gpu - O_ref, axis=1) /
                                       np.linalg.norm(O_ref, axis=1)).max())
    return out


def stored_oracle_rows(name):
    """(spins, log psi, E_loc) of the 256 stored oracle rows of a workload
    (tests/golden/make_oracle_rows.py), or None if the file is absent or its
    configurations do not regenerate."""
    from workloads import WORKLOADS, random_sz0_spins_fast
    path = os.path.join(ROOT, "tests", "golden", f"oracle_rows_{name}.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    sp = random_sz0_spins_fast(WORKLOADS[name].N, d["rows"], d["seed"])
    if hashlib.sha256(np.ascontiguousarray(sp).tobytes()).hexdigest() != d["spins_sha256"]:
        return None
    cz = lambda a: np.array([complex(x, y) for x, y in a])
    return sp, cz(d["logpsi"]), cz(d["eloc"])


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


def kernel_ms(m, names, fn, steps):
    """Run fn steps times with the library's per-kernel HIP events on; return
    {kernel: (ms per launch, launches per step)}."""
    import torch
    torch.cuda.synchronize()
    m.profile(True)
    for k in names:
        m.profile_read(k, reset=True)
    for _ in range(steps):
        fn()
    out = {}
    for k in names:
        ms, n = m.profile_read(k, reset=True)
        out[k] = (ms / n if n else 0.0, n / steps)
    m.profile(False)
    return out


def sample_spins(m, w, seed=2002):
    """nqs_sample: w.n_chains chains from uniformly random Sz = 0 starts,
    burn-in 20 N proposals, automatic N_skip, w.n_per_chain samples each."""
    import torch
    from workloads import random_sz0_spins_fast
    init = torch.from_numpy(random_sz0_spins_fast(w.N, w.n_chains, seed)).cuda()
    state = m.chain_init(init)
    m.profile(True)
    m.profile_read("sample", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp, acc_rate, nskip = m.sample(state, w.n_per_chain, n_skip=0, n_burn=20 * w.N, seed=seed)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    k_ms, k_n = m.profile_read("sample", reset=True)
    m.profile(False)
    nskip = int(nskip.item())
    props = w.n_chains * (20 * w.N + w.n_per_chain * nskip)
    acc = float(acc_rate.mean().item())
    # per proposal and (image, hidden unit): the exchange factor (10 flops) and,
    # when accepted, the tanh addition (t - T)/(1 - t T) (~20 flops)
    fl = props * w.G * w.n_rbm * w.n_hidden * (FLOPS_PER_FACTOR + 20.0 * acc)
    # one RBM with M in {8, 16, 32, 72} (FP32) keeps tanh(theta) in registers
    # (6x6 M = 72: eight lanes per image); otherwise the chain's cache
    # [G][K M] complex FP32 is read every proposal and written back
    reg = w.n_rbm == 1 and w.n_hidden in (8, 16, 32, 72) and w.precision != "fp64" and w.G <= 512
    reg8 = reg and w.G == 288 and w.n_hidden == 72
    leg = {"workload": w.name, "chains": w.n_chains, "per_chain": w.n_per_chain,
           "burn_in": 20 * w.N, "n_skip": nskip, "acceptance": acc, "seconds": t,
           "kernel": ("sample_reg8_kernel" if reg8 else "sample_reg_kernel") if reg
                     else "sample_kernel",
           "sampler_kernel_ms": k_ms, "sampler_launches": k_n,
           "proposals_per_s": props / t,
           "roofline": {"bound": "alu", "achieved": fl / t / 1e12,
                        "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                        "frac": fl / t / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                        "flops_per_image_hidden_proposal": "10 + 20 x acceptance"}}
    if not reg:
        # the cache and the image's site-pair rows (tables far larger than the
        # L2) read, the cache written back on acceptance
        nb = props * w.G * w.n_rbm * w.n_hidden * 8.0 * (2.0 + acc)
        leg["roofline"] = {"bound": "hbm", "achieved": nb / t / 1e9, "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": nb / t / 1e9 / PEAK_HBM_GBS,
                           "bytes_per_proposal": "G K M x 8 B x (2 + acceptance): the cache "
                                                 "and the site-pair rows read, the cache "
                                                 "written back on acceptance",
                           "alu_frac": fl / t / 1e12 / PEAK_FP32_VECTOR_TFLOPS}
    return sp, leg


def leg_precision_stored(name, steps=2):
    """split-BF16 vs FP32 theta for one workload: nqs_eloc throughput at the
    workload's sample count, and both precisions' errors on the 256 stored
    oracle rows (tests/golden/oracle_rows_<name>.json)."""
    import dataclasses
    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params, random_sz0_spins_fast
    base = WORKLOADS[name]
    S = base.n_chains * base.n_per_chain
    rows = stored_oracle_rows(name)
    sp = torch.from_numpy(random_sz0_spins_fast(base.N, S, 4005)).cuda()
    out = {"workload": name, "S": S}
    for prec in ("fp32", "bf16x2"):
        w = dataclasses.replace(base, precision=prec)
        m = NQS.from_workload(w)
        m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
        ms = timed(lambda: m.eloc(sp), steps, 1)
        rec = {"ms_eloc": ms, "configs_sym_images_per_s": S * w.n_rbm * w.G / (ms / 1e3)}
        if rows is not None:
            lp, el = m.eloc(torch.from_numpy(rows[0]).cuda())
            rec.update(errors_of(lp.cpu().numpy(), el.cpu().numpy(), rows[1], rows[2]))
            rec["mean_eloc_per_site_oracle"] = float(rows[2].real.mean() / w.N)
            rec["configurations"] = "256 stored oracle rows (uniform Sz = 0, seed 4004)"
        out[prec] = rec
        del m
    return out


def leg_theta(m, sp, S, w, steps=3):
    """nqs_logpsi alone (theta GEMM + log 2cosh + LSE): 4N useful MFMA flops per
    complex theta; the log 2cosh epilogue runs on the VALU beside it."""
    import torch
    out = torch.empty(S, dtype=torch.complex128, device="cuda")
    ms = timed(lambda: out.copy_(m.logpsi(sp)), steps, 1)
    flops = 4.0 * w.N * S * w.G * w.n_rbm * w.n_hidden
    # FP32 models run theta on BF16 MFMA too (the exact three-term split of W,
    # site-grouped: ceil(3 (N/4) / 8) 16x16x32 MFMAs per 16 x 16 tile); split
    # BF16 takes ceil(2N / 32) (hi and lo halves of W), FP64 N/4 16x16x4 FP64
    peak = {"fp64": PEAK_FP64_TFLOPS, "fp32": PEAK_BF16_MFMA_TFLOPS,
            "bf16x2": PEAK_BF16_MFMA_TFLOPS}[w.precision]
    km = kernel_ms(m, ("theta", "lse"), lambda: m.logpsi(sp), steps)
    t_ms = km["theta"][0] * km["theta"][1]
    tiles = S * (w.G // 16) * (w.n_rbm * w.n_hidden // 8)
    if w.precision == "fp32":
        executed = tiles * -(-3 * (w.N // 4) // 8) * 16.0 * 16 * 32 * 2
    elif w.precision == "bf16x2":
        executed = tiles * -(-2 * w.N // 32) * 16.0 * 16 * 32 * 2
    else:
        executed = flops
    return {"precision": w.precision, "S": S, "ms": ms,
            "configs_sym_images_per_s": S * w.n_rbm * w.G / (ms / 1e3),
            "kernel_ms": {k: v[0] * v[1] for k, v in km.items()},
            "roofline": {"kernel": "theta_kernel", "bound": "mfma",
                         "achieved": flops / (t_ms / 1e3) / 1e12, "peak": peak,
                         "unit": "TFLOP/s", "frac": flops / (t_ms / 1e3) / 1e12 / peak,
                         "flops": flops,
                         "executed_mfma_tflops": executed / (t_ms / 1e3) / 1e12}}


def grad_roofline(w, S, ms):
    """8 N flops per (configuration, image, hidden unit): the theta recompute
    (4 N) and the contraction with the image (4 N), both on FP32-accumulating MFMA."""
    flops = 8.0 * w.N * S * w.G * w.n_rbm * w.n_hidden
    peak = PEAK_FP64_TFLOPS if w.precision == "fp64" else PEAK_FP32_MFMA_TFLOPS
    return {"bound": "mfma", "achieved": flops / (ms / 1e3) / 1e12, "peak": peak,
            "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / 1e12 / peak, "flops": flops}


def leg_6x6(steps=10):
    """The 6x6 M = 72 FP32 workload: 4096 chains x 64 samples from nqs_sample,
    nqs_eloc with the fused kernel (one launch), its roofline at 10 flops per
    factor, and nqs_grad with the fused gradient kernel."""
    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params
    w = WORKLOADS["6x6_fp32_eloc"]
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(draw_params(w).reshape(-1)))
    sp, sleg = sample_spins(m, w)
    S = sp.shape[0]
    holder = {}
    ms = timed(lambda: holder.update(r=m.eloc(sp)), steps, 2)
    km = kernel_ms(m, ("eloc_bonds",), lambda: m.eloc(sp), steps)
    nc = n_antiparallel(sp.cpu().numpy(), square_bonds(w.L)).astype(np.int64)
    flops = FLOPS_PER_FACTOR * float(nc.sum()) * w.G * w.n_rbm * w.n_hidden
    kms = km["eloc_bonds"][0]
    ms_g = timed(lambda: m.grad(sp), 3, 1)
    return {"workload": w.name, "S": S, "ms_eloc": ms,
            "configs_sym_images_per_s": S * w.n_rbm * w.G / (ms / 1e3),
            "sample": sleg,
            "roofline": {"kernel": "eloc_fused_kernel", "bound": "alu",
                         "achieved": flops / (kms / 1e3) / 1e12, "peak": PEAK_FP32_VECTOR_TFLOPS,
                         "unit": "TFLOP/s",
                         "frac": flops / (kms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                         "avg_launch_ms": kms, "flops_per_launch": flops,
                         "traffic": counted_traffic(w.name)},
            "grad": {"ms": ms_g, "roofline": grad_roofline(w, S, ms_g)}}


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
    """Two-hop e2 + FP64 moments on the 6x6 Lanczos workload (8192 samples),
    and the wide models' e2 on small samples."""
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
    bonds = square_bonds(w.L)
    factors = float(twohop_hops(sp.cpu().numpy(), bonds)) * w.G * w.n_rbm * w.n_hidden
    flops = FLOPS_PER_FACTOR * factors
    out = {"workload": w.name, "S": S, "ms": ms,
           "configs_per_s": S / (ms / 1e3), "h1_per_site": res["h1"] / w.N,
           "e_p1_per_site": res["e_p1"] / w.N, "factors": factors,
           "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12,
                        "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                        "frac": flops / (ms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                        "flops_per_factor": FLOPS_PER_FACTOR}}
    out["wide_models"] = {}
    for name, Sw in (("8x8_k4_m256", 64), ("10x10_m400", 16)):
        ww = WORKLOADS[name]
        mw = NQS.from_workload(ww)
        mw.set_params(torch.from_numpy(draw_params(ww).reshape(-1)))
        spw = torch.from_numpy(random_sz0_spins_fast(ww.N, Sw, 3003)).cuda()
        msw = timed(lambda: mw.lanczos_moments(spw, exact=False, want_e1e2=False), 1, 1)
        fw = float(twohop_hops(spw.cpu().numpy(), square_bonds(ww.L))) * ww.G * ww.n_rbm * ww.n_hidden
        out["wide_models"][name] = {"S": Sw, "ms": msw, "ms_per_config": msw / Sw, "factors": fw,
                                    "factors_per_s": fw / (msw / 1e3),
                                    "frac": FLOPS_PER_FACTOR * fw / (msw / 1e3) / 1e12 /
                                    PEAK_FP32_VECTOR_TFLOPS}
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
    names = ("theta", "lse", "eloc_bonds", "eloc_finish", "twohop", "twohop_finish", "hop3")
    km = kernel_ms(m, names, lambda: m.lanczos_moments_p2(sp, exact=False, want_e123=False), 1)
    bonds = square_bonds(w.L)
    nb = neighbours(spins, bonds)
    factors = float(twohop_hops(spins, bonds) + twohop_hops(nb, bonds)) * w.G * w.n_rbm * w.n_hidden
    flops = FLOPS_PER_FACTOR * factors
    return {"workload": w.name, "S": S, "neighbour_configs": int(len(nb)), "ms": ms,
            "configs_per_s": S / (ms / 1e3), "h1_per_site": res["h1"] / w.N,
            "e_p1_per_site": res["e_p1"] / w.N, "e_p2_per_site": res["e_p2"] / w.N,
            "degenerate": res["degenerate"], "factors": factors,
            "kernel_ms": {k: round(v[0] * v[1], 3) for k, v in km.items()},
            "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12,
                         "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / (ms / 1e3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                         "flops_per_factor": FLOPS_PER_FACTOR}}


def leg_sq(m, sp, S, w, steps=5):
    """nqs_structure_factor over the benchmark's configurations (uniform
    weights): per configuration and momentum q, N real-times-complex FMAs
    (4 FP64 flops each) and |F(q)|^2; timed on the library's own events."""
    m.structure_factor(sp)
    km = kernel_ms(m, ("sq",), lambda: m.structure_factor(sp), steps)
    ms = km["sq"][0]
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
    N_skip = 5/r from the previous step) and of nqs_vmc_step with both solvers.
    Then the 4x4 complex M = 16 model trained for 200 steps of 2048 samples
    from N(0, 0.01): its exact energy against exact diagonalisation of the
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


def leg_sr(m, w, O, el, steps=1):
    """The sample-space SR step on the timed step's O and E_loc: Gram matrix and
    Cholesky factorisation + solves timed with the library's HIP events; then
    the same system by matrix-free CG in parameter space."""
    import torch
    S = O.shape[0]
    holder = {}
    ms_sr = timed(lambda: holder.update(d=m.sr_solve(O, el, 1e-6, 0.01)), steps, 0)
    km = kernel_ms(m, ("gram", "cholesky"), lambda: m.sr_solve(O, el, 1e-6, 0.01), 1)
    kc = kernel_ms(m, ("cg",), lambda: holder.update(
        cg=m.sr_solve_cg(O, el, 1e-6, 0.01, tol=1e-8, max_iter=200)), 1)
    d_cg, iters, resid = holder["cg"]
    ms_cg = kc["cg"][0] * kc["cg"][1]
    o_bytes = O.numel() * O.element_size()
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
    g_ms = km["gram"][0] * km["gram"][1]
    c_ms = km["cholesky"][0] * km["cholesky"][1]
    pk_gram = PEAK_FP64_TFLOPS if w.precision == "fp64" else PEAK_FP32_MFMA_TFLOPS
    return {"workload": w.name, "S": S, "P": m.P, "precision": w.precision, "ms_sr": ms_sr,
            "gram": {"ms": g_ms, "flops_lower_half": flops_gram, "bound": "mfma",
                     "achieved": flops_gram / g_ms / 1e9, "peak": pk_gram,
                     "unit": "TFLOP/s", "frac": flops_gram / g_ms / 1e9 / pk_gram},
            "cholesky_and_solves": {"ms": c_ms, "flops": flops_chol, "bound": "mfma",
                                    "achieved": flops_chol / c_ms / 1e9,
                                    "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                    "frac": flops_chol / c_ms / 1e9 / PEAK_FP64_TFLOPS},
            "cg_parameter_space": cg,
            "dtheta_norm": float(holder["d"].abs().pow(2).sum().sqrt().item())}


# ------------------------------------------------------------------ the step

class Step:
    """One pass of the hot path on device-resident configurations: log psi,
    E_loc and O_k in one nqs_eloc_grad call (for the wide models the gradient
    takes its image weights from the E_loc pass), outputs kept for the error
    check; eloc() and grad() are the two separate calls."""

    def __init__(self, m, sp):
        import torch
        self.m, self.sp, self.S = m, sp, sp.shape[0]
        self.lp = torch.empty(self.S, dtype=torch.complex128, device="cuda")
        self.el = torch.empty(self.S, dtype=torch.complex128, device="cuda")
        self.O = torch.empty((self.S, m.P), dtype=m.o_dtype, device="cuda")
        self.ws_e = torch.empty(max(256, int(m.lib.nqs_workspace_bytes(m._ctx, 1, self.S))),
                                dtype=torch.uint8, device="cuda")
        self.ws_g = torch.empty(max(256, int(m.lib.nqs_workspace_bytes(m._ctx, 3, self.S))),
                                dtype=torch.uint8, device="cuda")
        self.ws_eg = torch.empty(max(256, int(m.lib.nqs_workspace_bytes(m._ctx, 10, self.S))),
                                 dtype=torch.uint8, device="cuda")

    def eloc(self):
        from paper_2206_14307_amd.nqs import _ptr, _stream
        m = self.m
        m._check(m.lib.nqs_eloc(m._ctx, _ptr(self.sp), self.S, _ptr(self.lp), _ptr(self.el),
                                _ptr(self.ws_e), self.ws_e.numel(), _stream()), "nqs_eloc")

    def grad(self):
        from paper_2206_14307_amd.nqs import _ptr, _stream
        m = self.m
        m._check(m.lib.nqs_grad(m._ctx, _ptr(self.sp), self.S, _ptr(self.O), None,
                                _ptr(self.ws_g), self.ws_g.numel(), _stream()), "nqs_grad")

    def __call__(self):
        from paper_2206_14307_amd.nqs import _ptr, _stream
        m = self.m
        m._check(m.lib.nqs_eloc_grad(m._ctx, _ptr(self.sp), self.S, _ptr(self.lp), _ptr(self.el),
                                     _ptr(self.O), _ptr(self.ws_eg), self.ws_eg.numel(),
                                     _stream()), "nqs_eloc_grad")

    def rows(self, idx):
        import torch
        ix = torch.from_numpy(np.asarray(idx)).cuda()
        return (self.lp[ix].cpu().numpy(), self.el[ix].cpu().numpy(),
                self.O[ix].cpu().numpy().astype(np.complex128))


STEP_KERNELS = ("theta", "lse", "eloc_bonds", "eloc_finish", "grad")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="10x10_m400")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--legs", default="fp32,theta,6x6,precision,lanczos,lanczos2,sq,sr,vmc",
                    help="comma-separated subset of the extra legs to run")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--write-counters", nargs=3, metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 counter CSVs into the committed JSON and exit")
    args = ap.parse_args()
    if args.write_counters:
        print(json.dumps(write_counters(*args.write_counters), indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the hot path is measured at "
                                   "--gpus 1 only (the multi-GPU sharding is a design, "
                                   "not an implementation)"}))
        sys.exit(2)

    import dataclasses
    import torch
    from paper_2206_14307_amd import NQS
    from workloads import WORKLOADS, draw_params

    w = WORKLOADS[args.workload]
    params = draw_params(w)
    m = NQS.from_workload(w)
    m.set_params(torch.from_numpy(params.reshape(-1)))
    # the configurations come from the sampler: n_chains x n_per_chain samples,
    # automatic N_skip, burn-in 20 N proposals per chain
    sp, sample_leg = sample_spins(m, w)
    S = sp.shape[0]
    log(f"sampled {S} configurations in {sample_leg['seconds']:.2f} s "
        f"(N_skip {sample_leg['n_skip']}, acceptance {sample_leg['acceptance']:.3f})")
    step = Step(m, sp)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step")
    # per-kernel HIP events (recorded on the call's stream around each launch) over as
    # many further steps
    km = kernel_ms(m, STEP_KERNELS, step, min(args.steps, 5))
    spins_np = sp.cpu().numpy()
    nc = n_antiparallel(spins_np, square_bonds(w.L)).astype(np.int64)
    factors = float(nc.sum()) * w.G * w.n_rbm * w.n_hidden
    dom = "eloc_bonds"
    avg_ms, launches = km[dom]
    flops_per_launch = FLOPS_PER_FACTOR * factors / launches
    achieved = flops_per_launch / (avg_ms / 1e3) / 1e12
    wide = w.n_rbm * w.n_hidden > 128
    roofline = {"kernel": "eloc_wide_kernel" if wide else "eloc_fused_kernel", "bound": "alu",
                "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                "traffic": counted_traffic(args.workload),
                "avg_launch_ms": avg_ms, "launches_per_step": launches,
                "flops_per_launch": flops_per_launch, "flops_per_factor": FLOPS_PER_FACTOR,
                "factors_per_step": factors,
                "kernel_ms_per_step": {k: v[0] * v[1] for k, v in km.items()}}
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    result = {
        "metric": "configs*sym-images/s for logpsi+E_loc+dlogpsi, 1 GPU, at stated energy error",
        "value": S * w.n_rbm * w.G / (ms_step / 1e3),
        "unit": "configs*sym-images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x2+f32" if w.precision == "bf16x2" else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": f"{w.L}x{w.L}", "J2": w.J2,
                   "n_rbm": w.n_rbm, "n_hidden": w.n_hidden, "sym_images": w.G,
                   "configs": S, "theta": w.precision,
                   "step": "nqs_eloc_grad: log psi + E_loc + O_k (W, a, b) in one call, the "
                           "gradient's image weights from the E_loc pass",
                   "params": "N(0,0.01) complex, seed %d" % w.seed,
                   "spins": "exchange Metropolis samples (nqs_sample, %d chains x %d), seed 2002"
                            % (w.n_chains, w.n_per_chain)},
        "roofline": roofline,
    }
    legs = {"sample": sample_leg}
    which = set() if args.no_legs else set(args.legs.split(","))

    # oracle on a bounded sample of the timed configurations (spawned workers)
    cpu, errs = None, None
    if not args.no_cpu_baseline:
        cpu, refs = cpu_baseline(args.workload, params, spins_np)
        log(f"cpu baseline: {cpu['value']:.3g} {cpu['unit']} on {cpu['cores']} cores")
        lp_g, el_g, O_g = step.rows(refs["idx"])
        errs = errors_of(lp_g, el_g, refs["logpsi"], refs["eloc"], O_g, refs["O"])
        errs["mean_eloc_per_site_oracle"] = float(refs["eloc"].real.mean() / w.N)
        errs["configurations"] = "the CPU-baseline sample of the timed configurations"
        log(f"errors vs oracle: {errs}")
    result["errors"] = errs

    # the step's two calls timed apart: nqs_eloc, and nqs_grad (its own theta, log-sum-exp
    # and contraction) with the backward's MFMA fraction
    ms_eloc = timed(step.eloc, 3, 0)
    ms_grad = timed(step.grad, 3, 0)
    legs["eloc"] = {"S": S, "ms": ms_eloc}
    legs["grad"] = {"S": S, "ms": ms_grad, "roofline": grad_roofline(w, S, ms_grad)}
    log(f"eloc {ms_eloc:.1f} ms, grad {ms_grad:.1f} ms")

    if "fp32" in which and w.precision == "bf16x2":
        # the same step with theta in FP32 on the same configurations
        w32 = dataclasses.replace(w, precision="fp32")
        m32 = NQS.from_workload(w32)
        m32.set_params(torch.from_numpy(params.reshape(-1)))
        step32 = Step(m32, sp)
        ms32 = timed(step32, 3, 1)
        rec = {"ms_per_step": ms32, "value": S * w.n_rbm * w.G / (ms32 / 1e3),
               "kernel_ms_per_step": {k: v[0] * v[1] for k, v in
                                      kernel_ms(m32, STEP_KERNELS, step32, 2).items()}}
        if cpu is not None:
            lp_g, el_g, O_g = step32.rows(refs["idx"])
            rec["errors"] = errors_of(lp_g, el_g, refs["logpsi"], refs["eloc"], O_g, refs["O"])
        legs["fp32_theta_step"] = rec
        del step32, m32
        log(f"fp32 theta step: {ms32:.1f} ms")
    if "theta" in which:
        legs["theta_bf16x2" if w.precision == "bf16x2" else "theta"] = leg_theta(m, sp, S, w)
        if w.precision == "bf16x2":
            w32 = dataclasses.replace(w, precision="fp32")
            m32 = NQS.from_workload(w32)
            m32.set_params(torch.from_numpy(params.reshape(-1)))
            legs["theta_fp32"] = leg_theta(m32, sp, S, w32)
            del m32
        log("theta legs done")
    if "sr" in which:
        legs["sr"] = leg_sr(m, w, step.O, step.el)
        log(f"sr leg: {legs['sr']['ms_sr']:.1f} ms")
    del step
    torch.cuda.empty_cache()
    if "sq" in which:
        legs["structure_factor"] = leg_sq(m, sp, S, w)
    if "6x6" in which:
        legs["6x6_fp32_eloc"] = leg_6x6()
        log(f"6x6 leg: {legs['6x6_fp32_eloc']['ms_eloc']:.2f} ms")
    if "precision" in which:
        legs["bf16x2_vs_fp32_8x8"] = leg_precision_stored("8x8_k4_m256")
        legs["bf16x2_vs_fp32_10x10"] = leg_precision_stored("10x10_m400")
        log("precision legs done")
    if "lanczos" in which:
        legs["lanczos_two_hop"] = leg_lanczos()
        log(f"lanczos leg: {legs['lanczos_two_hop']['ms']:.2f} ms")
    if "lanczos2" in which:
        legs["lanczos_p2"] = leg_lanczos2()
        log(f"lanczos p=2 leg: {legs['lanczos_p2']['ms']:.1f} ms")
    if "vmc" in which:
        legs["vmc_training"] = leg_vmc()
        log(f"vmc leg: {legs['vmc_training']['ms_per_training_step']:.1f} ms per 6x6 step")
    result["legs"] = legs
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
