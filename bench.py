#!/usr/bin/env python3
"""Benchmark of the all-vs-all cRMSD hot path on one MI355X.

One step = one full pass of the hot path over the N=20,000 x L=150 ensemble
(prep -> fused MFMA contraction + FP64 Eq. 2 epilogue + packed store ->
FP64 fix-up), split-BF16 precision by default, inputs already resident in
HBM.  Prints ONE JSON line on stdout; progress goes to stderr.

The roofline entry is for the dominant kernel (the fused tile kernel): its
average duration is measured live with HIP events recorded by the library on
the stream it launches on; achieved = algorithmic flops per launch (18 L per
pair: nine length-L dot products, FMA = 2 flops) / that duration.  HBM
traffic comes from a committed rocprofv3 counter summary under profiles/ and
is reported only while the kernel sources still match the hash recorded
there.

The CPU baseline is the FP64 oracle timed on this host's cores on a bounded
sample of the same workload (the all-vs-all of its first n models), and the
maximum error of the GPU scores is measured against the same oracle on a
sample of pairs; both run outside the timed region.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("all-vs-all cRMSD pairs/s (N=20k,L=150); MFMA util; max err vs FP64 oracle (Å)")
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "bf16x4": 2500.0, "fp64": 78.6,
               "int8": 5000.0}
HBM_PEAK_GBS = 8000.0
# FP64 flops per pair of the Eq. 2 epilogue as written (an FMA counts 2):
# coefficients c2, c1, det 67; start and floors 7; three Newton steps 36 and
# the convergence test 1; the two refined square roots and the combination 27;
# the score 2.  The reference frame adds 18 FP64 additions per pair (the
# per-model terms), issued but not part of the method.
EPI_FLOPS = 140.0
KBLOCK = {"fp32": 8, "bf16": 16, "fp16": 16, "bf16x4": 16, "fp64": 1}
KERNEL_SOURCES = ["paper_1302_4000_amd/csrc/tile.hip", "paper_1302_4000_amd/csrc/eq2.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def profile_value(prec: str, workload: str, kind: str, key: str):
    """A figure from a committed rocprofv3 summary of the tile kernel
    (profiles/tile_<prec>_<workload>_<kind>.md), or None when there is none
    or the kernel sources changed since it was taken."""
    pat = os.path.join(ROOT, "profiles", f"tile_{prec}_{workload}_{kind}.md")
    for f in glob.glob(pat):
        txt = open(f).read()
        m_h = re.search(r"source-sha256:\s*([0-9a-f]+)", txt)
        m_b = re.search(re.escape(key) + r":\s*([0-9.eE+-]+)", txt)
        if m_h and m_b and m_h.group(1) == kernel_hash():
            return float(m_b.group(1))
    return None


def traffic_from_profiles(prec: str, workload: str):
    """HBM bytes per tile-kernel launch (FETCH_SIZE / WRITE_SIZE summary)."""
    return profile_value(prec, workload, "hbm_traffic", "traffic-bytes-per-launch")


def issued_mfma_flops(prec: str, N: int, L: int) -> float:
    """MFMA flops the tile kernel issues: every 32x32 pair block of the upper
    triangle of 64x64 tiles, padded K, and three products in split modes."""
    kb = KBLOCK[prec]
    Lp = -(-L // kb) * kb
    Np = -(-N // 64) * 64
    nb = Np // 64
    T = nb * (nb + 1) // 2
    waves = 4 * T - nb          # the wave below the diagonal of a diagonal tile idles
    prod = {"bf16": 3, "fp16": 3, "bf16x4": 4}.get(prec, 1)
    return waves * 32 * 32 * 9 * Lp * 2.0 * prod


# Untimed load before every timed region: after host-side data generation
# the GPU has idled and its clocks come back up over the first tens of
# milliseconds of work (three warmup steps of the headline leave its first
# timed steps about 4% slow); the figures are of the steady state.
RAMP_MS = 100.0


def ramp(torch, fn, min_ms=RAMP_MS):
    """Untimed calls of fn() for about min_ms of wall time."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max((time.perf_counter() - t0) * 1e3, 1e-3)
    n = max(1, min(10000, int(min_ms / one)))
    for _ in range(n):
        fn()
    torch.cuda.synchronize()


def time_path(cl, torch, x, prec, steps, warmup):
    N, L = x.shape[0], x.shape[1]
    P = N * (N - 1) // 2
    out = torch.empty(P, dtype=torch.float32, device=x.device)
    ws = torch.empty(cl.workspace_size(N, L, prec), dtype=torch.uint8, device=x.device)
    ramp(torch, lambda: cl.crmsd_matrix(x, prec, out=out, ws=ws))
    for _ in range(warmup):
        cl.crmsd_matrix(x, prec, out=out, ws=ws)
    torch.cuda.synchronize()
    dev = x.device.index
    cl.binding.stage_timing(dev, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        cl.crmsd_matrix(x, prec, out=out, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, ncalls = cl.binding.stage_times(dev)
    cl.binding.stage_timing(dev, 0)
    assert ncalls == steps
    ms = (t1 - t0) * 1e3 / steps
    return dict(ms_per_step=ms, pairs_per_s=P / (ms * 1e-3),
                prep_ms=stage_ms[0] / steps, tile_ms=stage_ms[1] / steps,
                fixup_ms=stage_ms[2] / steps, fixup_blocks=cl.fixup_count(ws)), out


BINS = [(0.0, 0.5), (0.5, 2.0), (2.0, 5.0), (5.0, 1e30)]


def error_bins(d, r):
    """Max and p99 of |error| per oracle-score bin."""
    import numpy as np
    res = {}
    for lo, hi in BINS:
        m = (r >= lo) & (r < hi)
        key = f"{lo:g}-{hi:g}A" if hi < 1e29 else f">={lo:g}A"
        res[key] = [float(d[m].max()), float(np.quantile(d[m], 0.99))] if m.any() else [0.0, 0.0]
    return res


def host_cpu():
    """What the CPU baseline ran on: model name, logical CPUs of the host,
    CPUs this process may use, and the OpenMP thread setting."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"model": model, "nproc_host": os.cpu_count(), "cpus_allowed": allowed,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_leg(x_np, outs, want_cpu, threads):
    """Maximum error of GPU scores vs the FP64 oracle on a pair sample, and
    the oracle's own throughput on a bounded sample of the workload."""
    import numpy as np
    import torch

    import oracle
    N = x_np.shape[0]
    rng = np.random.default_rng(7)
    i = rng.integers(0, N, 100000)
    j = rng.integers(0, N, 100000)
    keep = i != j
    I, J = np.minimum(i, j)[keep], np.maximum(i, j)[keep]
    ii, jj = np.triu_indices(min(50, N), 1)
    I2 = rng.integers(0, min(50, N), 10000)
    J2 = rng.integers(min(50, N), N, 10000)
    strata = {"uniform_1e5": (I, J), "near_identical_1225": (ii, jj), "near_vs_bulk_1e4": (I2, J2)}
    refs = {name: oracle.crmsd_pairs(x_np, a, b, threads=threads)
            for name, (a, b) in strata.items()}
    errs = {}
    for prec, out in outs.items():
        e = {}
        allerr, allref = [], []
        for name, (a, b) in strata.items():
            k = torch.from_numpy(oracle.packed_index(a, b, N)).to(out.device)
            got = out[k].cpu().numpy().astype(np.float64)
            d = np.abs(got - refs[name])
            e[name] = float(d.max())
            allerr.append(d)
            allref.append(refs[name])
        e["max"] = max(e.values())
        e["by_bin_max_p99"] = error_bins(np.concatenate(allerr), np.concatenate(allref))
        errs[prec] = e
    cpu = None
    if want_cpu:
        # bounded sample: all-vs-all of the first n models, sized to ~15 s
        n0 = min(N, 400)
        t = time.perf_counter()
        oracle.crmsd_matrix(x_np[:n0], threads=threads)
        rate = n0 * (n0 - 1) / 2 / (time.perf_counter() - t)
        n = int(min(N, max(n0, (2 * rate * 15.0) ** 0.5)))
        t = time.perf_counter()
        oracle.crmsd_matrix(x_np[:n], threads=threads)
        dt = time.perf_counter() - t
        pairs = n * (n - 1) // 2
        # one thread, on a smaller sample (about 2 s)
        n1 = int(min(N, max(50, (2 * rate / threads * 2.0) ** 0.5)))
        t = time.perf_counter()
        oracle.crmsd_matrix(x_np[:n1], threads=1)
        dt1 = time.perf_counter() - t
        cpu = {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"all-vs-all of the first {n} models of the same ensemble "
                         f"({pairs} pairs, {dt:.1f} s, FP64 explicit Kabsch, OpenMP)",
               "host": host_cpu(),
               "one_thread": {"value": n1 * (n1 - 1) / 2 / dt1, "unit": "pairs/s",
                              "sample": f"all-vs-all of the first {n1} models ({dt1:.1f} s)"}}
    return errs, cpu


TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "bf16x4": 5e-4}


def raw_outputs(cl, torch, x, precs, force=None):
    """Scores with the FP64 fix-up disabled (tolerance 0): the raw error of
    the contraction + epilogue that the fix-up flag has to cover.  `force`:
    {name: (products, schedule, band)} for names that run a forced
    configuration of split-BF16."""
    outs = {}
    for name in precs:
        p = "bf16" if force and name in force else name
        cl.set_tolerance(p, 0.0)
        if force and name in force:
            cl.force_config(*force[name])
        try:
            outs[name + "_raw"] = cl.crmsd_matrix(x, p)
        finally:
            cl.set_tolerance(p, TOL[p])
            cl.force_config(None)
    torch.cuda.synchronize()
    return outs


def config2_leg(cl, torch, steps, threads, with_error):
    """The FP32 path at N=5,000, L=300 (10% unrelated folds, sigma up to
    8 A): pairs/s of the whole call, and its error against the oracle on
    1e5 uniform pairs, after and before the fix-up; split-BF16 beside it."""
    import numpy as np

    import oracle
    from paper_1302_4000_amd import synth
    x_np = synth.workload("n5000_l300")
    N, L = x_np.shape[0], x_np.shape[1]
    P = N * (N - 1) // 2
    x = torch.from_numpy(x_np).cuda()
    res = {"workload": "n5000_l300", "N": N, "L": L, "pairs": P}
    outs = {}
    for prec in ("fp32", "bf16"):
        r, out = time_path(cl, torch, x, prec, steps, 2)
        res[prec] = r
        outs[prec] = out
    if with_error:
        outs.update(raw_outputs(cl, torch, x, ("fp32", "bf16")))
        rng = np.random.default_rng(17)
        i = rng.integers(0, N, 100000)
        j = rng.integers(0, N, 100000)
        k = i != j
        I, J = np.minimum(i, j)[k], np.maximum(i, j)[k]
        ref = oracle.crmsd_pairs(x_np, I, J, threads=threads)
        idx = torch.from_numpy(oracle.packed_index(I, J, N)).cuda()
        for name, out in outs.items():
            d = np.abs(out[idx].cpu().numpy().astype(np.float64) - ref)
            res.setdefault("max_err_A", {})[name] = {"max": float(d.max()),
                                                     "by_bin_max_p99": error_bins(d, ref)}
        res["error_sample"] = f"{len(I)} uniform pairs"
    return res


def timed(torch, fn, steps, warmup):
    """Mean wall ms of fn() over `steps` calls after the clock ramp and
    `warmup` calls, synchronised."""
    ramp(torch, fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def batched_leg(cl, torch, steps, with_error=False, threads=1):
    """64 uneven ensembles (N ~ logU[100,2000], L ~ logU[50,500]) in one
    launch sequence, replayed from the cached graph; with_error compares a
    per-ensemble pair sample (uniform pairs and the first and last rows)
    with the FP64 oracle."""
    import numpy as np
    from paper_1302_4000_amd import synth
    ens = synth.make_batch()
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    res = {"ensembles": len(ens), "pairs": b.n_out,
           "models": int(sum(e.shape[0] for e in ens))}
    samples = []
    if with_error:
        rng = np.random.default_rng(19)
        for e in ens:
            n = e.shape[0]
            i = rng.integers(0, n, 300)
            j = rng.integers(0, n, 300)
            k = i != j
            I = np.r_[np.minimum(i, j)[k], np.zeros(n - 1, np.int64), np.arange(n - 2, -1, -1)]
            J = np.r_[np.maximum(i, j)[k], np.arange(1, n), np.full(n - 1, n - 1)]
            samples.append((I, J))
    refs = None
    for prec in ("bf16", "fp32"):
        ws = torch.empty(cl.batched_workspace_size(b, prec), dtype=torch.uint8, device="cuda")
        out = torch.empty(b.n_out, dtype=torch.float32, device="cuda")
        ms = timed(torch, lambda: cl.crmsd_batched(b, flat, prec, out=out, ws=ws), steps, 2)
        r = {"ms_per_call": ms, "pairs_per_s": b.n_out / (ms * 1e-3)}
        if with_error:
            import oracle
            if refs is None:
                refs = [oracle.crmsd_pairs(e, I, J, threads=threads)
                        for e, (I, J) in zip(ens, samples)]
            views = b.split(out)
            worst, allerr, allref = 0.0, [], []
            for e, (I, J), ref, v in zip(ens, samples, refs, views):
                got = v[torch.from_numpy(oracle.packed_index(I, J, e.shape[0])).cuda()]
                d = np.abs(got.cpu().numpy().astype(np.float64) - ref)
                allerr.append(d)
                allref.append(ref)
            d, rr = np.concatenate(allerr), np.concatenate(allref)
            r["max_err_A"] = {"max": float(d.max()), "by_bin_max_p99": error_bins(d, rr)}
            r["error_sample"] = (f"{len(d)} pairs: per ensemble ~300 uniform pairs plus its "
                                 "first and last rows")
        res[prec] = r
    return res


def backward_leg(cl, torch, steps):
    """Forward + hand-written backward of the mean pairwise cRMSD over the
    N=4096, L=256 ensemble, and of the mean cRMSD of every model against the
    native (target-vs-many)."""
    from paper_1302_4000_amd import synth
    x_np, native = synth.grad_workload()
    N, L = x_np.shape[0], x_np.shape[1]
    P = N * (N - 1) // 2
    x = torch.from_numpy(x_np).cuda()
    ref = torch.from_numpy(native[None]).cuda()
    g = torch.full((P,), 1.0 / P, device="cuda")
    gt = torch.full((N, 1), 1.0 / N, device="cuda")
    res = {"workload": "n4096_l256", "N": N, "L": L, "pairs": P}
    dev = x.device.index
    for prec in ("fp32", "bf16"):
        out = cl.crmsd_matrix(x, prec)
        fwd = timed(torch, lambda: cl.crmsd_matrix(x, prec, out=out), steps, 1)
        cl.crmsd_backward(x, out, g, prec)
        torch.cuda.synchronize()
        cl.binding.stage_timing(dev, steps)
        bwd = timed(torch, lambda: cl.crmsd_backward(x, out, g, prec), steps, 0)
        stage_ms, ncalls = cl.binding.stage_times(dev)
        cl.binding.stage_timing(dev, 0)
        assert ncalls == steps
        pairs_ms, grad_ms = stage_ms[1] / steps, stage_ms[2] / steps
        # gradient contraction: 9 multiply-adds per (model, partner, atom),
        # FP32 MFMA with an FP64 fold per partner block
        grad_tf = 18.0 * N * (N - 1) * L / (grad_ms * 1e-3) / 1e12
        tv = cl.crmsd_cross(x, ref, prec)
        tfwd = timed(torch, lambda: cl.crmsd_cross(x, ref, prec, out=tv), steps, 1)
        tbwd = timed(torch, lambda: cl.crmsd_cross_backward(x, ref, tv, gt, prec), steps, 1)
        res[prec] = {"forward_ms": fwd, "backward_ms": bwd,
                     "backward_stages_ms": {"prep": stage_ms[0] / steps, "pairs_pass": pairs_ms,
                                            "gradient_pass": grad_ms},
                     "gradient_tflops": grad_tf,
                     "gradient_frac_of_fp32_mfma_peak": grad_tf / PEAK_TFLOPS["fp32"],
                     "fwd_bwd_pairs_per_s": P / ((fwd + bwd) * 1e-3),
                     "target_vs_many_forward_ms": tfwd, "target_vs_many_backward_ms": tbwd}
    return res


def sizes_leg(cl, torch, steps):
    """The headline recipe (split-BF16, L = 150) at the smallest and the
    largest decoy-set size of the paper's I-TASSER benchmark (12,500 and
    32,000 models per target; Results and Discussion, Table 1): pairs/s of
    the whole call at each size, with the configuration the table gives it."""
    from paper_1302_4000_amd import synth
    res = {}
    for N in (12500, 32000):
        x = torch.from_numpy(synth.workload("n20000_l150", N=N)).cuda()
        r, out = time_path(cl, torch, x, "bf16", steps, 2)
        r["kernel_config"] = cl.get_config(N, x.shape[1], "bf16")
        res[f"n{N}_l150"] = r
        del x, out
        torch.cuda.empty_cache()
    return res


def threshold_leg(cl, torch, x, steps):
    """Pairs below 3.2 A (the paper's threshold example) on the same
    ensemble, emitted without storing the packed matrix."""
    N = x.shape[0]
    P = N * (N - 1) // 2
    res = {"cutoff_A": 3.2}
    for prec in ("bf16",):
        _, _, _, n = cl.crmsd_threshold(x, 3.2, prec)
        cap = n + 1024
        ws = torch.empty(cl.binding.lib().clusco_crmsd_threshold_workspace_size(
            cl.binding.handle(x.device.index), N, x.shape[1], cl.PRECISION[prec]),
            dtype=torch.uint8, device=x.device)
        ms = timed(torch, lambda: cl.crmsd_threshold(x, 3.2, prec, capacity=cap, ws=ws,
                                                      sync=False), steps, 1)
        res[prec] = {"ms_per_call": ms, "pairs_per_s": P / (ms * 1e-3), "pairs_below": n}
    return res


def drmsd_leg(cl, torch, x, x_np, steps, with_error):
    """All-vs-all dRMSD (Eq. 5) on the same ensemble: a Gram product over
    K = L(L-1)/2 distance deviations per model.  Algorithmic work 2 K flops
    per pair (one length-K dot product); issued 3x (split) on MFMA."""
    import numpy as np
    N, L = x.shape[0], x.shape[1]
    P = N * (N - 1) // 2
    K = L * (L - 1) // 2
    res = {"K": K}
    for prec in ("bf16",):
        out = torch.empty(P, dtype=torch.float32, device=x.device)
        ws = torch.empty(cl.drmsd_workspace_size(N, L, prec), dtype=torch.uint8, device=x.device)
        ramp(torch, lambda: cl.drmsd_matrix(x, prec, out=out, ws=ws))
        dev = x.device.index
        cl.binding.stage_timing(dev, steps)
        t0 = time.perf_counter()
        for _ in range(steps):
            cl.drmsd_matrix(x, prec, out=out, ws=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        st, n = cl.binding.stage_times(dev)
        cl.binding.stage_timing(dev, 0)
        assert n == steps
        tile_ms = st[1] / steps
        alg = 2.0 * K * P
        r = {"ms_per_call": ms, "pairs_per_s": P / (ms * 1e-3),
             "stages_ms": {"prep_ms": st[0] / steps, "tile_ms": tile_ms,
                           "fixup_ms": st[2] / steps},
             "fixup_blocks": cl.fixup_count(ws),
             "tile_algorithmic_tflops": alg / (tile_ms * 1e-3) / 1e12,
             "tile_frac_of_bf16_peak": alg / (tile_ms * 1e-3) / (PEAK_TFLOPS["bf16"] * 1e12),
             "tile_mfma_util": 3.0 * 2.0 * (-(-K // 16) * 16) * P / (tile_ms * 1e-3)
             / (PEAK_TFLOPS["bf16"] * 1e12)}
        if with_error:
            import oracle
            rng = np.random.default_rng(11)
            i = rng.integers(0, N, 20000)
            j = rng.integers(0, N, 20000)
            k = i != j
            I, J = np.minimum(i, j)[k], np.maximum(i, j)[k]
            ii, jj = np.triu_indices(min(N, 50), 1)
            I, J = np.r_[I, ii], np.r_[J, jj]
            got = out[torch.from_numpy(oracle.packed_index(I, J, N)).to(x.device)].cpu().numpy()
            r["max_err_A"] = float(np.abs(got.astype(np.float64) - oracle.drmsd_pairs(x_np, I, J)).max())
            r["error_sample"] = f"{len(I)} pairs: uniform + all pairs of models 0-49"
        res[prec] = r
        del out, ws
    return res


def cmo_leg(cl, torch, x, x_np, steps, with_error):
    """All-vs-all contact map overlap (Eq. 6-7, cut-off 8 A): an int8 Gram
    product of 0/1 contact vectors over K = L(L-1)/2 atom pairs.  Algorithmic
    work 2 K integer operations per pair against the int8 MFMA peak."""
    import numpy as np
    N, L = x.shape[0], x.shape[1]
    P = N * (N - 1) // 2
    K = L * (L - 1) // 2
    out = torch.empty(P, dtype=torch.float32, device=x.device)
    ws = torch.empty(cl.cmo_workspace_size(N, L), dtype=torch.uint8, device=x.device)
    ramp(torch, lambda: cl.cmo_matrix(x, 8.0, out=out, ws=ws))
    dev = x.device.index
    cl.binding.stage_timing(dev, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        cl.cmo_matrix(x, 8.0, out=out, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st, n = cl.binding.stage_times(dev)
    cl.binding.stage_timing(dev, 0)
    assert n == steps
    kern_ms = st[1] / steps
    ops = 2.0 * K * P
    r = {"K": K, "cutoff_A": 8.0, "ms_per_call": ms, "pairs_per_s": P / (ms * 1e-3),
         "kernels_ms": kern_ms, "int8_tops": ops / (kern_ms * 1e-3) / 1e12,
         "frac_of_int8_peak": ops / (kern_ms * 1e-3) / (PEAK_TFLOPS["int8"] * 1e12)}
    if with_error:
        import oracle
        rng = np.random.default_rng(13)
        i = rng.integers(0, N, 5000)
        j = rng.integers(0, N, 5000)
        k = i != j
        I, J = np.minimum(i, j)[k], np.maximum(i, j)[k]
        got = out[torch.from_numpy(oracle.packed_index(I, J, N)).to(x.device)].cpu().numpy()
        want = oracle.cmo_pairs(x_np, I, J, 8.0).astype(np.float32)
        r["exact_matches"] = f"{int((got == want).sum())}/{len(I)}"
    del out, ws
    return r


def kmedoids_leg(cl, torch, D, N, steps):
    """K-means with member centres (k = 20, the paper's setting for decoy
    sets) over the packed matrix the main path produced.  Each update pass
    streams the whole packed matrix once: 4 bytes per pair per pass."""
    k = 20
    init = [(c * N) // k for c in range(k)]
    ws = torch.empty(cl.binding.lib().clusco_cluster_workspace_size(
        cl.binding.handle(D.device.index), N, k), dtype=torch.uint8, device=D.device)
    r = cl.kmedoids(D, N, k, init, 100, ws=ws)
    torch.cuda.synchronize()
    ms = timed(torch, lambda: cl.kmedoids(D, N, k, init, 100, ws=ws), steps, 1)
    ms_async = timed(torch, lambda: cl.kmedoids(D, N, k, init, 20, ws=ws, check_every=0), steps, 1)
    info = r["info"].cpu().tolist()
    passes = info[1] + (0 if info[2] else 1)
    gbs = passes * 4.0 * D.numel() / (ms * 1e-3) / 1e9
    return {"k": k, "ms_per_call": ms, "updates": info[1], "converged": bool(info[2]),
            "representative_cluster": info[0],
            "matrix_passes": passes, "matrix_stream_gbs": gbs, "frac_of_hbm_peak": gbs / 8000.0,
            "ms_async_max_iter_20": ms_async}


def copy_calibration(nbytes: int):
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--workload", default="n20000_l150")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true", help="skip the oracle error sample")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32-path comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and backward measurements")
    ap.add_argument("--leg", choices=["backward", "batched"], default=None,
                    help="only run one supporting measurement and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the all-vs-all cRMSD kernels run on a single "
              "MI355X; multi-GPU sharding is a design note only (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import numpy as np
    import torch

    import paper_1302_4000_amd as cl
    from paper_1302_4000_amd import synth

    if args.leg == "backward":
        log("[bench] backward only: N=4096 L=256")
        print(json.dumps({"leg": "backward", **backward_leg(cl, torch, args.steps)}), flush=True)
        return
    if args.leg == "batched":
        log("[bench] batched only: 64 uneven ensembles")
        print(json.dumps({"leg": "batched", **batched_leg(cl, torch, args.steps)}), flush=True)
        return

    log(f"[bench] generating {args.workload}")
    x_np = synth.workload(args.workload)
    N, L = x_np.shape[0], x_np.shape[1]
    P = N * (N - 1) // 2
    x = torch.from_numpy(x_np).cuda()
    torch.cuda.synchronize()

    prec = args.precision
    # the kernel configuration the tuning table gives this size (split-BF16:
    # three or four MFMA products per K-block)
    kcfg = cl.get_config(N, L, prec)
    iprec = "bf16x4" if prec == "bf16" and kcfg["products"] == 4 else prec
    log(f"[bench] {prec}: kernel configuration {kcfg}; warmup {args.warmup}, steps {args.steps}")
    main_res, main_out = time_path(cl, torch, x, prec, args.steps, args.warmup)
    log(f"[bench] {prec}: {main_res}")
    outs = {prec: main_out}
    if not args.no_error:
        outs.update(raw_outputs(cl, torch, x, [prec] + ([] if args.no_compare or prec == "fp32"
                                                        else ["fp32"])))
    cmp = None
    if not args.no_compare and prec != "fp32":
        steps = max(2, args.steps // 3)
        log(f"[bench] fp32 comparison: steps {steps}")
        cmp_res, cmp_out = time_path(cl, torch, x, "fp32", steps, 1)
        log(f"[bench] fp32: {cmp_res}")
        fl = issued_mfma_flops("fp32", N, L)
        cmp = dict(cmp_res, steps=steps,
                   mfma_util=fl / (cmp_res["tile_ms"] * 1e-3) / (PEAK_TFLOPS["fp32"] * 1e12),
                   algorithmic_tflops=18.0 * L * P / (cmp_res["tile_ms"] * 1e-3) / 1e12)
        outs["fp32"] = cmp_out
    variants = {}
    if not args.no_compare and prec == "bf16":
        # split-BF16 with the other product count than the table chose
        other = 3 if kcfg["products"] == 4 else 4
        name = f"bf16_x{other}"
        force = {name: (other, kcfg["schedule"], kcfg["band"])}
        steps = max(2, args.steps // 3)
        log(f"[bench] {name}: split-BF16 forced to {other} products, steps {steps}")
        cl.force_config(*force[name])
        try:
            vres, vout = time_path(cl, torch, x, "bf16", steps, 1)
        finally:
            cl.force_config(None)
        vres["mfma_util"] = issued_mfma_flops("bf16x4" if other == 4 else "bf16", N, L) / (
            vres["tile_ms"] * 1e-3) / (PEAK_TFLOPS["bf16"] * 1e12)
        log(f"[bench] {name}: {vres}")
        variants[name] = vres
        outs[name] = vout
        if not args.no_error:
            outs.update(raw_outputs(cl, torch, x, [name], force))
        for vp in ("fp16", "bf16x4"):
            steps = max(2, args.steps // 3)
            log(f"[bench] {vp} variant: steps {steps}")
            vres, vout = time_path(cl, torch, x, vp, steps, 1)
            vres["mfma_util"] = issued_mfma_flops(vp, N, L) / (vres["tile_ms"] * 1e-3) / (
                PEAK_TFLOPS[vp] * 1e12)
            log(f"[bench] {vp}: {vres}")
            variants[vp] = vres
            outs[vp] = vout

    # every host CPU this process may run on (the box's whole share)
    threads = max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                  else (os.cpu_count() or 1))
    extra = {}
    if not args.no_extra:
        log("[bench] config n5000_l300 (FP32 path at scale)")
        extra["n5000_l300"] = config2_leg(cl, torch, max(3, args.steps // 2), threads,
                                          not args.no_error)
        log(f"[bench] n5000_l300: {extra['n5000_l300']}")
        log("[bench] decoy-set sizes 12,500 and 32,000 (split-BF16, L=150)")
        extra["sizes"] = sizes_leg(cl, torch, max(3, args.steps // 2))
        log(f"[bench] sizes: {extra['sizes']}")
        log("[bench] threshold 3.2 A")
        extra["threshold"] = threshold_leg(cl, torch, x, max(3, args.steps // 2))
        log(f"[bench] threshold: {extra['threshold']}")
        log("[bench] batched: 64 uneven ensembles")
        extra["batched"] = batched_leg(cl, torch, max(3, args.steps // 2), not args.no_error,
                                       threads)
        log(f"[bench] batched: {extra['batched']}")
        log("[bench] K-means (member centres) on the packed matrix")
        extra["kmedoids"] = kmedoids_leg(cl, torch, main_out, N, max(3, args.steps // 3))
        log(f"[bench] kmedoids: {extra['kmedoids']}")
        log("[bench] contact map overlap all-vs-all")
        extra["cmo"] = cmo_leg(cl, torch, x, x_np, max(3, args.steps // 3), not args.no_error)
        log(f"[bench] cmo: {extra['cmo']}")
        log("[bench] dRMSD all-vs-all")
        extra["drmsd"] = drmsd_leg(cl, torch, x, x_np, max(3, args.steps // 3), not args.no_error)
        log(f"[bench] drmsd: {extra['drmsd']}")
        log("[bench] backward: N=4096 L=256")
        extra["backward"] = backward_leg(cl, torch, max(3, args.steps // 2))
        log(f"[bench] backward: {extra['backward']}")

    errs, cpu = (None, None)
    if not (args.no_error and args.no_cpu_baseline):
        log(f"[bench] oracle leg on {threads} host threads")
        errs, cpu = oracle_leg(x_np, outs if not args.no_error else {}, not args.no_cpu_baseline,
                               threads)

    tile_s = main_res["tile_ms"] * 1e-3
    alg = 18.0 * L * P                      # contraction flops the method needs
    issued = issued_mfma_flops(iprec, N, L)
    epi = EPI_FLOPS * P                     # FP64 epilogue flops the method needs
    prof_ms = profile_value(iprec, args.workload, "kernel_trace", "avg-ms-per-launch")
    # The split modes are bound by the FP64 vector ALU (the per-pair Eq. 2
    # epilogue; the committed counters show the vector ALU busier than the
    # matrix cores, and removing the epilogue arithmetic removes its whole
    # time), the FP32 mode by the FP32 matrix cores.
    alu = prec != "fp32"
    work, peak = (epi, PEAK_TFLOPS["fp64"]) if alu else (alg, PEAK_TFLOPS["fp32"])
    achieved = work / tile_s / 1e12
    counters = {k: profile_value(iprec, args.workload, "counters", k)
                for k in ("mfma-busy-frac", "valu-busy-frac", "mfma-valu-coexec-frac",
                          "valu-insts-per-pair", "fp64-insts-per-pair")}
    roof = {"bound": "alu" if alu else "mfma", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic_from_profiles(iprec, args.workload),
            "kernel": f"staged_kernel<{iprec}>", "kernel_ms": main_res["tile_ms"],
            # the same fraction from the committed rocprofv3 trace of this
            # kernel (another box: box-to-box spread applies)
            "profile_kernel_ms": prof_ms,
            "profile_frac": (work / (prof_ms * 1e-3) / 1e12 / peak) if prof_ms else None,
            "work": ("FP64 Eq. 2 epilogue, %.0f flops per pair" % EPI_FLOPS) if alu else
                    "contraction, 18 L flops per pair",
            # the matrix-core side: the method's 18 L flops per pair, and what
            # the kernel issues (padded K, split products, whole 32x32 blocks)
            "mfma": {"algorithmic_tflops": alg / tile_s / 1e12,
                     "algorithmic_frac": alg / tile_s / 1e12 / PEAK_TFLOPS[prec],
                     "issued_tflops": issued / tile_s / 1e12,
                     "issued_frac": issued / tile_s / (PEAK_TFLOPS[prec] * 1e12),
                     "effective_vs_fp32_peak": alg / tile_s / 1e12 / PEAK_TFLOPS["fp32"]},
            "fp64_epilogue": {"flops_per_pair": EPI_FLOPS,
                              "achieved": epi / tile_s / 1e12,
                              "frac": epi / tile_s / 1e12 / PEAK_TFLOPS["fp64"]},
            # busy fractions and instruction counts of this kernel from the
            # committed rocprofv3 counter summary (null when the kernel sources
            # changed since)
            "counters": counters if any(v is not None for v in counters.values()) else None,
            "output_hbm_gbs": 4.0 * P / tile_s / 1e9,
            "source_sha256": kernel_hash()}
    line = {
        "metric": METRIC, "value": main_res["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "clock_ramp_ms": RAMP_MS,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "L": L, "pairs": P,
                   "precision": {"bf16": f"split_bf16x{kcfg['products']}",
                                 "fp16": "split_fp16x3", "fp32": "fp32"}[prec],
                   "kernel_config": kcfg,
                   "epilogue": "fp64", "parallelism": "single_gpu"},
        "stages_ms": {k: main_res[k] for k in ("prep_ms", "tile_ms", "fixup_ms")},
        "fixup_blocks": main_res["fixup_blocks"],
        "roofline": roof,
        "max_err_A": errs,
        "fp32_path": cmp,
        "split_variants": variants or None,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
