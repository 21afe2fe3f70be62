"""Tuner of the per-bucket kernel configuration (writes tuning/<arch>.json).

The decoy sets the paper clusters are of very uneven size (Results and
Discussion: 56 I-TASSER targets of 12,500 to 32,000 models, Table 1; the
Figure 1 proteins of 71 to 887 residues), and no single kernel configuration
is best over that range.  For every precision and every (N bucket, L bucket)
this script times the whole all-vs-all call (prep, contraction with the
Eq. 2 epilogue, FP64 fix-up) on a synthetic ensemble of the bucket's
representative size (with near-identical models, as decoy sets have: see
near()), for each candidate configuration forced through
clusco_force_config, and records the fastest.  Then the same inside a
batched call (an entry with "call": "batched"), where the per-call costs are
shared and the best choice for small ensembles differs: k such ensembles (k
from BATCH_PAIRS, at most 32) are added to a fixed background of typical
batch work (BACKGROUNDS: ensembles in the reference frame with three
products, so the batch already pays for the reference pass and a
three-product tile launch; never of the bucket being timed) and each
candidate is set for the bucket through a temporary table; the background's
share is the same for every candidate, so the fastest batch is the bucket's
best marginal choice:

  products   split-BF16 only: 3 or 4 MFMA products per K-block (4 costs a
             third more MFMA issue and leaves far fewer pairs to the fix-up)
  schedule   staged (one tile per workgroup, LDS-staged operands) or
             persistent (ping-pong workgroups)
  band       tile rows per band of the tile order (only where the tile grid
             is wider than a band)
  frame      contract the models (0) or their residuals from the reference
             structure after superposition onto it (1; far fewer pairs for
             the fix-up, a few more FP64 operations per pair)

Times are HIP events on the stream the library launches on (torch's current
stream).  The table is loaded by the library at handle creation
(include/clusco.h); run this on the target device and commit the output:

    python -m paper_1302_4000_amd.tune --out paper_1302_4000_amd/tuning/gfx950.json
"""
from __future__ import annotations

import argparse
import atexit
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

# Bucket lower bounds.  N: powers of two from 256 to 16384 (the last bucket
# holds the paper's largest sets); L: 64 to 512 residues.
# Pairs of the k ensembles a bucket is timed with for its batched entry, and
# the background batch they join: (N, L) of each background ensemble (all in
# one bucket); the bucket of the first background is timed with the second.
BATCH_PAIRS = 2_000_000
BACKGROUNDS = [[(1448, 181), (1448, 181)], [(2896, 362)]]
N_EDGES = [2, 256, 512, 1024, 2048, 4096, 8192, 16384]
L_EDGES = [1, 64, 128, 256, 512]
PRECISIONS = {"fp32": "fp32", "split_bf16": "bf16", "split_fp16": "fp16",
              "split_bf16x4": "bf16x4"}


def representative(edges, i, top, floor):
    """Geometric middle of bucket i, its lower bound raised to `floor` (the
    first buckets start at sizes no ensemble of protein models has); the last
    bucket: `top`."""
    lo = max(edges[i], floor)
    hi = edges[i + 1] if i + 1 < len(edges) else None
    if hi is None:
        return top
    return int(round(math.sqrt(lo * hi)))


def near(N):
    """Near-identical models of an ensemble of N (noise 0.05 A): decoy sets
    hold near-duplicate structures, and without the reference frame their
    pairs are the ones the FP64 fix-up recomputes, so the tuning ensembles
    carry them in the headline workload's proportion (50 of 20,000)."""
    return max(2, N // 400)


def bucket(edges, x):
    """Index of the bucket of x (edges: ascending lower bounds)."""
    return max(i for i, e in enumerate(edges) if x >= e)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ramp(torch, fn, min_ms=100.0):
    """Untimed calls of fn() for about min_ms: after the host-side ensemble
    generation the GPU has idled, and its clocks come back up over the first
    tens of milliseconds of work; without this the first candidates of a
    bucket are timed slow."""
    fn()
    torch.cuda.synchronize()
    t0 = time.time()
    while (time.time() - t0) * 1e3 < min_ms:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def time_call(torch, fn, target_ms=2.0, reps=5):
    """Median per-call milliseconds of fn() (enough calls per sample for
    about target_ms of GPU time), after two warm-up calls."""
    fn()
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    fn()
    e.record()
    e.synchronize()
    est = max(s.elapsed_time(e), 1e-3)
    k = max(1, min(200, int(target_ms / est)))
    samples = []
    for _ in range(reps):
        s.record()
        for _ in range(k):
            fn()
        e.record()
        e.synchronize()
        samples.append(s.elapsed_time(e) / k)
    return float(np.median(samples))


def candidates(prec, N):
    nb = -(-N // 64)
    bands = [8, 16, 32] if nb > 16 else [16]
    prods = {"split_bf16": [3, 4], "split_bf16x4": [4]}.get(prec, [3])
    # the persistent schedule serves problems without the reference frame
    return [(p, sch, b, f) for p in prods for sch in ("staged", "persistent") for b in bands
            for f in ((0, 1) if sch == "staged" else (0,))]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None, help="output JSON (default: tuning/<arch>.json "
                    "next to the library)")
    ap.add_argument("--precisions", default=",".join(PRECISIONS))
    ap.add_argument("--n-top", type=int, default=20000, help="representative N of the last bucket")
    ap.add_argument("--l-top", type=int, default=700, help="representative L of the last bucket")
    ap.add_argument("--margin", type=float, default=0.02,
                    help="keep the default configuration unless a candidate is this much faster")
    args = ap.parse_args(argv)

    import torch

    from . import binding, synth
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    arch = getattr(props, "gcnArchName", "gfx950").split(":")[0]
    out_path = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                                        f"{arch}.json")
    os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
    binding.load_tuning(None)          # time with no table in the way
    precs = [p for p in args.precisions.split(",") if p]
    bgs = [([torch.from_numpy(synth.make_ensemble(9000 + 8 * g + m, n, l, sigma=(0.5, 6.0),
                                                  near_identical=near(n)))
             for m, (n, l) in enumerate(shapes)],
            (bucket(N_EDGES, shapes[0][0]), bucket(L_EDGES, shapes[0][1])), shapes)
           for g, shapes in enumerate(BACKGROUNDS)]
    tmp_fd, tmp_table = tempfile.mkstemp(suffix=".json", prefix="clusco_candidate_")
    os.close(tmp_fd)
    atexit.register(lambda: os.path.exists(tmp_table) and os.remove(tmp_table))
    entries = []
    t_start = time.time()
    for nb in range(len(N_EDGES)):
        N = representative(N_EDGES, nb, args.n_top, 64)
        for lb in range(len(L_EDGES)):
            L = representative(L_EDGES, lb, args.l_top, 24)
            x = torch.from_numpy(synth.make_ensemble(7000 + 16 * nb + lb, N, L, sigma=(0.5, 6.0),
                                                     near_identical=near(N))).to(dev)
            P = N * (N - 1) // 2
            out = torch.empty(P, dtype=torch.float32, device=dev)
            k = max(1, min(32, round(BATCH_PAIRS / P)))
            background, bg_bucket, bg_shapes = bgs[1] if (nb, lb) == bgs[0][1] else bgs[0]
            batch = binding.Batch(bg_shapes + [(N, L)] * k)
            flat = batch.pack(background + [x.cpu()] + [torch.from_numpy(synth.make_ensemble(
                7000 + 16 * nb + lb + 4096 * m, N, L, sigma=(0.5, 6.0), near_identical=near(N)))
                for m in range(1, k)], dev)
            bout = torch.empty(batch.n_out, dtype=torch.float32, device=dev)
            for prec in precs:
                p = PRECISIONS[prec]
                ws = torch.empty(max(256, binding.workspace_size(N, L, p)), dtype=torch.uint8,
                                 device=dev)
                ms = {}
                ramp(torch, lambda: binding.crmsd_matrix(x, p, out=out, ws=ws))
                for prod, sch, band, fr in candidates(prec, N):
                    binding.force_config(prod, sch, band, fr)
                    ms[f"x{prod}/{sch}/{band}/f{fr}"] = time_call(
                        torch, lambda: binding.crmsd_matrix(x, p, out=out, ws=ws))
                binding.force_config(None)
                default = ("x4" if prec == "split_bf16x4" else "x3") + "/staged/16/f1"
                best = min(ms, key=ms.get)
                if default in ms and ms[default] <= ms[best] * (1.0 + args.margin):
                    best = default
                prod, sch, band, fr = best.split("/")
                entries.append({"precision": prec, "n_bucket": nb, "l_bucket": lb,
                                "N": N, "L": L, "products": int(prod[1:]), "schedule": sch,
                                "band": int(band), "frame": int(fr[1:]), "ms": ms,
                                "pairs_per_s": P / (ms[best] * 1e-3)})
                log(f"[tune] {prec:13s} N={N:6d} L={L:4d}: {best:22s} {ms[best]:8.3f} ms "
                    f"(default {ms.get(default, float('nan')):8.3f} ms)")
                del ws
                # the same bucket's k ensembles inside a batched call with the
                # background, the candidate set for the bucket by a table
                bws = torch.empty(max(256, binding.batched_workspace_size(batch, p)),
                                  dtype=torch.uint8, device=dev)
                bms = {}
                for prod, sch, band, fr in candidates(prec, N):
                    ents = [
                        {"precision": prec, "n_bucket": bg_bucket[0], "l_bucket": bg_bucket[1],
                         "call": "batched", "products": 4 if prec == "split_bf16x4" else 3,
                         "schedule": "staged", "band": 16, "frame": 1}]
                    ents.append({"precision": prec, "n_bucket": nb, "l_bucket": lb,
                                 "call": "batched", "products": prod, "schedule": sch,
                                 "band": band, "frame": fr})
                    with open(tmp_table, "w") as f:
                        json.dump({"arch": arch, "n_edges": N_EDGES, "l_edges": L_EDGES,
                                   "entries": ents}, f)
                    binding.load_tuning(tmp_table)
                    bms[f"x{prod}/{sch}/{band}/f{fr}"] = time_call(
                        torch, lambda: binding.crmsd_batched(batch, flat, p, out=bout, ws=bws))
                binding.load_tuning(None)
                bbest = min(bms, key=bms.get)
                if default in bms and bms[default] <= bms[bbest] * (1.0 + args.margin):
                    bbest = default
                prod, sch, band, fr = bbest.split("/")
                entries.append({"precision": prec, "n_bucket": nb, "l_bucket": lb,
                                "call": "batched", "N": N, "L": L, "ensembles": k,
                                "background": bg_shapes,
                                "products": int(prod[1:]), "schedule": sch, "band": int(band),
                                "frame": int(fr[1:]), "ms": bms,
                                "batch_pairs_per_s": batch.n_out / (bms[bbest] * 1e-3)})
                log(f"[tune] {prec:13s} N={N:6d} L={L:4d} batched x{k}: {bbest:22s} "
                    f"{bms[bbest]:8.3f} ms")
                del bws
            del x, out, flat, bout
            torch.cuda.empty_cache()
    table = {
        "arch": arch,
        "device": props.name,
        "generator": "paper_1302_4000_amd/tune.py",
        "created": time.strftime("%Y-%m-%d %H:%M:%S UTC", time.gmtime()),
        "tuning_seconds": round(time.time() - t_start, 1),
        "workload": "per bucket: one synthetic ensemble of the representative (N, L), "
                    "sigma ~ U(0.5, 6) A, max(2, N / 400) near-identical models "
                    "(paper_1302_4000_amd.synth.make_ensemble, seed "
                    "7000 + 16 n_bucket + l_bucket); time of the whole all-vs-all call "
                    "(median of 5 samples, HIP events); batched entries: one batched call "
                    "over the background (ensembles of the listed shapes, seeds 9000 + 8 g + m, "
                    "three products in the reference frame) and k = clamp(2e6 / pairs, "
                    "1, 32) ensembles of the bucket (further seeds + 4096 m) under each "
                    "candidate",
        "n_edges": N_EDGES,
        "l_edges": L_EDGES,
        "entries": entries,
    }
    with open(out_path, "w") as f:
        json.dump(table, f, indent=1)
    log(f"[tune] wrote {out_path} ({len(entries)} entries, {table['tuning_seconds']} s)")
    # the library must accept what was written
    binding.load_tuning(out_path)
    return out_path


if __name__ == "__main__":
    main()
