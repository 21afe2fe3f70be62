"""GPU parity of every kernel configuration the tuning table can choose
(products 3 / 4 for split-BF16, staged / persistent schedule, band widths,
reference frame on / off) against the FP64 oracle, for single ensembles, cross comparisons and
batches; a batch whose ensembles take different configurations (mixed
product counts) must equal single calls made under the same table, and a
table's batched entries, where it has them, decide the batch's
configuration."""
import json

import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "bf16x4": 5e-4}
CONFIGS = [(p, s, b, f) for p in (3, 4) for s in ("staged", "persistent") for b in (8, 16, 3)
           for f in (0, 1)]


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    for p, t in TOL.items():
        m.set_tolerance(p, t)
    saved = m.binding.tuning_path()
    yield m
    m.force_config(None)
    m.load_tuning(saved or None)


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def ens_1100():
    x = synth.make_ensemble(4242, 1100, 77, sigma=(0.3, 5.0), near_identical=12)
    return x, oracle.crmsd_matrix(x)


@pytest.mark.parametrize("cfg", CONFIGS, ids=[f"x{p}-{s}-b{b}-f{f}" for p, s, b, f in CONFIGS])
@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_forced_config_all_pairs(cl, ens_1100, cfg, prec):
    if prec == "fp32" and cfg[0] == 4:
        pytest.skip("products apply to split-BF16 only")
    x, want = ens_1100
    say(f"[config] N=1100 L=77 {prec} products={cfg[0]} {cfg[1]} band={cfg[2]} frame={cfg[3]}")
    cl.force_config(*cfg)
    try:
        got = cl.crmsd_matrix(dev(x), prec).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
    finally:
        cl.force_config(None)
    err = np.abs(got - want).max()
    say(f"  max err {err:.3e} A")
    assert err < TOL[prec]


@pytest.mark.parametrize("cfg", [(3, "persistent", 8, 1), (4, "persistent", 16, 0),
                                 (4, "staged", 3, 1), (3, "staged", 16, 1)])
def test_forced_config_cross(cl, cfg):
    say(f"[config] cross Na=200 Nb=97 L=64 bf16 {cfg}")
    x = synth.make_ensemble(515, 297, 64, sigma=(0.3, 4.0))
    A, B = x[:200], x[200:]
    want = oracle.crmsd_cross(A, B)
    cl.force_config(*cfg)
    try:
        got = cl.crmsd_cross(dev(A), dev(B), "bf16").cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
    finally:
        cl.force_config(None)
    assert np.abs(got - want).max() < TOL["bf16"]


def batch():
    ens = synth.make_batch(E=12, scale_n=0.1)
    ens += [synth.make_ensemble(21, 70, 33), synth.make_ensemble(22, 2, 5),
            synth.make_ensemble(23, 1, 9)]
    return ens


def check_batch_against_single(cl, ens, prec):
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    out = cl.crmsd_batched(b, flat, prec)
    torch.cuda.synchronize()
    for e, part in zip(ens, b.split(out)):
        if e.shape[0] < 2:
            continue
        got = part.cpu().numpy().astype(np.float64)
        assert np.abs(got - oracle.crmsd_matrix(e)).max() < TOL[prec], e.shape
        single = cl.crmsd_matrix(dev(e), prec).cpu()
        assert torch.equal(single, part.cpu()), e.shape


@pytest.mark.parametrize("cfg", [(3, "staged", 16, 1), (4, "staged", 8, 0),
                                 (3, "persistent", 16, 1), (4, "persistent", 3, 1),
                                 (3, "staged", 16, 0)])
@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_forced_config_batch(cl, cfg, prec):
    if prec == "fp32" and cfg[0] == 4:
        pytest.skip("products apply to split-BF16 only")
    ens = batch()
    say(f"[config] batch of {len(ens)} {prec} {cfg}")
    cl.force_config(*cfg)
    try:
        check_batch_against_single(cl, ens, prec)
    finally:
        cl.force_config(None)


def test_mixed_table_batch(cl, tmp_path):
    """A table that gives short models three products and long ones four,
    the staged schedule with the reference frame to two buckets and the
    persistent one (no frame) to the rest: one batch then mixes both product
    counts, and most of its work prefers the persistent schedule, which the
    framed ensembles rule out; every ensemble must equal its single call
    under the same table (the batch's schedule never changes an ensemble's
    arithmetic)."""
    entries = []
    for nb in range(3):
        for lb in range(3):
            entries.append({"precision": "split_bf16", "n_bucket": nb, "l_bucket": lb,
                            "products": 4 if lb >= 1 else 3,
                            "schedule": "staged" if nb == lb < 2 else "persistent",
                            "band": [16, 8, 3][lb], "frame": 1})
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    p = tmp_path / "mixed.json"
    p.write_text(json.dumps({"arch": arch, "n_edges": [2, 64, 160], "l_edges": [1, 60, 200],
                             "entries": entries}))
    saved = cl.binding.tuning_path()
    cl.load_tuning(str(p))
    try:
        ens = batch()
        cfgs = [cl.get_config(e.shape[0], e.shape[1], "bf16") for e in ens if e.shape[0] > 1]
        kinds = {c["products"] for c in cfgs}
        say(f"[config] mixed-table batch of {len(ens)}: product counts {sorted(kinds)}")
        assert kinds == {3, 4}
        assert {(c["schedule"], c["frame"]) for c in cfgs} == {("staged", 1), ("persistent", 0)}
        check_batch_against_single(cl, ens, "bf16")
    finally:
        cl.load_tuning(saved or None)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batched_table_entries(cl, tmp_path, prec):
    """A table whose batched entries differ from its single-call entries
    (single calls: four products without the reference frame; ensembles in
    a batched call: three products with it): the batch follows the batched
    entries — each ensemble equals a single call forced to its batched
    configuration, and at least one differs from its single call under the
    table (so the batched entries took effect) — and matches the oracle."""
    name = {"bf16": "split_bf16", "fp32": "fp32"}[prec]
    entries = []
    for nb in range(3):
        for lb in range(3):
            entries.append({"precision": name, "n_bucket": nb, "l_bucket": lb, "products": 4,
                            "schedule": "staged", "band": 8, "frame": 0})
            entries.append({"precision": name, "n_bucket": nb, "l_bucket": lb, "products": 3,
                            "schedule": "staged", "band": 16, "frame": 1, "call": "batched"})
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    p = tmp_path / "batched.json"
    p.write_text(json.dumps({"arch": arch, "n_edges": [2, 64, 160], "l_edges": [1, 60, 200],
                             "entries": entries}))
    saved = cl.binding.tuning_path()
    cl.load_tuning(str(p))
    try:
        ens = [e for e in batch() if e.shape[0] > 1]
        say(f"[config] batched-entry table, batch of {len(ens)} {prec}")
        b = cl.Batch([e.shape[:2] for e in ens])
        flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
        out = cl.crmsd_batched(b, flat, prec)
        torch.cuda.synchronize()
        differs = 0
        for e, part in zip(ens, b.split(out)):
            cb = cl.get_config(e.shape[0], e.shape[1], prec, batched=True)
            cs = cl.get_config(e.shape[0], e.shape[1], prec)
            assert (cb["band"], cb["frame"]) == (16, 1) and (cs["band"], cs["frame"]) == (8, 0)
            got = part.cpu()
            assert np.abs(got.numpy().astype(np.float64) - oracle.crmsd_matrix(e)).max() < TOL[prec]
            cl.force_config(cb["products"], cb["schedule"], cb["band"], cb["frame"])
            try:
                forced = cl.crmsd_matrix(dev(e), prec).cpu()
            finally:
                cl.force_config(None)
            assert torch.equal(forced, got), e.shape
            differs += not torch.equal(cl.crmsd_matrix(dev(e), prec).cpu(), got)
        assert differs > 0
    finally:
        cl.load_tuning(saved or None)
