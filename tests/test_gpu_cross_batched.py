"""GPU parity of the many-vs-reference (cross) and batched entry points
against the FP64 oracle, and consistency with the single-ensemble path."""
import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "fp64": 1e-6}


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    for p, t in TOL.items():
        m.set_tolerance(p, t)
    return m


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp64"])
@pytest.mark.parametrize("Na,Nb,L", [(70, 45, 33), (130, 1, 100), (1, 66, 17), (65, 64, 150)])
def test_cross_matches_oracle(cl, prec, Na, Nb, L):
    say(f"[cross] Na={Na} Nb={Nb} L={L} {prec}")
    x = synth.make_ensemble(77 + L, Na + Nb, L, sigma=(0.3, 4.0))
    A, B = x[:Na], x[Na:]
    want = oracle.crmsd_cross(A, B)
    got = cl.crmsd_cross(dev(A), dev(B), prec).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    assert got.shape == want.shape
    assert np.abs(got - want).max() < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_target_vs_many_n4096_l256(cl, prec):
    say(f"[cross] target-vs-many N=4096 L=256 {prec}")
    x, native = synth.grad_workload()
    got = cl.crmsd_cross(dev(x), dev(native[None]), prec).cpu().numpy()[:, 0].astype(np.float64)
    want = oracle.crmsd_cross(x, native[None])[:, 0]
    assert np.abs(got - want).max() < TOL[prec]


def test_cross_of_a_set_with_itself_matches_matrix(cl):
    say("[cross] self-cross vs packed matrix")
    x = synth.make_ensemble(5, 90, 40)
    C = cl.crmsd_cross(dev(x), dev(x), "fp32").cpu().numpy()
    m = cl.crmsd_matrix(dev(x), "fp32").cpu().numpy()
    I, J = np.triu_indices(90, 1)
    assert np.abs(C[I, J] - m).max() < 2e-4
    assert np.abs(np.diag(C)).max() < 1e-3


def small_batch():
    ens = synth.make_batch(E=16, scale_n=0.06)
    ens += [synth.make_ensemble(9, 1, 30), synth.make_ensemble(10, 2, 1),
            synth.make_ensemble(11, 33, 7), synth.make_ensemble(12, 0, 12)]
    return ens


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp64"])
def test_batched_matches_oracle_and_single_calls(cl, prec):
    ens = small_batch()
    say(f"[batched] {len(ens)} ensembles {[e.shape[:2] for e in ens]} {prec}")
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    out = cl.crmsd_batched(b, flat, prec)
    parts = b.split(out)
    for e, part in zip(ens, parts):
        if e.shape[0] < 2:
            assert part.numel() == 0
            continue
        got = part.cpu().numpy().astype(np.float64)
        want = oracle.crmsd_matrix(e)
        assert np.abs(got - want).max() < TOL[prec], e.shape
        # the same arithmetic as a single call with the configuration the
        # batch gives this ensemble (the table's batched entry)
        c = cl.get_config(e.shape[0], e.shape[1], prec, batched=True)
        cl.force_config(c["products"], c["schedule"], c["band"], c["frame"])
        try:
            single = cl.crmsd_matrix(dev(e), prec).cpu()
        finally:
            cl.force_config(None)
        assert torch.equal(single, part.cpu()), (e.shape, c)


def test_batched_graph_replay_is_stable(cl):
    say("[batched] graph replays")
    ens = synth.make_batch(E=8, scale_n=0.05)
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    ws = torch.empty(cl.batched_workspace_size(b, "bf16"), dtype=torch.uint8, device="cuda")
    out = torch.empty(b.n_out, dtype=torch.float32, device="cuda")
    ref = cl.crmsd_batched(b, flat, "bf16", out=out.clone(), ws=ws).clone()
    for rep in range(4):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        cl.crmsd_batched(b, flat, "bf16", out=out, ws=ws)   # replays the cached graph
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
    # new buffers: the graph is re-captured
    out2 = cl.crmsd_batched(b, flat.clone(), "bf16")
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)


@pytest.fixture(scope="module")
def full_batch():
    """The 64 uneven ensembles of the batched workload at full size (N ~
    logU[100, 2000], L ~ logU[50, 500]) and, per ensemble, a pair sample:
    300 uniform pairs plus its first row and its last column."""
    ens = synth.make_batch()
    rng = np.random.default_rng(23)
    samples = []
    for e in ens:
        n = e.shape[0]
        i = rng.integers(0, n, 300)
        j = rng.integers(0, n, 300)
        k = i != j
        I = np.r_[np.minimum(i, j)[k], np.zeros(n - 1, np.int64), np.arange(n - 1)]
        J = np.r_[np.maximum(i, j)[k], np.arange(1, n), np.full(n - 1, n - 1)]
        samples.append((I, J, oracle.crmsd_pairs(e, I, J)))
    return ens, samples


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp16", "bf16x4"])
def test_batched_full_size_sampled(cl, full_batch, prec):
    """The full 64-ensemble batch under the committed tuning table (its
    ensembles take different kernel configurations) against the oracle on
    each ensemble's pair sample; the longest models (L up to 500) are where
    the contraction error is largest."""
    ens, samples = full_batch
    say(f"[batched] full size: {len(ens)} ensembles, "
        f"N {min(e.shape[0] for e in ens)}..{max(e.shape[0] for e in ens)}, "
        f"L {min(e.shape[1] for e in ens)}..{max(e.shape[1] for e in ens)}, {prec}")
    tol = TOL.get(prec, 5e-4)
    cl.set_tolerance(prec, tol)
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    out = cl.crmsd_batched(b, flat, prec)
    torch.cuda.synchronize()
    worst = 0.0
    for e, (I, J, want), part in zip(ens, samples, b.split(out)):
        got = part[torch.from_numpy(oracle.packed_index(I, J, e.shape[0])).cuda()]
        err = float(np.abs(got.cpu().numpy().astype(np.float64) - want).max())
        worst = max(worst, err)
        assert err < tol, (e.shape, err)
    say(f"  max err {worst:.3e} A over {sum(len(s[0]) for s in samples)} pairs")


def test_cross_index_beyond_2_31(cl):
    """Na = Nb = 47,000: the dense output (2.209e9 scores) runs past 2^31
    elements; sampled against the oracle, including the last row and the row
    that crosses 2^31."""
    Na = Nb = 47000
    L = 4
    say(f"[cross] Na={Na} Nb={Nb} L={L} (dense index beyond 2^31), bf16")
    x = synth.make_ensemble(47, Na + Nb, L, sigma=(0.5, 4.0))
    A, B = x[:Na], x[Na:]
    rng = np.random.default_rng(47)
    ia = rng.integers(0, Na, 20000)
    ib = rng.integers(0, Nb, 20000)
    row = (2 ** 31) // Nb
    ia = np.r_[ia, np.full(Nb, row), np.full(500, Na - 1)]
    ib = np.r_[ib, np.arange(Nb), np.arange(Nb - 500, Nb)]
    k = ia.astype(np.int64) * Nb + ib
    assert k.max() == Na * Nb - 1 and (k >= 2 ** 31).any() and (k < 2 ** 31).any()
    out = cl.crmsd_cross(dev(A), dev(B), "bf16")
    torch.cuda.synchronize()
    assert out.shape == (Na, Nb)
    got = out.reshape(-1)[torch.from_numpy(k).cuda()].cpu().numpy().astype(np.float64)
    del out
    torch.cuda.empty_cache()
    want = oracle.crmsd_pairs(np.concatenate([A, B]), ia, Na + ib)
    err = np.abs(got - want)
    say(f"  {len(k)} pairs, max err {err.max():.3e}")
    assert err.max() < TOL["bf16"]


def test_batched_under_the_callers_graph_capture(cl):
    """A batched call captured into the caller's own graph (after one eager
    call with the same shapes, which caches the plan) replays to the eager
    result, with unrelated eager work between the replays; a shape signature
    with no cached plan is refused under capture (nothing is enqueued)."""
    say("[batched] caller's graph capture")
    ens = small_batch()
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    ws = torch.empty(cl.batched_workspace_size(b, "bf16"), dtype=torch.uint8, device="cuda")
    out = torch.empty(b.n_out, dtype=torch.float32, device="cuda")
    ref = cl.crmsd_batched(b, flat, "bf16", out=out, ws=ws).clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cl.crmsd_batched(b, flat, "bf16", out=out, ws=ws)
    x0 = dev(ens[0])
    for rep in range(4):
        out.fill_(-1.0)
        cl.crmsd_matrix(x0, "fp32")                  # other work on the same device
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
    # new shapes, never planned: refused under capture
    ens2 = [synth.make_ensemble(91, 41, 19), synth.make_ensemble(92, 37, 23)]
    b2 = cl.Batch([e.shape[:2] for e in ens2])
    flat2 = b2.pack([torch.from_numpy(e) for e in ens2], "cuda")
    ws2 = torch.empty(cl.batched_workspace_size(b2, "bf16"), dtype=torch.uint8, device="cuda")
    out2 = torch.empty(b2.n_out, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(cl.binding.ClucsoError):
        with torch.cuda.graph(g2):
            cl.crmsd_batched(b2, flat2, "bf16", out=out2, ws=ws2)
    torch.cuda.synchronize()
    # and works eagerly afterwards
    got = cl.crmsd_batched(b2, flat2, "bf16", out=out2, ws=ws2)
    torch.cuda.synchronize()
    for e, part in zip(ens2, b2.split(got)):
        assert np.abs(part.cpu().numpy().astype(np.float64) - oracle.crmsd_matrix(e)).max() < TOL["bf16"]
