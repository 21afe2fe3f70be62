"""GPU parity of the FP64 fix-up on blocks where nearly every pair is
recomputed (the dense fix-up kernel: models staged in LDS chunk by chunk),
with ragged edges: a last block row/column of 6 models and a last atom chunk
of 13 atoms.  Near-identical models (noise 0.02-0.06 A) put every pair far
below the split-bf16 flag threshold, so every recomputed score must match
the FP64 oracle to FP64 accuracy, in the packed matrix, the cross matrix,
threshold emission and the batched call.  The tests force the configuration
that sends every such pair to the fix-up (three products, no reference
frame): with the frame, or four products, the same pairs are accurate
enough without it.
"""
import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "fp64": 1e-6, "bf16x4": 5e-4}
FP64_TOL = 1e-6      # recomputed pairs (FP64 from the raw coordinates)


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    for p, t in TOL.items():
        m.set_tolerance(p, t)
    m.force_config(3, "staged", 16, 0)
    yield m
    m.force_config(None)


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def near(seed, N, L):
    return synth.make_ensemble(seed, N, L, sigma=(0.02, 0.06))


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
@pytest.mark.parametrize("N,L", [(70, 77), (64, 32), (38, 200)])
def test_dense_blocks_matrix(cl, prec, N, L):
    say(f"[fixup] near-identical N={N} L={L} {prec}")
    x = near(300 + N + L, N, L)
    want = oracle.crmsd_matrix(x)
    assert want.max() < 0.5
    got = cl.crmsd_matrix(dev(x), prec).cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    say(f"  max err {err.max():.3e} A (scores up to {want.max():.3f} A)")
    assert err.max() < FP64_TOL


def test_dense_blocks_cross(cl):
    say("[fixup] near-identical cross 70 x 45, L=77, bf16")
    x = near(401, 115, 77)
    A, B = x[:70], x[70:]
    want = oracle.crmsd_cross(A, B)
    got = cl.crmsd_cross(dev(A), dev(B), "bf16").cpu().numpy().astype(np.float64)
    assert np.abs(got - want).max() < FP64_TOL


def test_dense_blocks_threshold(cl):
    say("[fixup] near-identical threshold N=70 L=77 bf16, cutoff 1 A")
    N = 70
    x = near(402, N, 77)
    want = oracle.crmsd_matrix(x)
    i, j, s, n = cl.crmsd_threshold(dev(x), 1.0, "bf16")
    assert n == N * (N - 1) // 2                 # every pair exactly once
    i, j, s = i.cpu().numpy(), j.cpu().numpy(), s.cpu().numpy().astype(np.float64)
    k = oracle.packed_index(i, j, N)
    assert np.all(i < j) and np.unique(k).size == n
    assert np.abs(s - want[k]).max() < FP64_TOL


def test_dense_blocks_batched(cl):
    ens = [near(403, 70, 77), near(404, 38, 200), synth.make_ensemble(405, 50, 60)]
    say(f"[fixup] batched {[e.shape[:2] for e in ens]} bf16")
    b = cl.Batch([e.shape[:2] for e in ens])
    flat = b.pack([torch.from_numpy(e) for e in ens], "cuda")
    parts = b.split(cl.crmsd_batched(b, flat, "bf16"))
    for e, part in zip(ens, parts):
        want = oracle.crmsd_matrix(e)
        got = part.cpu().numpy().astype(np.float64)
        tol = FP64_TOL if want.max() < 0.5 else TOL["bf16"]
        assert np.abs(got - want).max() < tol, e.shape
        assert torch.equal(cl.crmsd_matrix(dev(e), "bf16").cpu(), part.cpu()), e.shape
