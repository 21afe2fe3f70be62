"""GPU parity of the threshold emission (pairs within a cRMSD cutoff) against
the FP64 oracle and against the stored all-vs-all scores."""
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


def as_set(i, j):
    return set(zip(i.cpu().numpy().tolist(), j.cpu().numpy().tolist()))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp64"])
def test_threshold_matches_oracle(cl, prec):
    say(f"[threshold] N=200 L=100 {prec}")
    x = synth.workload("n200_l100")
    N = len(x)
    ref = oracle.crmsd_matrix(x)
    cutoff = float(np.median(ref))
    I, J = np.triu_indices(N, 1)
    i, j, s, n = cl.crmsd_threshold(torch.from_numpy(x).cuda(), cutoff, prec)
    got = as_set(i, j)
    assert len(got) == n == i.numel()                     # no duplicates
    tol = TOL[prec]
    sure_in = {(a, b) for a, b, r in zip(I, J, ref) if r < cutoff - tol}
    maybe = {(a, b) for a, b, r in zip(I, J, ref) if abs(r - cutoff) <= tol}
    assert sure_in <= got and got <= sure_in | maybe
    k = oracle.packed_index(i.cpu().numpy(), j.cpu().numpy(), N)
    assert np.abs(s.cpu().numpy() - ref[k]).max() < tol
    assert np.all(i.cpu().numpy() < j.cpu().numpy())


def test_threshold_equals_stored_scores_at_scale(cl):
    say("[threshold] N=20000 L=150 bf16 cutoff 3.2 A vs the packed matrix")
    x = torch.from_numpy(synth.workload("n20000_l150")).cuda()
    full = cl.crmsd_matrix(x, "bf16")
    below = (full < 3.2).nonzero().squeeze(1)
    i, j, s, n = cl.crmsd_threshold(x, 3.2, "bf16")
    say(f"  {n} pairs below 3.2 A, matrix has {below.numel()}")
    N = 20000
    k = (i.long() * (2 * N - i.long() - 1)) // 2 + j.long() - i.long() - 1
    assert torch.all(i < j)
    assert torch.unique(k).numel() == n
    assert float((full[k] - s).abs().max()) < 1e-5
    diff = abs(n - below.numel())
    near = int(((full - 3.2).abs() < 1e-5).sum())
    assert diff <= near


def test_threshold_capacity_and_empty(cl):
    say("[threshold] capacity overflow, N < 2")
    x = torch.from_numpy(synth.workload("n200_l100")).cuda()
    i, j, s, n = cl.crmsd_threshold(x, 1e9, "fp32", capacity=1000)
    assert n == 200 * 199 // 2 and i.numel() == 1000
    ref = oracle.crmsd_matrix(synth.workload("n200_l100"))
    k = oracle.packed_index(i.cpu().numpy(), j.cpu().numpy(), 200)
    assert np.abs(s.cpu().numpy() - ref[k]).max() < 1e-4
    _, _, _, n0 = cl.crmsd_threshold(x, 0.0, "fp32")
    assert n0 == 0
    _, _, _, n1 = cl.crmsd_threshold(x[:1], 5.0, "fp32")
    assert n1 == 0
