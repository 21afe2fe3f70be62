"""GPU parity of the hand-written backward: against the FP64 oracle's Kabsch
gradient (whose own pins include central finite differences), against FP64
central differences of the oracle's forward (h = 1e-3 A) on 32-model subsets
of the N=4096, L=256 ensemble, on sampled models of the full-size ensemble,
for the many-vs-reference (target) loss, and through torch.autograd."""
import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    return m


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def rel_err(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-30))


@pytest.fixture(scope="module")
def ens():
    x, native = synth.grad_workload()
    return x, native


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp64"])
def test_mean_loss_gradient_subset(cl, ens, prec):
    say(f"[backward] 32-model subset, mean pairwise loss, {prec}")
    x = ens[0][:32]
    N = len(x)
    P = N * (N - 1) // 2
    g = np.full(P, 1.0 / P)
    want = oracle.crmsd_matrix_grad(x, g)
    xd = dev(x)
    out = cl.crmsd_matrix(xd, prec)
    got = cl.crmsd_backward(xd, out, torch.full((P,), 1.0 / P, device="cuda"), prec)
    got = got.cpu().numpy().astype(np.float64)
    e = rel_err(got, want)
    say(f"  max rel err {e:.2e}")
    assert e < (2e-3 if prec == "bf16" else 2e-4)
    assert np.abs(got.sum(1)).max() < 1e-6 * np.abs(want).max() * 256


def test_gradient_matches_finite_differences(cl, ens):
    say("[backward] central differences h=1e-3 of the FP64 oracle forward")
    x = ens[0][32:64].astype(np.float64)
    N = len(x)
    P = N * (N - 1) // 2
    rng = np.random.default_rng(3)
    G = rng.normal(size=P)
    xd = dev(x)
    out = cl.crmsd_matrix(xd, "fp32")
    got = cl.crmsd_backward(xd, out, torch.from_numpy(G.astype(np.float32)).cuda(), "fp32")
    got = got.cpu().numpy().astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    h = 1e-3
    for idx in [(0, 0, 0), (5, 100, 1), (17, 255, 2), (31, 128, 0), (12, 3, 1)]:
        xp, xm = x32.copy(), x32.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.crmsd_matrix(xp) @ G - oracle.crmsd_matrix(xm) @ G) / (2 * h)
        say(f"  {idx}: gpu {got[idx]:+.6e} fd {fd:+.6e}")
        assert abs(got[idx] - fd) < 1e-4 * np.abs(got).max() + 1e-5


def test_full_size_sampled_models(cl, ens):
    say("[backward] N=4096 L=256 mean loss, 8 sampled models")
    x = ens[0]
    N = len(x)
    P = N * (N - 1) // 2
    xd = dev(x)
    out = cl.crmsd_matrix(xd, "fp32")
    grad = cl.crmsd_backward(xd, out, torch.full((P,), 1.0 / P, device="cuda"), "fp32")
    torch.cuda.synchronize()
    rows = np.array([0, 1, 777, 2048, 3001, 4094, 4095, 1234])
    want = oracle.crmsd_matrix_grad_rows(x, np.full(P, 1.0 / P), rows)
    got = grad.cpu().numpy()[rows].astype(np.float64)
    e = rel_err(got, want)
    say(f"  max rel err {e:.2e}")
    assert e < 2e-4


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_target_vs_many_gradient(cl, ens, prec):
    say(f"[backward] target-vs-many N=4096 L=256 {prec}")
    x, native = ens
    N = len(x)
    g = np.full((N, 1), 1.0 / N)
    wantA, wantB = oracle.crmsd_cross_grad(x, native[None], g)
    a, b = dev(x), dev(native[None])
    out = cl.crmsd_cross(a, b, prec)
    ga, gb = cl.crmsd_cross_backward(a, b, out, torch.full((N, 1), 1.0 / N, device="cuda"), prec)
    ea = rel_err(ga.cpu().numpy().astype(np.float64), wantA)
    eb = rel_err(gb.cpu().numpy().astype(np.float64), wantB)
    say(f"  rel err A {ea:.2e} B {eb:.2e}")
    tol = 2e-3 if prec == "bf16" else 2e-4
    assert ea < tol and eb < tol


def test_cross_gradient_rectangular(cl):
    say("[backward] cross 70 x 45, L=33")
    x = synth.make_ensemble(41, 115, 33, sigma=(0.5, 3.0))
    A, B = x[:70], x[70:]
    G = np.random.default_rng(4).normal(size=(70, 45))
    wantA, wantB = oracle.crmsd_cross_grad(A, B, G)
    a, b = dev(A), dev(B)
    out = cl.crmsd_cross(a, b, "fp32")
    ga, gb = cl.crmsd_cross_backward(a, b, out, torch.from_numpy(G.astype(np.float32)).cuda())
    assert rel_err(ga.cpu().numpy().astype(np.float64), wantA) < 2e-4
    assert rel_err(gb.cpu().numpy().astype(np.float64), wantB) < 2e-4


def test_autograd_mean_and_target_loss(cl, ens):
    say("[backward] autograd: mean pairwise + target loss")
    x, native = ens
    x = x[:48]
    N = len(x)
    xd = dev(x).requires_grad_(True)
    ref = dev(native[None])
    loss = cl.crmsd_matrix_ad(xd).mean() + cl.crmsd_cross_ad(xd, ref).mean()
    loss.backward()
    P = N * (N - 1) // 2
    want = oracle.crmsd_matrix_grad(x, np.full(P, 1.0 / P))
    want += oracle.crmsd_cross_grad(x, native[None], np.full((N, 1), 1.0 / N))[0]
    assert rel_err(xd.grad.cpu().numpy().astype(np.float64), want) < 2e-4


def test_zero_and_tiny_ensembles(cl):
    say("[backward] N=1 and N=2")
    x1 = torch.ones(1, 7, 3, device="cuda")
    g = cl.crmsd_backward(x1, torch.empty(0, device="cuda"), torch.empty(0, device="cuda"))
    assert torch.all(g == 0)
    x = synth.make_ensemble(8, 2, 9)
    out = cl.crmsd_matrix(dev(x))
    g = cl.crmsd_backward(dev(x), out, torch.ones(1, device="cuda")).cpu().numpy()
    want = oracle.crmsd_matrix_grad(x, np.ones(1))
    assert rel_err(g.astype(np.float64), want) < 2e-4
