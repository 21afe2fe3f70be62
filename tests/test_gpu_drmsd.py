"""GPU parity of the all-vs-all dRMSD (Algorithms, Eq. 5) against the FP64
oracle, element by element on small ensembles (several 128-model tiles and a
ragged tail) and on sampled pairs at N=20000, L=150.  Tolerances (A, max
absolute error) are the per-precision ones of include/clusco.h."""
import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "fp64": 1e-6, "bf16x4": 5e-4}


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


def run(cl, x, prec):
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    out = cl.drmsd_matrix(xd, prec)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x4", "fp64"])
def test_n300_l60_all_pairs(cl, prec):
    say(f"[drmsd] N=300 L=60 all pairs, {prec}")
    x = synth.make_ensemble(11, 300, 60, sigma=(0.3, 5.0))
    want = oracle.drmsd_matrix(x)
    got = run(cl, x, prec).cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    say(f"  max err {err.max():.3e} A, mean {err.mean():.3e}")
    assert err.max() < TOL[prec]


@pytest.mark.parametrize("N,L", [(2, 2), (3, 3), (5, 7), (33, 17), (65, 33), (77, 5),
                                 (129, 64), (130, 100), (257, 23), (40, 160), (37, 161),
                                 (70, 230)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ragged_shapes(cl, N, L, prec):
    say(f"[drmsd] ragged N={N} L={L} {prec}")
    x = synth.make_ensemble(2000 + N + L, N, L, sigma=(0.3, 5.0))
    want = oracle.drmsd_matrix(x)
    got = run(cl, x, prec).cpu().numpy().astype(np.float64)
    assert got.shape == want.shape
    assert np.abs(got - want).max() < TOL[prec]


def test_single_atom_and_tiny(cl):
    say("[drmsd] L=1 gives zeros; N in {0, 1} gives nothing")
    x = torch.randn(40, 1, 3, device="cuda")
    assert torch.count_nonzero(cl.drmsd_matrix(x)).item() == 0
    for N in (0, 1):
        assert cl.drmsd_matrix(torch.zeros(N, 10, 3, device="cuda")).numel() == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x4"])
def test_degenerate_models(cl, prec):
    say(f"[drmsd] degenerate models {prec}")
    rng = np.random.default_rng(0)
    L = 40
    A = synth.random_walk(rng, L)
    R = synth.random_rotations(rng, 4)
    flip = np.diag([1.0, 1.0, -1.0])
    t = rng.normal(0, 4, L)
    models = [A, A.copy(), A @ R[0].T + 3.0,           # identical and rigid copies: 0
              A @ flip, A @ flip @ R[1].T,              # mirror images: 0 as well
              t[:, None] * np.array([1.0, 0, 0]),       # collinear
              A + rng.normal(0, 0.01, A.shape),         # near-identical
              A + rng.normal(0, 0.001, A.shape),
              1.5 * A,                                  # scaled
              np.zeros((L, 3)) + 5.0]                   # a single point repeated
    x = np.stack(models).astype(np.float32)
    want = oracle.drmsd_matrix(x)
    got = run(cl, x, prec).cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    say(f"  max err {err.max():.3e}")
    assert err.max() < TOL[prec]


def test_deterministic(cl):
    say("[drmsd] determinism N=300 L=50")
    x = synth.make_ensemble(5, 300, 50)
    assert torch.equal(run(cl, x, "bf16").cpu(), run(cl, x, "bf16").cpu())


def random_pairs(rng, N, n):
    i = rng.integers(0, N, n)
    j = rng.integers(0, N, n)
    keep = i != j
    return np.minimum(i, j)[keep], np.maximum(i, j)[keep]


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_n20000_l150_sampled(cl, prec):
    say(f"[drmsd] N=20000 L=150 sampled, {prec}")
    x = synth.workload("n20000_l150")
    out = run(cl, x, prec)
    rng = np.random.default_rng(3)
    I, J = random_pairs(rng, 20000, 20000)
    ii, jj = np.triu_indices(50, 1)                     # the near-identical group
    I = np.r_[I, ii, np.zeros(199, np.int64), np.arange(19800, 19999)]
    J = np.r_[J, jj, np.arange(1, 200), np.full(199, 19999)]
    k = torch.from_numpy(oracle.packed_index(I, J, 20000)).cuda()
    got = out[k].cpu().numpy().astype(np.float64)
    want = oracle.drmsd_pairs(x, I, J)
    err = np.abs(got - want)
    say(f"  {len(I)} pairs, max err {err.max():.3e} A at oracle {want[int(np.argmax(err))]:.3f} A")
    assert err.max() < TOL[prec]
    assert torch.isfinite(out).all()
