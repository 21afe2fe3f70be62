"""Calibration of the fix-up's error model against the FP64 oracle.

With the fix-up disabled (tolerance 0) every score comes straight from the
FP32-accumulated contraction and the FP64 Eq. 2 epilogue.  For each precision
and model length the test measures, on sampled pairs,
    eff = |s_gpu - s| * s * L / (E_i + E_j)
(s the oracle's cRMSD, E = L R^2 the radii), the quantity the error model
bounds by eps(precision, L) (clusco_flag_epsilon), and checks
  * eff <= eps for every sampled pair (the model's coefficients sit a margin
    above the measured maxima), and
  * the guarantee the fix-up relies on: every pair the flag would leave alone
    (s >= 2 eps (E_i + E_j) / (L tol)) has a raw error below tol / 2.
Ensembles: random frames (the workload generator) and pre-aligned copies of
one native (the split's rounding residuals of two models then correlate),
each with 50 near-identical models, at L = 150, 300 and 500."""
import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "bf16x4": 5e-4}


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    return m


def say(*a):
    print(*a, flush=True)


def ensemble(L, aligned, N=1024):
    seed = 900 + L + (1 if aligned else 0)
    if not aligned:
        return synth.make_ensemble(seed, N, L, sigma=(0.5, 6.0), near_identical=50)
    rng = np.random.Generator(np.random.PCG64(seed))
    native = synth.random_walk(rng, L) + 17.0          # one frame, off the origin
    sig = rng.uniform(0.5, 6.0, N)
    sig[:50] = 0.05
    return (native[None] + rng.standard_normal((N, L, 3)) * sig[:, None, None]).astype(np.float32)


def sample_pairs(N, seed):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, N, 20000)
    j = rng.integers(0, N, 20000)
    k = i != j
    I, J = np.minimum(i, j)[k], np.maximum(i, j)[k]
    ii, jj = np.triu_indices(50, 1)
    I2 = rng.integers(0, 50, 4000)
    J2 = rng.integers(50, N, 4000)
    return np.r_[I, ii, I2], np.r_[J, jj, J2]


def measure(cl, x, prec):
    """(eff, err, s, Esum) over the sample with the fix-up off."""
    N, L = x.shape[0], x.shape[1]
    I, J = sample_pairs(N, L)
    s = oracle.crmsd_pairs(x, I, J)
    c = x.astype(np.float64) - x.astype(np.float64).mean(1, keepdims=True)
    E = (c * c).sum((1, 2))
    xd = torch.from_numpy(x).cuda()
    cl.set_tolerance(prec, 0.0)
    try:
        out = cl.crmsd_matrix(xd, prec)
        got = out[torch.from_numpy(oracle.packed_index(I, J, N)).cuda()].cpu().numpy()
    finally:
        cl.set_tolerance(prec, TOL[prec])
    err = np.abs(got.astype(np.float64) - s)
    Es = E[I] + E[J]
    return err * s * L / Es, err, s, Es


@pytest.mark.parametrize("L", [150, 300, 500])
@pytest.mark.parametrize("aligned", [False, True], ids=["random_frames", "pre_aligned"])
def test_error_model(cl, L, aligned):
    x = ensemble(L, aligned)
    for prec, tol in TOL.items():
        say(f"[error model] L={L} {'pre-aligned' if aligned else 'random frames'} {prec}")
        eff, err, s, Es = measure(cl, x, prec)
        eps = cl.binding.flag_epsilon(prec, L)
        unflagged = s >= 2.0 * eps * Es / (L * tol)
        worst = float(err[unflagged].max()) if unflagged.any() else 0.0
        say(f"  max eff {eff.max():.3g}  eps {eps:.3g}  ratio {eff.max() / eps:.2f}  "
            f"max raw err of unflagged pairs {worst:.3g} A (tol {tol:g})")
        assert eff.max() <= eps, (prec, L, eff.max(), eps)
        assert worst <= tol / 2, (prec, L, worst)
