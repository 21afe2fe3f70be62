"""Calibration of the fix-up's error model against the FP64 oracle.

With the fix-up disabled (tolerance 0) every score comes straight from the
FP32-accumulated contraction and the FP64 Eq. 2 epilogue.  The library
assumes (clusco_flag_epsilon) that a pair's score error is at most
    (eps (W_i + W_j) + 2e-10 (E_i + E_j)) / (L s),
s the oracle's cRMSD, E = L R^2 the radii and W the squared size of what the
MFMAs contracted: the centred model (W = E) without the reference frame, its
residual from the reference after optimal superposition with it.  The latter
is W_i = L cRMSD(model i, reference)^2 by Eq. 1, with the reference the
ensemble's first model, so the oracle gives it too.  Besides, the operands
carry the contracted vectors rounded to the precision's representation
(relative error u = 2^-24 in FP32, 2^-22 for the FP16 hi + lo split, 2^-18
for BF16 hi + lo), so the GPU scores models moved by at most u |v| per
coordinate; cRMSD then moves by at most the RMS of those moves,
u (sqrt(W_i / L) + sqrt(W_j / L)), a floor that does not grow as s -> 0.
For each precision, model length and frame setting the test checks, on
sampled pairs,
  * that every sampled error is within the bound plus that floor (the
    model's coefficients sit a margin above the measured maxima), and
  * the guarantee the fix-up relies on: every pair the flag would leave alone
    (bound below tol / 2) has a raw error below tol / 2.
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
EPS_E = 2e-10
UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -18, "fp16": 2.0 ** -22, "bf16x4": 2.0 ** -18}


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    yield m
    m.force_config(None)
    for p, t in TOL.items():
        m.set_tolerance(p, t)


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


def raw_scores(cl, xd, prec, I, J, frame):
    """Scores of the sampled pairs with the fix-up off, under the staged
    schedule with the given frame setting."""
    N = xd.shape[0]
    cl.set_tolerance(prec, 0.0)
    cl.force_config(4 if prec == "bf16x4" else 3, "staged", 16, frame)
    try:
        out = cl.crmsd_matrix(xd, prec)
        got = out[torch.from_numpy(oracle.packed_index(I, J, N)).cuda()].cpu().numpy()
    finally:
        cl.force_config(None)
        cl.set_tolerance(prec, TOL[prec])
    return got.astype(np.float64)


@pytest.mark.parametrize("L", [150, 300, 500])
@pytest.mark.parametrize("aligned", [False, True], ids=["random_frames", "pre_aligned"])
def test_error_model(cl, L, aligned):
    x = ensemble(L, aligned)
    N = x.shape[0]
    I, J = sample_pairs(N, L)
    s = oracle.crmsd_pairs(x, I, J)
    c = x.astype(np.float64) - x.astype(np.float64).mean(1, keepdims=True)
    E = (c * c).sum((1, 2))
    # residual size in the reference frame: L cRMSD(model, model 0)^2
    to_ref = oracle.crmsd_pairs(x, np.zeros(N, np.int64), np.arange(N))
    Wf = L * to_ref ** 2
    xd = torch.from_numpy(x).cuda()
    for frame, W in ((0, E), (1, Wf)):
        for prec, tol in TOL.items():
            say(f"[error model] L={L} {'pre-aligned' if aligned else 'random frames'} "
                f"{prec} frame={frame}")
            got = raw_scores(cl, xd, prec, I, J, frame)
            err = np.abs(got - s)
            eps = cl.binding.flag_epsilon(prec, L)
            bound = (eps * (W[I] + W[J]) + EPS_E * (E[I] + E[J])) / (L * s)
            floor = UNIT[prec] * (np.sqrt(W[I] / L) + np.sqrt(W[J] / L))
            ratio = err / (bound + floor)
            unflagged = bound <= tol / 2
            worst = float(err[unflagged].max()) if unflagged.any() else 0.0
            say(f"  max err {err.max():.3g} A, max err / (bound + floor) {ratio.max():.2f}, "
                f"flagged {int((~unflagged).sum())}/{len(s)}, max raw err of unflagged "
                f"{worst:.3g} A (tol {tol:g})")
            assert ratio.max() <= 1.0, (prec, L, frame, ratio.max())
            assert worst <= tol / 2, (prec, L, frame, worst)
