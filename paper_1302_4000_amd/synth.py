"""Seeded synthetic protein-model ensembles.

This module only draws coordinates; it contains none of the cRMSD arithmetic.
Both the HIP path and the FP64 oracle consume what it produces, so it imports
nothing from either.

The paper's workloads are decoy sets of equal-length C-alpha models of one
protein (Results and Discussion: 4state_reduced, vhp_mcmd with 6256 models of
36 residues, I-TASSER sets of 12,500-32,000 models of 60-108 residues; Figure 1
with chains of 71, 215 and 887 residues).  None of those sets is available, so
ensembles of the same shape are generated:

* native: a random walk with 3.8 A steps (the C-alpha virtual-bond length) in
  uniformly random directions, starting at the origin;
* model: native + i.i.d. Gaussian noise with a per-model sigma, then a uniform
  random rotation (Shoemake: a normalised 4-D Gaussian quaternion) and a
  translation drawn from N(0, 20^2) per axis.

Draw order from one ``numpy.random.Generator(PCG64(seed))`` is fixed: native
steps, then per-model sigmas, noise, quaternions, translations (and, where a
workload asks for it, the permutation and fresh walks of unrelated folds).
Generation runs in float64 and is cast to float32 once at the end; float32 is
what the library receives.
"""
from __future__ import annotations

import numpy as np

BOND = 3.8


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_walk(rng, L: int, bond: float = BOND) -> np.ndarray:
    """float64 [L,3] chain with fixed step length ``bond`` and isotropic steps."""
    if L <= 0:
        return np.zeros((0, 3))
    steps = rng.standard_normal((L - 1, 3))
    steps /= np.linalg.norm(steps, axis=1, keepdims=True)
    x = np.zeros((L, 3))
    if L > 1:
        x[1:] = np.cumsum(bond * steps, axis=0)
    return x


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [...,3,3] from unit quaternions [...,4] (w,x,y,z)."""
    w, x, y, z = (q[..., k] for k in range(4))
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_rotations(rng, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return quat_to_rot(q)


def make_ensemble(seed, N: int, L: int, sigma=(0.5, 4.0), *, unrelated_frac: float = 0.0,
                  near_identical: int = 0, near_sigma: float = 0.05,
                  translate: float = 20.0, rng=None) -> np.ndarray:
    """float32 [N,L,3] ensemble of noisy, rigidly moved copies of one native.

    ``near_identical`` models (indices 0..near_identical-1) use ``near_sigma``
    instead of a drawn sigma.  ``unrelated_frac`` of the models (indices chosen
    by a permutation) are replaced by independent random walks that get the
    same rotation and translation as the model they replace and no noise.
    """
    rng = _rng(seed) if rng is None else rng
    native = random_walk(rng, L)
    sig = rng.uniform(sigma[0], sigma[1], size=N)
    if near_identical:
        sig[:near_identical] = near_sigma
    noise = rng.standard_normal((N, L, 3)) * sig[:, None, None]
    R = random_rotations(rng, N)
    t = rng.standard_normal((N, 3)) * translate
    body = native[None] + noise
    n_unrel = int(round(unrelated_frac * N))
    if n_unrel:
        idx = rng.permutation(N)[:n_unrel]
        for k in idx:
            body[k] = random_walk(rng, L)
    x = np.einsum("nab,nlb->nla", R, body) + t[:, None, :]
    return x.astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the paper's ensemble scale (N up to 32,000
# models, L from 36 to 887 residues).
# ---------------------------------------------------------------------------

WORKLOADS = {
    "n200_l100": dict(seed=1, N=200, L=100, sigma=(0.5, 4.0)),
    "n5000_l300": dict(seed=2, N=5000, L=300, sigma=(0.5, 8.0), unrelated_frac=0.10),
    "n20000_l150": dict(seed=3, N=20000, L=150, sigma=(0.5, 4.0), near_identical=50),
    "n4096_l256": dict(seed=5, N=4096, L=256, sigma=(1.0, 4.0)),
}


def workload(name: str, N: int | None = None) -> np.ndarray:
    """Generate a named workload; ``N`` truncates the ensemble (same draws
    only when equal to the full size)."""
    kw = dict(WORKLOADS[name])
    if N is not None:
        kw["N"] = N
    return make_ensemble(**kw)


def grad_workload(N: int | None = None):
    """Ensemble and the float32 native used as the reference of the
    target-vs-many loss."""
    kw = dict(WORKLOADS["n4096_l256"])
    if N is not None:
        kw["N"] = N
    rng = _rng(kw.pop("seed"))
    # the native is the first draw of the same stream that builds the ensemble
    state = rng.bit_generator.state
    native = random_walk(rng, kw["L"]).astype(np.float32)
    rng.bit_generator.state = state
    x = make_ensemble(None, rng=rng, **kw)
    return x, native


def batch_shapes(seed: int = 4, E: int = 64, n_range=(100, 2000), l_range=(50, 500)):
    """Per-ensemble (N, L) drawn log-uniformly, one child seed per ensemble."""
    children = np.random.SeedSequence(seed).spawn(E)
    shapes = []
    for ss in children:
        r = _rng(ss)
        n = int(round(np.exp(r.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        l = int(round(np.exp(r.uniform(np.log(l_range[0]), np.log(l_range[1])))))
        shapes.append((n, l, ss))
    return shapes


def make_batch(seed: int = 4, E: int = 64, n_range=(100, 2000), l_range=(50, 500),
               sigma=(0.5, 6.0), scale_n: float = 1.0):
    """List of float32 ensembles of uneven (N, L).  ``scale_n`` shrinks every
    N (for quick tests) without changing the drawn L."""
    out = []
    for n, l, ss in batch_shapes(seed, E, n_range, l_range):
        r = _rng(ss)
        r.uniform(size=2)  # the two shape draws
        n_eff = max(2, int(round(n * scale_n)))
        out.append(make_ensemble(None, n_eff, l, sigma, rng=r))
    return out
