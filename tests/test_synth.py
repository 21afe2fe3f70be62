"""Seeded input generator: determinism, chain geometry, workload shapes."""
import numpy as np

from paper_1302_4000_amd import synth


def test_deterministic_per_seed():
    a = synth.make_ensemble(7, 10, 20)
    b = synth.make_ensemble(7, 10, 20)
    c = synth.make_ensemble(8, 10, 20)
    assert a.dtype == np.float32 and a.shape == (10, 20, 3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_native_steps_are_bond_length():
    x = synth.random_walk(np.random.default_rng(0), 200)
    d = np.linalg.norm(np.diff(x, axis=0), axis=1)
    assert np.allclose(d, 3.8, atol=1e-12)


def test_noise_level_and_rigid_motion():
    # sigma=0 gives rigid copies: every intra-model distance equals the native's
    x = synth.make_ensemble(3, 5, 30, sigma=(0.0, 0.0)).astype(np.float64)
    D = lambda m: np.linalg.norm(m[:, None] - m[None], axis=-1)
    for k in range(1, 5):
        assert np.abs(D(x[k]) - D(x[0])).max() < 1e-3


def test_near_identical_and_unrelated():
    x = synth.make_ensemble(3, 60, 40, near_identical=5, near_sigma=0.0).astype(np.float64)
    D = lambda m: np.linalg.norm(m[:, None] - m[None], axis=-1)
    assert np.abs(D(x[1]) - D(x[0])).max() < 1e-3
    y = synth.make_ensemble(2, 50, 40, unrelated_frac=0.1)
    assert y.shape == (50, 40, 3)


def test_batch_shapes_in_range():
    shapes = synth.batch_shapes()
    assert len(shapes) == 64
    for n, l, _ in shapes:
        assert 100 <= n <= 2000 and 50 <= l <= 500
    b = synth.make_batch(scale_n=0.05)
    assert [e.shape[1] for e in b] == [l for _, l, _ in shapes]


def test_grad_workload_native():
    x, nat = synth.grad_workload(8)
    assert x.shape == (8, 256, 3) and nat.shape == (256, 3) and nat.dtype == np.float32
    d = np.linalg.norm(np.diff(nat.astype(np.float64), axis=0), axis=1)
    assert np.allclose(d, 3.8, atol=1e-5)
