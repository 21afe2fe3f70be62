"""Pins for the oracle's contact map overlap (Algorithms, Eq. 6-7): worked
collinear examples (the Sorensen index by hand), the strict cut-off, invariance
under rigid motion and reflection (contacts are distances), symmetry and the
0..100 range, the no-contact reading, and SciPy's pdist as a brute-force
contact source."""
import numpy as np
import pytest

from paper_1302_4000_amd import synth


def line(n, s):
    return np.arange(n)[:, None] * np.array([s, 0.0, 0.0])


def test_worked_examples(orc):
    # spacing 5, cut-off 6: contacts (0,1) (1,2) (2,3) -> n = 3
    # spacing 2.5: adds (0,2) (1,3) at 5.0 -> n = 5, shared 3: S = 100 * 6 / 8
    assert orc.cmo(line(4, 5.0), line(4, 2.5), 6.0) == 75.0
    # spacing 3: (0,2) and (1,3) sit exactly at 6.0, not below it -> identical maps
    assert orc.cmo(line(4, 5.0), line(4, 3.0), 6.0) == 100.0
    # disjoint contact sets: A has only (0,1), B only (2,3)
    A = np.array([[0, 0, 0], [1, 0, 0], [20, 0, 0], [40, 0, 0.0]])
    B = np.array([[0, 0, 0], [20, 0, 0], [40, 0, 0], [41, 0, 0.0]])
    assert orc.cmo(A, B, 2.0) == 0.0
    # no contacts anywhere: 0 by the reading of 0 / 0
    assert orc.cmo(line(5, 10.0), line(5, 12.0), 3.0) == 0.0
    assert orc.cmo(line(1, 1.0), line(1, 1.0), 3.0) == 0.0


def test_rigid_motion_reflection_symmetry(orc):
    x = synth.make_ensemble(3, 12, 40, sigma=(0.5, 3.0)).astype(np.float64)
    R = synth.random_rotations(np.random.default_rng(2), 2)
    flip = np.diag([1.0, 1.0, -1.0])
    for c in (4.0, 8.0, 12.0):
        for i, j in [(0, 1), (2, 7), (5, 11)]:
            s = orc.cmo(x[i], x[j], c)
            assert 0.0 <= s <= 100.0
            assert orc.cmo(x[j], x[i], c) == s
            assert orc.cmo(x[i] @ R[0].T + 9.0, x[j] @ flip @ R[1].T, c) == pytest.approx(s, abs=1e-12)
        assert orc.cmo(x[3], x[3], c) == 100.0


def test_bruteforce_pdist(orc):
    from scipy.spatial.distance import pdist
    x = synth.make_ensemble(4, 10, 37, sigma=(0.5, 4.0)).astype(np.float64)
    for c in (5.0, 8.0):
        for i, j in [(0, 1), (2, 9), (4, 6)]:
            a, b = pdist(x[i]) < c, pdist(x[j]) < c
            want = 200.0 * np.sum(a & b) / (a.sum() + b.sum())
            assert orc.cmo(x[i], x[j], c) == pytest.approx(want, abs=1e-12)


def test_matrix_and_pairs_agree(orc):
    x = synth.make_ensemble(6, 20, 25).astype(np.float64)
    m = orc.cmo_matrix(x, 8.0)
    I, J = np.triu_indices(20, 1)
    assert np.array_equal(orc.cmo_pairs(x, I, J, 8.0), m)
    assert m[orc.packed_index(3, 9, 20)] == orc.cmo(x[3], x[9], 8.0)
