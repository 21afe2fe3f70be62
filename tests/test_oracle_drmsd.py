"""Pins for the oracle's dRMSD (Algorithms, Eq. 5) that do not rely on the
oracle itself: closed forms for two atoms and for evenly spaced collinear
chains, invariance under rigid motion and under reflection (the distance
matrix loses chirality, as the paper notes), scale covariance, the bound
dRMSD <= 2 cRMSD against the independently pinned cRMSD oracle, and a
brute-force loop over atom pairs written with numpy's pairwise distances."""
import numpy as np
import pytest

from paper_1302_4000_amd import synth


@pytest.fixture(scope="module")
def ens():
    return synth.make_ensemble(51, 16, 29, sigma=(0.3, 3.0)).astype(np.float64)


def test_two_atoms(orc):
    rng = np.random.default_rng(0)
    for _ in range(10):
        A, B = rng.normal(0, 4, (2, 3)), rng.normal(0, 4, (2, 3))
        dA, dB = np.linalg.norm(A[1] - A[0]), np.linalg.norm(B[1] - B[0])
        assert abs(orc.drmsd(A, B) - abs(dA - dB)) < 1e-12


@pytest.mark.parametrize("L", [3, 10, 57])
def test_evenly_spaced_collinear(orc, L):
    """d_ij = |i-j| s, so dRMSD = |sA - sB| sqrt(L(L+1)/6)
    (sum_{i<j} (j-i)^2 = L^2 (L^2-1) / 12)."""
    rng = np.random.default_rng(L)
    u, v = rng.normal(size=3), rng.normal(size=3)
    u /= np.linalg.norm(u)
    v /= np.linalg.norm(v)
    sA, sB = 3.8, 3.1
    A = np.arange(L)[:, None] * sA * u + 5.0
    B = np.arange(L)[:, None] * sB * v - 2.0
    assert abs(orc.drmsd(A, B) - abs(sA - sB) * np.sqrt(L * (L + 1) / 6.0)) < 1e-11


def test_rigid_motion_and_reflection_invariance(orc, ens):
    rng = np.random.default_rng(1)
    R = synth.random_rotations(rng, 2)
    flip = np.diag([1.0, 1.0, -1.0])
    for i, j in [(0, 1), (3, 9), (4, 15)]:
        r0 = orc.drmsd(ens[i], ens[j])
        assert abs(orc.drmsd(ens[i] @ R[0].T + 7.0, ens[j]) - r0) < 1e-11
        assert abs(orc.drmsd(ens[i], ens[j] @ flip @ R[1].T) - r0) < 1e-11
    A = synth.random_walk(np.random.default_rng(5), 30)
    assert orc.drmsd(A, A @ flip) < 1e-12          # chirality-blind
    assert orc.crmsd(A, A @ flip) > 0.5            # unlike cRMSD


def test_symmetry_scale_and_zero(orc, ens):
    assert orc.drmsd(ens[2], ens[2]) == 0.0
    assert abs(orc.drmsd(ens[2], ens[5]) - orc.drmsd(ens[5], ens[2])) < 1e-13
    for c in (0.5, 4.0):
        assert abs(orc.drmsd(c * ens[2], c * ens[5]) - c * orc.drmsd(ens[2], ens[5])) < 1e-11
    assert orc.drmsd(np.ones((1, 3)), np.zeros((1, 3))) == 0.0


def test_bounded_by_twice_crmsd(orc, ens):
    """|d^A_ij - d^B_ij| <= |delta_i| + |delta_j| after superposition, so
    dRMSD^2 <= 4 cRMSD^2."""
    for i in range(len(ens)):
        for j in range(i + 1, len(ens), 3):
            assert orc.drmsd(ens[i], ens[j]) <= 2.0 * orc.crmsd(ens[i], ens[j]) + 1e-12


def test_bruteforce_pairwise_distances(orc, ens):
    from scipy.spatial.distance import pdist
    for i, j in [(0, 7), (8, 11), (12, 13)]:
        dA, dB = pdist(ens[i]), pdist(ens[j])
        want = np.sqrt(np.mean((dA - dB) ** 2))
        assert abs(orc.drmsd(ens[i], ens[j]) - want) < 1e-12


def test_matrix_and_pairs_agree(orc, ens):
    m = orc.drmsd_matrix(ens)
    I, J = np.triu_indices(len(ens), 1)
    assert np.array_equal(orc.drmsd_pairs(ens, I, J), m)
    assert m[orc.packed_index(3, 9, len(ens))] == orc.drmsd(ens[3], ens[9])
