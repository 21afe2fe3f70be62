"""Pins for the oracle's gradient of cRMSD: FP64 central finite differences
of the oracle's own forward value (h = 1e-3 A and smaller), translation
invariance (the gradient sums to zero over atoms), rotation invariance (zero
net torque), and the packed / cross reductions against per-pair sums."""
import numpy as np
import pytest

from paper_1302_4000_amd import synth


def fd_grad(f, x, h):
    g = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        g[idx] = (f(xp) - f(xm)) / (2 * h)
    return g


@pytest.fixture(scope="module")
def pair():
    x = synth.make_ensemble(21, 2, 17, sigma=(1.0, 3.0)).astype(np.float64)
    return x[0], x[1]


def test_pair_gradient_matches_central_differences(orc, pair):
    A, B = pair
    r, gA, gB = orc.crmsd_grad_pair(A, B)
    for h in (1e-3, 1e-4):
        fA = fd_grad(lambda a: orc.crmsd(a, B), A, h)
        fB = fd_grad(lambda b: orc.crmsd(A, b), B, h)
        assert np.abs(fA - gA).max() < 50 * h * h + 1e-8
        assert np.abs(fB - gB).max() < 50 * h * h + 1e-8


def test_gradient_invariants(orc, pair):
    A, B = pair
    r, gA, gB = orc.crmsd_grad_pair(A, B)
    assert np.abs(gA.sum(0)).max() < 1e-13          # translation invariance
    assert np.abs(gB.sum(0)).max() < 1e-13
    a = A - A.mean(0)
    b = B - B.mean(0)
    assert np.abs(np.cross(a, gA).sum(0)).max() < 1e-12   # rotation invariance
    assert np.abs(np.cross(b, gB).sum(0)).max() < 1e-12
    # Euler: cRMSD is 1-homogeneous in the pair of centred models
    assert abs((a * gA).sum() + (b * gB).sum() - r) < 1e-12


def test_gradient_of_identical_pair_is_zero(orc, pair):
    A, _ = pair
    r, gA, gB = orc.crmsd_grad_pair(A, A)
    assert r < 1e-12
    assert np.abs(gA).max() < 1e-6 and np.abs(gB).max() < 1e-6


def test_matrix_gradient_is_sum_of_pair_gradients(orc):
    x = synth.make_ensemble(22, 7, 11, sigma=(0.5, 3.0)).astype(np.float64)
    N = len(x)
    rng = np.random.default_rng(0)
    g = rng.normal(size=N * (N - 1) // 2)
    got = orc.crmsd_matrix_grad(x, g)
    want = np.zeros_like(x)
    k = 0
    for i in range(N):
        for j in range(i + 1, N):
            _, gA, gB = orc.crmsd_grad_pair(x[i], x[j])
            want[i] += g[k] * gA
            want[j] += g[k] * gB
            k += 1
    assert np.abs(got - want).max() < 1e-12


def test_matrix_gradient_fd_on_mean_loss(orc):
    """loss = mean over pairs; FD on a few coordinates of a small ensemble."""
    x = synth.make_ensemble(23, 6, 9, sigma=(0.5, 3.0)).astype(np.float64)
    N = len(x)
    P = N * (N - 1) // 2
    g = np.full(P, 1.0 / P)
    G = orc.crmsd_matrix_grad(x, g)
    h = 1e-4
    for idx in [(0, 0, 0), (3, 4, 2), (5, 8, 1), (2, 1, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (orc.crmsd_matrix(xp).mean() - orc.crmsd_matrix(xm).mean()) / (2 * h)
        assert abs(fd - G[idx]) < 1e-8


def test_cross_gradient_is_sum_of_pair_gradients(orc):
    x = synth.make_ensemble(24, 5, 13, sigma=(0.5, 3.0)).astype(np.float64)
    A, B = x[:3], x[3:]
    g = np.random.default_rng(1).normal(size=(3, 2))
    gA, gB = orc.crmsd_cross_grad(A, B, g)
    wA, wB = np.zeros_like(A), np.zeros_like(B)
    for i in range(3):
        for j in range(2):
            _, a, b = orc.crmsd_grad_pair(A[i], B[j])
            wA[i] += g[i, j] * a
            wB[j] += g[i, j] * b
    assert np.abs(gA - wA).max() < 1e-12 and np.abs(gB - wB).max() < 1e-12


def test_matrix_gradient_rows_match_full(orc):
    x = synth.make_ensemble(25, 9, 12, sigma=(0.5, 3.0)).astype(np.float64)
    N = len(x)
    g = np.random.default_rng(2).normal(size=N * (N - 1) // 2)
    full = orc.crmsd_matrix_grad(x, g)
    rows = np.array([0, 4, 8, 4])
    assert np.abs(orc.crmsd_matrix_grad_rows(x, g, rows) - full[rows]).max() < 1e-12
