"""Pins for the oracle's clustering of the score matrix (K-means with member
centres, representative by the smallest <R>/f), checked against facts that do
not come from the oracle: 1-D groups where the medoid is the median and the
mean pairwise distance has a closed form, the lowest-index tie rules, the
fixed-point property of the result re-derived by brute force on the square
matrix (FP64 sums of the float32 scores, as the definition states), k = 1
(the global 1-median) and k = N, and the tie-margin diagnostic on exact and
clear-cut cases."""
import numpy as np
import pytest


def line_matrix(x):
    x = np.asarray(x, dtype=np.float64)
    i, j = np.triu_indices(len(x), 1)
    return np.abs(x[i] - x[j]).astype(np.float32)


def square(D, N):
    S = np.zeros((N, N))
    i, j = np.triu_indices(N, 1)
    S[i, j] = D
    S[j, i] = D
    return S


def test_separated_groups_medians_and_closed_forms(orc):
    # groups of n equally spaced points (spacing s): medoid = middle point,
    # mean pairwise distance = s (n + 1) / 3
    groups = [(5, 1.0, 0.0), (7, 0.5, 100.0), (3, 0.5, 200.0), (9, 0.3, 300.0)]
    x, start = [], []
    for n, s, off in groups:
        start.append(len(x))
        x += [off + s * t for t in range(n)]
    N = len(x)
    perm = np.random.default_rng(0).permutation(N)     # scramble model order
    xs = np.array(x)[perm]
    inv = np.argsort(perm)
    init = [inv[st] for st in start]                    # one seed per group (its first point)
    r = orc.kmedoids(line_matrix(xs), N, 4, init)
    assert r["converged"]
    for c, ((n, s, off), st) in enumerate(zip(groups, start)):
        members = np.sort(inv[st:st + n])
        assert np.array_equal(np.sort(np.flatnonzero(r["labels"] == c)), members)
        assert r["medoids"][c] == inv[st + n // 2]
        assert r["sizes"][c] == n
        assert abs(r["mean_r"][c] - s * (n + 1) / 3.0) < 1e-5
    score = [s * (n + 1) / 3.0 * N / n for n, s, _ in groups]
    assert r["rep_cluster"] == int(np.argmin(score)) == 3   # not the tightest group (2): f counts
    # the closest call of any update: in the final groups the median beats
    # its neighbours by s per other member, s / (n - 1) after the division;
    # earlier updates can only have been further from a tie or equal
    assert 0.0 < r["tie_margin"] <= min(s / (n - 1) for n, s, _ in groups) + 1e-6
    assert r["representative"] == r["medoids"][r["rep_cluster"]]


def test_tie_rules(orc):
    # 0,1,2,3: members 1 and 2 tie on the in-cluster sum -> lowest index wins
    r = orc.kmedoids(line_matrix([0, 1, 2, 3, 50]), 5, 2, [3, 4])
    assert list(r["medoids"]) == [1, 4]
    assert r["tie_margin"] == 0.0                       # the exact tie is reported
    # model 2 is equidistant from medoids 0 and 4 -> the lower cluster index
    r = orc.kmedoids(line_matrix([0, 5, 10, 100, 15]), 5, 2, [1, 4], max_iter=0)
    assert r["labels"][2] == 0 and r["iterations"] == 0


def test_fixed_point_by_brute_force(orc):
    rng = np.random.default_rng(1)
    pts = np.r_[rng.normal(0, 1, (40, 2)), rng.normal(6, 1, (30, 2)), rng.normal((0, 9), 1, (25, 2))]
    N = len(pts)
    i, j = np.triu_indices(N, 1)
    D = np.linalg.norm(pts[i] - pts[j], axis=1).astype(np.float32)
    S = square(D, N)
    for k, seed in ((3, 2), (5, 3), (8, 4)):
        init = np.random.default_rng(seed).choice(N, k, replace=False)
        r = orc.kmedoids(D, N, k, init)
        assert r["converged"]
        med, lab = r["medoids"], r["labels"]
        assert len(set(med)) == k
        q = S.astype(np.float32).astype(np.float64)
        for m in range(N):                               # nearest medoid, lowest index on ties
            d = S[m, med]
            want = int(np.flatnonzero(med == m)[0]) if m in med else int(np.argmin(d))
            assert lab[m] == want
        for c in range(k):                               # medoid minimises the in-cluster sum
            mem = np.flatnonzero(lab == c)
            cost = q[np.ix_(mem, mem)].sum(1)
            assert med[c] == mem[int(np.argmin(cost))]
            n = len(mem)
            assert r["sizes"][c] == n
            if n > 1:
                assert abs(r["mean_r"][c] - S[np.ix_(mem, mem)].sum() / (n * (n - 1))) < 1e-5


def test_k_equals_one_is_the_global_median(orc):
    rng = np.random.default_rng(5)
    pts = rng.normal(0, 3, (60, 3))
    N = len(pts)
    i, j = np.triu_indices(N, 1)
    D = np.linalg.norm(pts[i] - pts[j], axis=1).astype(np.float32)
    r = orc.kmedoids(D, N, 1, [17])
    assert np.all(r["labels"] == 0)
    assert r["medoids"][0] == int(np.argmin(square(D, N).sum(1)))
    assert r["rep_cluster"] == 0


def test_k_equals_n_and_argument_checks(orc):
    D = line_matrix([0, 1, 3, 7])
    r = orc.kmedoids(D, 4, 4, [3, 2, 1, 0])
    assert list(r["labels"]) == [3, 2, 1, 0] and r["converged"] and r["iterations"] == 1
    assert r["rep_cluster"] == -1 and r["representative"] == -1   # no cluster has a pair
    for bad in ([0, 0], [0, 9]):
        with pytest.raises(ValueError):
            orc.kmedoids(D, 4, 2, bad)
    with pytest.raises(ValueError):
        orc.kmedoids(D, 4, 5, [0, 1, 2, 3, 3])
