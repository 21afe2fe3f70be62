"""Fixed-point check of a clustering of a packed score matrix (K-means with
member centres, representative by min <R>/f) by plain FP64 sums, with the
slack that a sum of scores each rounded to a multiple of Q = 2^-20 allows:
a member's sum may be off by (n - 1) Q / 2, so the chosen medoid must be
within (n - 1) Q of the smallest FP64 sum, <R> within Q / 2 of the FP64
mean, and the representative within Q N / n of the smallest <R> N / n."""
import numpy as np

import oracle

Q = 2.0 ** -20


def scores(D, N, i, j):
    """D(i, j) in FP64 for index arrays (0 on the diagonal)."""
    i, j = np.broadcast_arrays(np.asarray(i, np.int64), np.asarray(j, np.int64))
    a, b = np.minimum(i, j), np.maximum(i, j)
    out = np.zeros(a.shape)
    m = a != b
    out[m] = D[oracle.packed_index(a[m], b[m], N)]
    return out


def cluster_sums(D, N, mem):
    """FP64 sums of every member's scores to the other members of `mem`."""
    cost = np.zeros(len(mem))
    for s0 in range(0, len(mem), 256):
        I, J = np.meshgrid(mem[s0:s0 + 256], mem, indexing="ij")
        cost[s0:s0 + 256] = scores(D, N, I, J).sum(1)
    return cost


def check_fixed_point(D, N, k, got):
    """Asserts that `got` (labels, medoids, sizes, mean_r, info) is a valid
    final state of the method on the float32 matrix D."""
    lab, med = np.asarray(got["labels"]), np.asarray(got["medoids"])
    assert len(set(med.tolist())) == k and np.all((med >= 0) & (med < N))
    idx = np.arange(N)
    dist = np.stack([scores(D, N, idx, m) for m in med], 1)
    want = np.argmin(dist, 1)                       # first minimum = lowest cluster on ties
    want[med] = np.arange(k)
    assert np.array_equal(lab, want), "labels are not the nearest medoids"
    assert np.array_equal(got["sizes"], np.bincount(lab, minlength=k)), "sizes"
    sc = np.full(k, np.inf)
    for c in range(k):
        mem = np.flatnonzero(lab == c)
        n = len(mem)
        cost = cluster_sums(D, N, mem)
        if got["info"][2]:
            mc = cost[np.flatnonzero(mem == med[c])[0]]
            assert mc <= cost.min() + (n - 1) * Q * (1 + 1e-9) + 1e-9, \
                f"medoid of cluster {c} is {mc - cost.min():.3g} above the in-cluster minimum"
        if n > 1:
            mr = cost.sum() / (n * (n - 1.0))
            assert abs(got["mean_r"][c] - mr) <= Q / 2 + 1e-9, f"<R> of cluster {c}"
            sc[c] = mr * N / n
    rep = int(got["info"][0])
    if np.isfinite(sc).any():
        assert rep >= 0 and sc[rep] <= sc.min() + Q * N / got["sizes"][rep] + 1e-9, "representative"
    else:
        assert rep == -1
