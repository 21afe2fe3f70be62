"""The fixed-point check used by the GPU clustering tests accepts the
oracle's own results and rejects states that are not fixed points."""
import numpy as np
import pytest

from kmedoids_check import check_fixed_point


def as_got(r):
    return {"labels": r["labels"], "medoids": r["medoids"], "sizes": r["sizes"],
            "mean_r": r["mean_r"], "info": np.array([r["rep_cluster"], r["iterations"],
                                                     int(r["converged"])])}


@pytest.fixture(scope="module")
def case(orc):
    rng = np.random.default_rng(3)
    pts = np.r_[rng.normal(0, 1, (50, 2)), rng.normal(7, 1, (40, 2)), rng.normal((0, 9), 1, (30, 2))]
    N = len(pts)
    i, j = np.triu_indices(N, 1)
    D = np.linalg.norm(pts[i] - pts[j], axis=1).astype(np.float32)
    r = orc.kmedoids(D, N, 3, [0, 1, 2])
    assert r["converged"]
    return D, N, r


def test_accepts_the_oracle(case):
    D, N, r = case
    check_fixed_point(D, N, 3, as_got(r))


def test_rejects_a_wrong_medoid(case):
    D, N, r = case
    g = as_got(r)
    c = 0
    mem = np.flatnonzero(g["labels"] == c)
    g["medoids"] = g["medoids"].copy()
    g["medoids"][c] = mem[mem != g["medoids"][c]][0]
    with pytest.raises(AssertionError):
        check_fixed_point(D, N, 3, g)


def test_rejects_a_wrong_label(case):
    D, N, r = case
    g = as_got(r)
    g["labels"] = g["labels"].copy()
    m = int(np.flatnonzero(~np.isin(np.arange(N), g["medoids"]))[0])
    g["labels"][m] = (g["labels"][m] + 1) % 3
    with pytest.raises(AssertionError):
        check_fixed_point(D, N, 3, g)


def test_rejects_a_wrong_mean(case):
    D, N, r = case
    g = as_got(r)
    g["mean_r"] = g["mean_r"] + 1e-5
    with pytest.raises(AssertionError):
        check_fixed_point(D, N, 3, g)
