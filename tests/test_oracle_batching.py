"""Pins of the oracle's batching and clustering (App. A.1 "Batching and clustering"; App.
A.2.1, Fig. "clustering"), no GPU:

  * K-means on box dimensions recovers well separated groups exactly, and its result is a
    fixed point of Lloyd's iteration (every box at its nearest centre, every centre the mean
    of its boxes) -- checked by brute force over the centres;
  * the composite box dimensions are the bounding boxes of the dense nu_J;
  * solving the clusters one after another changes nothing under the per-cell stopping rule
    (the cells of a partition are independent problems), and under the batch rule every
    batch meets the rule on its own.
"""
import numpy as np

import oracle
import synth


def test_kmeans_recovers_separated_groups():
    rng = np.random.default_rng(0)
    centres = [(4, 5), (20, 22), (40, 9)]
    dims, truth = [], []
    for g, (a, b) in enumerate(centres):
        for _ in range(15):
            dims.append((a + rng.integers(-1, 2), b + rng.integers(-1, 2)))
            truth.append(g)
    perm = rng.permutation(len(dims))
    dims = np.array(dims)[perm]
    truth = np.array(truth)[perm]
    groups = oracle.kmeans_boxes(dims, 3)
    assert len(groups) == 3
    found = sorted(sorted(truth[g].tolist()) for g in groups)
    for f in found:
        assert len(set(f)) == 1 and len(f) == 15
    # clusters by decreasing centre area: (20,22) 440, (40,9) 360, (4,5) 20
    assert [int(truth[g[0]]) for g in groups] == [1, 2, 0]
    assert all(g == sorted(g) for g in groups)


def test_kmeans_is_a_lloyd_fixed_point():
    rng = np.random.default_rng(1)
    dims = np.stack([rng.integers(6, 60, 200), rng.integers(6, 60, 200)], axis=1)
    for k in (1, 2, 5, 9):
        groups = oracle.kmeans_boxes(dims, k)
        assert sorted(i for g in groups for i in g) == list(range(200))
        cent = np.array([dims[g].mean(axis=0) for g in groups])
        for q, g in enumerate(groups):
            for i in g:
                d = ((dims[i] - cent) ** 2).sum(axis=1)
                assert d[q] <= d.min() + 1e-9
        if k == 1:
            assert len(groups) == 1


def test_composite_box_dims_are_dense_bounding_boxes():
    N, s = 16, 2
    mu = synth.gaussian_mixture(N, 3, 1e-2, 4)
    nu = synth.gaussian_mixture(N, 3, 1e-2, 1004)
    dd = oracle.DomDec(mu, nu, s)
    eps = 2.0 / N ** 2
    dd.iterate("A", eps, fixed_iters=30)
    dd.iterate("B", eps, fixed_iters=30)
    for which in ("A", "B"):
        got = dd.composite_box_dims(which)
        for J, basic in enumerate(dd.parts[which]):
            dense = np.zeros(N * N)
            for i in basic:
                dense[dd.nu_i[i][0]] += 1.0
            r, c = np.nonzero(dense.reshape(N, N))
            assert tuple(got[J]) == (r.max() - r.min() + 1, c.max() - c.min() + 1)


def _state(N=32, seed=2):
    w = synth.workload("mix256", seed=seed, N=N)
    return w.mu, w.nu, w.init


def test_batches_change_nothing_under_the_per_cell_rule():
    N, s = 32, 2
    mu, nu, init = _state(N)
    a = oracle.DomDec(mu, nu, s, init)
    b = oracle.DomDec(mu, nu, s, init)
    eps = 1.0 / N ** 2
    nb = []
    for which in "ABAB":
        a.iterate(which, eps, tol=1e-7, rule=1)
        out = b.iterate_batched(which, eps, 3, tol=1e-7, rule=1)
        nb.append(len(out["batches"]))
    assert max(nb) >= 2
    for (ia, va), (ib, vb) in zip(a.nu_i, b.nu_i):
        assert np.array_equal(ia, ib) and np.array_equal(va, vb)


def test_every_batch_meets_the_batch_rule():
    N, s = 32, 2
    mu, nu, init = _state(N, seed=5)
    dd = oracle.DomDec(mu, nu, s, init)
    eps = 1.0 / N ** 2
    dd.iterate("A", eps, fixed_iters=5)
    tol = 1e-6
    out = dd.iterate_batched("B", eps, 4, tol=tol)
    assert len(out["batches"]) >= 2
    for g, st in zip(out["batches"], out["stats"]):
        assert st["err_total"] <= tol * st["mass"]
    # basic cells stay feasible after the batches are combined: the basic masses exactly (up
    # to rounding; balancing runs before truncation), the Y-marginal up to the truncated mass
    # (entries below 1e-15, at most N^2 per basic cell)
    assert dd.basic_mass_error() <= 1e-12
    assert dd.y_marginal_error() <= 1e-15 * N ** 2 * len(dd.nu_i)
