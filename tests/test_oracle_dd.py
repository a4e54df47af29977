"""Pins of the oracle's domain decomposition (no GPU).

  * partition structure and connectedness of the partition graph
    (Def. "Basic and composite partitions", Def. "Partition graph");
  * feasibility of every iterate: sum_i nu_i = nu, sum_y nu_i = m_i after balancing
    (Alg. "DomDecIter" keeps pi in Pi(mu, nu));
  * a single composite cell reduces DD to the global Sinkhorn solve;
  * convergence to the unique global optimum on a small grid (Prop. "Convergence of
    the hybrid scheme", which covers plain DD);
  * monotone objective and weak duality D <= E (App. A.2.2 definitions).
"""
import numpy as np
import pytest

import oracle
import synth


def _small(N=16, s=2, seed=0):
    mu = synth.gaussian_mixture(N, 3, 1e-2, seed)
    nu = synth.gaussian_mixture(N, 3, 1e-2, seed + 1000)
    return mu, nu


def test_partitions_cover_and_connect():
    n = 8
    for which in ("A", "B"):
        cells = oracle.composite_partition(n, which)
        flat = sorted(i for c in cells for i in c)
        assert flat == list(range(n * n))
    A = oracle.composite_partition(n, "A")
    B = oracle.composite_partition(n, "B")
    assert all(len(c) == 4 for c in A)
    assert sorted(len(c) for c in B) == sorted([1] * 4 + [2] * 4 * (n // 2 - 1) + [4] * (n // 2 - 1) ** 2)
    # partition graph: vertices A u B, edge when two cells share a basic cell
    V = [("A", k) for k in range(len(A))] + [("B", k) for k in range(len(B))]
    sets = [set(c) for c in A] + [set(c) for c in B]
    seen = {0}
    stack = [0]
    while stack:
        u = stack.pop()
        for v in range(len(V)):
            if v not in seen and sets[u] & sets[v]:
                seen.add(v)
                stack.append(v)
    assert len(seen) == len(V)


def test_feasibility_and_balancing():
    mu, nu = _small(16, 2)
    dd = oracle.DomDec(mu, nu, 2)
    eps = (2.0 / 16) ** 2
    for k in range(4):
        # balancing alone restores the basic masses to rounding
        dd.iterate("AB"[k % 2], eps, tol=1e-4, truncate=False)
        assert dd.basic_mass_error() < 2e-16  # a few ulps of m_i ~ 1/64
        assert dd.y_marginal_error() < 1e-15
        assert all(np.all(v >= 0) for _, v in dd.nu_i)
    for k in range(4):
        # truncation drops entries below 1e-15: at most |supp| * 1e-15 per basic cell
        dd.iterate("AB"[k % 2], eps, tol=1e-4)
        assert dd.basic_mass_error() < 1e-15 * 256
        assert dd.y_marginal_error() < 1e-15 * 256 * 64
        assert all(np.all(v >= 1e-15) for _, v in dd.nu_i)


def test_single_cell_equals_global_sinkhorn():
    N = 8
    mu, nu = _small(N)
    eps = (2.0 / N) ** 2
    dd = oracle.DomDec(mu, nu, 4)  # n = 2: the A partition is one cell covering X
    assert len(dd.parts["A"]) == 1
    dd.iterate("A", eps, tol=1e-14, max_iter=100000, balance=False, truncate=False)
    _, _, P, _ = oracle.global_sinkhorn(mu, nu, eps, tol=1e-14)
    xpix, ysup, plan = dd.cell_plans("A")[0]
    D = np.zeros_like(P)
    D[np.ix_(xpix, ysup)] = plan
    assert np.max(np.abs(D - P)) < 1e-15


def test_dd_converges_to_global_optimum():
    N = 16
    mu, nu = _small(N, seed=2)
    eps = (2.0 / N) ** 2
    a, b, P, _ = oracle.global_sinkhorn(mu, nu, eps, tol=1e-13)
    Estar = oracle.primal_dense(mu, nu, P, eps)
    Dstar = oracle.dual_value(mu, nu, a, b, eps)
    assert abs(Estar - Dstar) < 1e-11 * abs(Estar)
    dd = oracle.DomDec(mu, nu, 4)
    Es = []
    for k in range(60):
        # inner tolerance 1e-11 sits above the float64 error floor of the cell solves
        dd.iterate("AB"[k % 2], eps, tol=1e-11, max_iter=5000)
        Es.append(dd.primal(eps))
    Es = np.array(Es)
    assert np.all(np.diff(Es) <= 1e-10 * abs(Es[0]))  # monotone up to the inner tolerance
    assert np.all(Es >= Dstar - 1e-12)  # weak duality
    assert (Es[-1] - Estar) / Estar < 1e-9


def test_basic_cells_are_contiguous_blocks():
    N, s = 16, 4
    cells = oracle.basic_cell_pixels(N, s)
    owner = np.full(N * N, -1)
    for i, p in enumerate(cells):
        assert np.all(owner[p] == -1)
        owner[p] = i
        k1, k2 = p // N, p % N
        r, c = divmod(i, N // s)
        assert set(k1) == set(range(r * s, r * s + s)) and set(k2) == set(range(c * s, c * s + s))
    assert np.all(owner >= 0)


def test_stitched_dual_weak_duality_and_zero_gap():
    """Stitched dual (the gap of the DD iterate): D(alpha+, beta+) never exceeds the optimum
    (weak duality, checked with dual_value's general formula on the same point), and the gap
    E(pi) - D closes as DD converges to the global optimum."""
    N = 16
    mu, nu = _small(N, seed=2)
    eps = (2.0 / N) ** 2
    a, b, P, _ = oracle.global_sinkhorn(mu, nu, eps, tol=1e-13)
    Estar = oracle.primal_dense(mu, nu, P, eps)
    dd = oracle.DomDec(mu, nu, 4)
    gaps = []
    for k in range(60):
        dd.iterate("AB"[k % 2], eps, tol=1e-11, max_iter=5000)
        if k >= 1:
            D, al, be = dd.stitched_dual(eps)
            # the Y-update makes the exp term of the dual exactly its constant
            Dg = oracle.dual_value(mu, nu, al, be, eps)
            assert abs(D - Dg) <= 1e-12 * abs(D)
            assert D <= Estar + 1e-12 * abs(Estar)
            gaps.append(dd.primal(eps) - D)
    gaps = np.array(gaps)
    assert gaps[0] > 1e-6 * Estar        # far from the optimum at the start
    assert 0 <= gaps[-1] < 1e-8 * Estar  # closed at convergence
    # a gauge shift of one cell's potential (the cell problem's invariance) leaves D unchanged
    D0, _, _ = dd.stitched_dual(eps)
    dd.alpha["B"][3] = dd.alpha["B"][3] + 0.37
    dd.alpha["A"][0] = dd.alpha["A"][0] - 1.25
    D1, _, _ = dd.stitched_dual(eps)
    assert abs(D1 - D0) <= 1e-12 * abs(D0)


@pytest.mark.parametrize("name,N", [("mix256", 64), ("flow512", 64), ("mix256", 128)])
def test_sparse_init_aggregates_to_feasible_basic_marginals(name, N):
    """Right after init from a sparse coupling (Knothe-Rosenblatt or a map coupling), the basic
    cell Y-marginals carry the masses of the coupling (Sec. 2.3, the state nu_i is the
    Y-marginal of pi restricted to X_i x Y): sum_y nu_i = m_i and sum_i nu_i = nu."""
    w = synth.workload(name, N=N)
    o = oracle.DomDec(w.mu, w.nu, w.s, w.init)
    mi = np.array([v.sum() for _, v in o.nu_i])
    assert np.abs(mi - o.m).max() <= 1e-15
    tot = np.zeros(N * N)
    for idx, v in o.nu_i:
        assert np.all(np.diff(idx) > 0) and np.all(v >= 0)
        np.add.at(tot, idx, v)
    assert np.abs(tot - o.nu).max() <= 1e-15
    assert np.abs(tot - o.nu).sum() <= 1e-14


@pytest.mark.parametrize("s", [1, 2, 4])
def test_sparse_init_matches_dense_brute_force(s):
    """Brute force on a tiny grid: materialise the coupling as a dense (N^2, N^2) matrix and sum
    its rows over each basic cell's s x s pixel block by explicit loops over (k1, k2)."""
    N = 8
    mu, nu = _small(N, s=2, seed=5)
    x, y, m = synth.kr_coupling(mu, nu)
    P = np.zeros((N * N, N * N))
    for a, b, v in zip(x, y, m):
        P[a, b] += v
    o = oracle.DomDec(mu, nu, s, (x, y, m))
    n = N // s
    for r in range(n):
        for c in range(n):
            want = np.zeros(N * N)
            for k1 in range(r * s, (r + 1) * s):
                for k2 in range(c * s, (c + 1) * s):
                    want += P[k1 * N + k2]
            got = np.zeros(N * N)
            idx, v = o.nu_i[r * n + c]
            got[idx] = v
            assert np.abs(got - want).max() <= 1e-17, (r, c)
