"""The library's host min-cost flow (network simplex, dd_mcf_solve) against the oracle's
successive-shortest-path solver and an LP solve (no GPU: the solver runs on the host)."""
import numpy as np
import pytest

import oracle


def _instance(rng, n, extra, cmax=50, smax=100, grid=False):
    if grid:
        side = int(round(n ** 0.5))
        n = side * side
        tails, heads = [], []
        for r in range(side):
            for c in range(side):
                for dr, dc in ((-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)):
                    rr, cc = r + dr, c + dc
                    if 0 <= rr < side and 0 <= cc < side:
                        tails.append(r * side + c)
                        heads.append(rr * side + cc)
    else:
        tails, heads = list(range(n)), list(range(n))
        for _ in range(extra):
            i, j = rng.integers(0, n, 2)
            if i != j:
                tails += [i, j]
                heads += [j, i]
    tail = np.array(tails, np.int32)
    head = np.array(heads, np.int32)
    cost = rng.integers(-cmax, cmax + 1, len(tail)).astype(np.int64)
    cost[tail == head] = 0
    sup = rng.integers(1, smax + 1, n).astype(np.int64)
    return n, tail, head, cost, sup


@pytest.mark.parametrize("seed", range(8))
def test_network_simplex_matches_oracle_and_is_certified(seed):
    import paper_2405_09400_amd as dd
    rng = np.random.default_rng(seed)
    n, tail, head, cost, sup = _instance(rng, 30, 60, grid=seed % 2 == 1)
    flow, pot = dd.mcf_solve(n, tail, head, cost, sup)
    assert np.all(flow >= 0)
    assert np.array_equal(np.bincount(tail, weights=flow, minlength=n).astype(np.int64), sup)
    assert np.array_equal(np.bincount(head, weights=flow, minlength=n).astype(np.int64), sup)
    rc = cost + pot[tail] - pot[n + head]
    assert np.all(rc >= 0) and np.all(rc[flow > 0] == 0)
    oflow, _, st = oracle.mcf_ssp(n, tail, head, cost, sup, sup)
    assert st == 0
    v = sum(int(f) * int(c) for f, c in zip(flow, cost))
    vo = sum(int(f) * int(c) for f, c in zip(oflow, cost))
    assert v == vo


def test_network_simplex_large_masses_grid():
    """The flow update's scale: masses summing to 2^40, costs up to 2^30, a 24x24 grid."""
    import paper_2405_09400_amd as dd
    rng = np.random.default_rng(11)
    n, tail, head, cost, _ = _instance(rng, 576, 0, cmax=1 << 30, grid=True)
    m = rng.uniform(0.5, 1.5, n)
    sup = oracle.largest_remainder(m / m.sum(), 1 << 40)
    flow, pot = dd.mcf_solve(n, tail, head, cost, sup)
    oflow, _, st = oracle.mcf_ssp(n, tail, head, cost, sup, sup)
    v = sum(int(f) * int(c) for f, c in zip(flow, cost))
    vo = sum(int(f) * int(c) for f, c in zip(oflow, cost))
    assert v == vo
    rc = cost + pot[tail] - pot[n + head]
    assert np.all(rc >= 0) and np.all(rc[flow > 0] == 0)


def test_network_simplex_matches_lp():
    linprog = pytest.importorskip("scipy.optimize").linprog
    import paper_2405_09400_amd as dd
    rng = np.random.default_rng(3)
    n, tail, head, cost, sup = _instance(rng, 40, 100)
    flow, _ = dd.mcf_solve(n, tail, head, cost, sup)
    m = len(tail)
    A = np.zeros((2 * n, m))
    A[tail, np.arange(m)] = 1
    A[n + head, np.arange(m)] = 1
    res = linprog(cost, A_eq=A, b_eq=np.concatenate([sup, sup]), bounds=(0, None), method="highs")
    assert abs(res.fun - float((flow * cost).sum())) < 1e-6
