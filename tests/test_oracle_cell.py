"""Pins of the oracle's cell Sinkhorn against closed forms, invariants and an
independent solver (no GPU).

Each test checks the oracle against something other than itself:
  * a 2x2 problem with a closed-form optimum (cross-ratio of the Gibbs form);
  * the cross-ratio invariant of Sinkhorn-form plans plus exact marginals, which
    together certify optimality (Prop. "Optimal entropic transport couplings" (iii));
  * a direct constrained minimisation of the primal objective with scipy SLSQP;
  * the eps -> infinity limit (product coupling);
  * the stopping rule of App. A.2.1, recomputed from dense plans;
  * gauge invariance alpha -> alpha + C (Prop. ... (ii)).
"""
import math

import numpy as np
import pytest

import oracle


def _solve(xc, mu, yc, nuJ, nuref, eps, **kw):
    a, b, it, err, n = oracle.sinkhorn_cells(np.array([0, len(mu)]), xc, mu, np.array([0, len(nuJ)]),
                                             yc, nuJ, nuref, eps, **kw)
    return a, b, oracle.cell_plan(xc, mu, a, yc, nuref, b, eps), n, err


def _random_cell(rng, nx_side=4, ny=30, grid=16):
    h = 1.0 / grid
    k = np.arange(nx_side)
    X = np.stack(np.meshgrid(k, k, indexing="ij"), -1).reshape(-1, 2)
    X = (X + 3 + 0.5) * h
    ypix = rng.choice(grid * grid, size=ny, replace=False)
    Y = np.stack([ypix // grid, ypix % grid], 1).astype(float)
    Y = (Y + 0.5) * h
    mu = rng.uniform(0.5, 1.5, len(X))
    mu /= mu.sum()
    nuJ = rng.uniform(0.2, 1.0, ny)
    nuJ *= mu.sum() / nuJ.sum()
    nuref = nuJ * rng.uniform(1.0, 3.0, ny)
    return X, mu, Y, nuJ, nuref, h


def test_closed_form_two_points():
    h = 0.1
    eps = h * h * 0.7
    X = np.array([[0.0, 0.0], [h, 0.0]])
    mu = np.array([0.5, 0.5])
    _, _, P, _, _ = _solve(X, mu, X.copy(), mu.copy(), mu.copy(), eps, tol=1e-15, max_iter=100000)
    r = math.exp(h * h / eps)
    p = r / (2.0 * (1.0 + r))
    expect = np.array([[p, 0.5 - p], [0.5 - p, p]])
    assert np.max(np.abs(P - expect)) < 1e-13


def test_cross_ratio_and_marginals_certify_optimality():
    rng = np.random.default_rng(1)
    X, mu, Y, nuJ, nuref, h = _random_cell(rng)
    eps = 2.0 * h * h
    _, _, P, n, _ = _solve(X, mu, Y, nuJ, nuref, eps, tol=1e-14, max_iter=100000)
    assert np.max(np.abs(P.sum(1) - mu)) < 1e-14 * 10
    assert np.max(np.abs(P.sum(0) - nuJ)) < 1e-15 * 10
    for _ in range(200):
        x, xp = rng.choice(len(X), 2, replace=False)
        y, yp = rng.choice(len(Y), 2, replace=False)
        ratio = P[x, y] * P[xp, yp] / (P[x, yp] * P[xp, y])
        expect = math.exp(2.0 * np.dot(X[x] - X[xp], Y[y] - Y[yp]) / eps)
        assert abs(ratio / expect - 1.0) < 1e-9


def test_matches_direct_primal_minimisation():
    scipy_opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, (3, 2))
    Y = rng.uniform(0, 1, (3, 2))
    mu = rng.uniform(0.5, 1.5, 3)
    mu /= mu.sum()
    nuJ = rng.uniform(0.5, 1.5, 3)
    nuJ /= nuJ.sum()
    nuref = nuJ * np.array([1.0, 1.5, 2.0])
    eps = 0.3
    c = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    ref = mu[:, None] * nuref[None, :]

    def f(p):
        P = p.reshape(3, 3)
        return float((c * P).sum() + eps * (P * np.log(P / ref) - P + ref).sum())

    def g(p):
        P = p.reshape(3, 3)
        return (c + eps * np.log(P / ref)).reshape(-1)

    cons = [{"type": "eq", "fun": lambda p, k=k: p.reshape(3, 3)[k].sum() - mu[k]} for k in range(3)]
    # one column constraint is implied by the others (equal totals) and is left out
    cons += [{"type": "eq", "fun": lambda p, k=k: p.reshape(3, 3)[:, k].sum() - nuJ[k]} for k in range(2)]
    p0 = np.outer(mu, nuJ).reshape(-1)
    res = scipy_opt.minimize(f, p0, jac=g, constraints=cons, bounds=[(1e-14, 1)] * 9, method="SLSQP",
                             options={"ftol": 1e-15, "maxiter": 2000})
    _, _, P, _, _ = _solve(X, mu, Y, nuJ, nuref, eps, tol=1e-15, max_iter=100000)
    assert np.max(np.abs(P - res.x.reshape(3, 3))) < 1e-6
    assert f(P.reshape(-1)) <= res.fun + 1e-12


def test_large_eps_tends_to_product():
    rng = np.random.default_rng(3)
    X, mu, Y, nuJ, nuref, h = _random_cell(rng)
    diam2 = 2.0
    devs = []
    for eps in (1e3 * diam2, 1e4 * diam2):
        _, _, P, _, _ = _solve(X, mu, Y, nuJ, nuref, eps, tol=1e-15, max_iter=1000)
        prod = np.outer(mu, nuJ) / mu.sum()
        dev = np.abs(P - prod).sum()
        assert dev <= 4.0 * diam2 / eps
        devs.append(dev)
    assert 9.0 < devs[0] / devs[1] < 11.0


@pytest.mark.parametrize("rule", [0, 1])
def test_stopping_rule(rule):
    rng = np.random.default_rng(11)
    cells = [_random_cell(rng) for _ in range(3)]
    xoff = np.cumsum([0] + [len(c[1]) for c in cells])
    yoff = np.cumsum([0] + [len(c[3]) for c in cells])
    X = np.concatenate([c[0] for c in cells])
    mu = np.concatenate([c[1] for c in cells])
    Y = np.concatenate([c[2] for c in cells])
    nuJ = np.concatenate([c[3] for c in cells])
    nuref = np.concatenate([c[4] for c in cells])
    h = cells[0][5]
    eps = 0.5 * h * h
    tol = 1e-6
    a, b, iters, err, n = oracle.sinkhorn_cells(xoff, X, mu, yoff, Y, nuJ, nuref, eps, tol=tol, rule=rule)

    def dense_err(al, be):
        e = []
        for j in range(3):
            P = oracle.cell_plan(X[xoff[j]:xoff[j + 1]], mu[xoff[j]:xoff[j + 1]], al[xoff[j]:xoff[j + 1]],
                                 Y[yoff[j]:yoff[j + 1]], nuref[yoff[j]:yoff[j + 1]],
                                 be[yoff[j]:yoff[j + 1]], eps)
            e.append(np.abs(P.sum(1) - mu[xoff[j]:xoff[j + 1]]).sum())
        return np.array(e)

    e_final = dense_err(a, b)
    assert np.allclose(e_final, err, rtol=0, atol=1e-14)  # both are differences of O(1e-2) sums
    masses = np.array([mu[xoff[j]:xoff[j + 1]].sum() for j in range(3)])
    if rule == 0:
        assert e_final.sum() <= tol * mu.sum()
        a2, b2, _, _, n2 = oracle.sinkhorn_cells(xoff, X, mu, yoff, Y, nuJ, nuref, eps, fixed_iters=n - 1)
        assert dense_err(a2, b2).sum() > tol * mu.sum()
    else:
        assert np.all(e_final <= tol * masses)
        for j in range(3):
            a2, b2, _, _, _ = oracle.sinkhorn_cells(xoff, X, mu, yoff, Y, nuJ, nuref, eps,
                                                    fixed_iters=int(iters[j]) - 1)
            assert dense_err(a2, b2)[j] > tol * masses[j]


def test_gauge_invariance_of_warm_start():
    rng = np.random.default_rng(5)
    X, mu, Y, nuJ, nuref, h = _random_cell(rng)
    eps = h * h
    a0 = rng.normal(0, h * h, len(mu))
    _, _, P1, _, _ = _solve(X, mu, Y, nuJ, nuref, eps, fixed_iters=7, alpha=a0)
    _, _, P2, _, _ = _solve(X, mu, Y, nuJ, nuref, eps, fixed_iters=7, alpha=a0 + 0.37)
    assert np.max(np.abs(P1 - P2)) < 1e-15
