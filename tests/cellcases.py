"""Random batches of cell problems in the layout of sinkhorn_batch, and their oracle solves.

Coordinates are in pixel units (h = 1, eps = kappa): X pixel i of a cell sits at i, Y pixel j
at j - E, so |x - y|^2 / eps = |i - j + E|^2 / kappa, the local cost of the GPU solver.
"""
from __future__ import annotations

import numpy as np

import oracle

NEG = -1.0e30


def random_cells(rng, ncells, xside, wlo, whi, kappa, zero_x_rows=True, zero_frac=0.1,
                 w2=None):
    """Random cell problems; box sides uniform in [wlo, whi] (the second side in w2 = (lo, hi)
    when given)."""
    dims = rng.integers(wlo, whi + 1, size=(ncells, 2)).astype(np.int32)
    if w2 is not None:
        dims[:, 1] = rng.integers(w2[0], w2[1] + 1, size=ncells)
    sizes = dims[:, 0].astype(np.int64) * dims[:, 1]
    base = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    shift = np.zeros((ncells, 2), np.int32)
    logmu = np.full((ncells, xside * xside), NEG)
    lognu = np.full(int(sizes.sum()), NEG)
    for c in range(ncells):
        W1, W2 = dims[c]
        shift[c] = [int(round((W1 - 1) / 2 - (xside - 1) / 2)) + rng.integers(-2, 3),
                    int(round((W2 - 1) / 2 - (xside - 1) / 2)) + rng.integers(-2, 3)]
        mu = rng.uniform(0.5, 1.5, (xside, xside)) * 1e-4
        if zero_x_rows and c % 3 == 1:
            mu[: xside // 2, :] = 0.0  # boundary cell padded with zero mass
        if zero_x_rows and c % 5 == 2:
            mu[:, : xside // 2] = 0.0
        g1 = np.exp(-((np.arange(W1) - rng.uniform(0, W1)) ** 2) / (2 * max(W1, 2) ** 2 / 4))
        g2 = np.exp(-((np.arange(W2) - rng.uniform(0, W2)) ** 2) / (2 * max(W2, 2) ** 2 / 4))
        nu = np.outer(g1, g2) * rng.uniform(0.5, 1.5, (W1, W2))
        if W1 * W2 > 4:
            nu[rng.uniform(size=(W1, W2)) < zero_frac] = 0.0
            if c % 4 == 3 and W1 > 2:
                nu[rng.integers(0, W1), :] = 0.0
        if nu.sum() <= 0:
            nu[0, 0] = 1.0
        nu *= mu.sum() / nu.sum()
        with np.errstate(divide="ignore"):
            lm = np.where(mu > 0, np.log(mu), NEG)
            ln = np.where(nu > 0, np.log(nu), NEG)
        logmu[c] = lm.reshape(-1)
        lognu[base[c]:base[c] + sizes[c]] = ln.reshape(-1)
    return dict(dims=dims, base=base, shift=shift, logmu=logmu, lognu=lognu, xside=xside, kappa=kappa)


def cell_arrays(cells, c):
    """Valid X/Y points of cell c: (xidx, X coords, mu, yidx, Y coords, nuJ) in pixel units."""
    xs = cells["xside"]
    W1, W2 = cells["dims"][c]
    E1, E2 = cells["shift"][c]
    lm = cells["logmu"][c]
    b0 = cells["base"][c]
    ln = cells["lognu"][b0:b0 + W1 * W2]
    xi = np.nonzero(lm > -1e29)[0]
    yi = np.nonzero(ln > -1e29)[0]
    X = np.stack([xi // xs, xi % xs], 1).astype(float)
    Y = np.stack([yi // W2 - E1, yi % W2 - E2], 1).astype(float)
    return xi, X, np.exp(lm[xi]), yi, Y, np.exp(ln[yi])


def gpu_plan(cells, c, f, g):
    """pi(i,j) = mu(i) nu_J(j) exp(f(i) + g(j) - C(i,j)) on the valid points, float64, from GPU
    potentials (reference mu (x) nu_J)."""
    xi, X, mu, yi, Y, nuJ = cell_arrays(cells, c)
    b0 = cells["base"][c]
    W1, W2 = cells["dims"][c]
    fv = np.asarray(f[c], np.float64)[xi]
    gv = np.asarray(g[b0:b0 + W1 * W2], np.float64)[yi]
    C = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1) / cells["kappa"]
    return np.exp(fv[:, None] + gv[None, :] - C) * mu[:, None] * nuJ[None, :]


def oracle_solve(cells, a0=None, **kw):
    """Oracle cell solves on the same cells; returns list of dense plans (valid X x valid Y), iters, n."""
    kappa = cells["kappa"]
    n = len(cells["dims"])
    xo, yo, Xs, mus, Ys, nus, als = [0], [0], [], [], [], [], []
    geo = []
    for c in range(n):
        xi, X, mu, yi, Y, nuJ = cell_arrays(cells, c)
        geo.append((xi, yi))
        Xs.append(X)
        mus.append(mu)
        Ys.append(Y)
        nus.append(nuJ)
        if a0 is None:
            als.append(np.zeros(len(xi)))
        else:
            # alpha (energy units) = eps f with eps = kappa in pixel units
            als.append(kappa * np.asarray(a0[c], np.float64)[xi])
        xo.append(xo[-1] + len(xi))
        yo.append(yo[-1] + len(yi))
    A, B, it, err, nit = oracle.sinkhorn_cells(np.array(xo), np.concatenate(Xs), np.concatenate(mus),
                                               np.array(yo), np.concatenate(Ys), np.concatenate(nus),
                                               np.concatenate(nus), kappa, alpha=np.concatenate(als), **kw)
    plans = []
    for c in range(n):
        plans.append(oracle.cell_plan(Xs[c], mus[c], A[xo[c]:xo[c + 1]], Ys[c], nus[c], B[yo[c]:yo[c + 1]],
                                      kappa))
    return plans, it, err, nit


def objective(cells, c, P):
    """E/eps = sum pi (C + log pi - log mu - log nuJ) - sum pi, for a plan on the valid points."""
    xi, X, mu, yi, Y, nuJ = cell_arrays(cells, c)
    C = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1) / cells["kappa"]
    pos = P > 0
    L = np.zeros_like(P)
    L[pos] = np.log(P[pos])
    ref = np.log(mu)[:, None] + np.log(nuJ)[None, :]
    return float((P * (C + L - ref))[pos].sum() - P.sum())


def subset(cells, idx):
    """The cells `idx` of a batch as a batch of their own (Y boxes repacked)."""
    idx = [int(c) for c in idx]
    dims = cells["dims"][idx]
    sizes = dims[:, 0].astype(np.int64) * dims[:, 1]
    base = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    lognu = np.concatenate([cells["lognu"][cells["base"][c]:cells["base"][c] + sizes[k]]
                            for k, c in enumerate(idx)]) if idx else np.zeros(0)
    return dict(dims=dims, base=base, shift=cells["shift"][idx], logmu=cells["logmu"][idx],
                lognu=lognu, xside=cells["xside"], kappa=cells["kappa"])
