"""Pins of the oracle's flow update and min-cost flow (no GPU).

  * integer min-cost flow: feasibility, complementary slackness with the returned
    node potentials, and the optimal value of an independent LP solve (scipy HiGHS);
  * singleton cells (s = 1): edge costs reduce to eq. (CostCoefficientSimple);
  * marginals preserved (Lemma "flow preserves marginals");
  * change of transport cost equals sum w_ij cbar_ij <= 0 (Lemma "transport
    non-increasing", eq. total-cost-update), checked on the dense new plan;
  * KL does not increase with gluing candidates (Lemma "properties of the gluing
    edge candidates", item 3);
  * mu (x) nu is a fixed point (Sec. 3.3).
"""
import numpy as np
import pytest

import oracle
import synth


def _mcf_instance(rng, n=12, extra=25):
    tails, heads = [], []
    for i in range(n):
        tails.append(i)
        heads.append(i)
    for _ in range(extra):
        i, j = rng.integers(0, n, 2)
        if i != j:
            tails += [i, j]
            heads += [j, i]
    tail = np.array(tails, np.int32)
    head = np.array(heads, np.int32)
    cost = rng.integers(-50, 50, len(tail)).astype(np.int64)
    cost[tail == head] = 0
    sup = rng.integers(1, 100, n).astype(np.int64)
    return n, tail, head, cost, sup


@pytest.mark.parametrize("seed", range(5))
def test_mcf_optimal_and_certified(seed):
    linprog = pytest.importorskip("scipy.optimize").linprog
    rng = np.random.default_rng(seed)
    n, tail, head, cost, sup = _mcf_instance(rng)
    flow, pot, st = oracle.mcf_ssp(n, tail, head, cost, sup, sup)
    assert st == 0
    assert np.all(flow >= 0)
    assert np.array_equal(np.bincount(tail, weights=flow, minlength=n).astype(np.int64), sup)
    assert np.array_equal(np.bincount(head, weights=flow, minlength=n).astype(np.int64), sup)
    rc = cost + pot[tail] - pot[n + head]
    assert np.all(rc >= 0)
    assert np.all(rc[flow > 0] == 0)
    m = len(tail)
    A = np.zeros((2 * n, m))
    A[tail, np.arange(m)] = 1
    A[n + head, np.arange(m)] = 1
    res = linprog(cost, A_eq=A, b_eq=np.concatenate([sup, sup]), bounds=(0, None), method="highs")
    assert res.status == 0
    assert abs(res.fun - float((flow * cost).sum())) < 1e-6


def _state(N=8, s=2, angle=90.0, scale=1.0, shift=(0.0, 0.0), seed=0):
    mu = synth.gaussian_mixture(N, 3, 1e-2, seed)
    tgt = synth.rotation_map(N, angle, scale, shift)
    nu, init = synth.map_coupling(mu, tgt)
    dd = oracle.DomDec(mu, nu, s, init)
    eps = (1.0 / N) ** 2
    dd.iterate("A", eps, fixed_iters=300, balance=False, truncate=False)
    dd.iterate("B", eps, fixed_iters=300, balance=False, truncate=False)
    return dd, eps


def _dense_pi(dd):
    """pi = sum_i pi_i from the last composite solve, as an (N^2, N^2) array."""
    NN = dd.N * dd.N
    P = np.zeros((NN, NN))
    for xpix, ysup, plan in dd.cell_plans():
        P[np.ix_(xpix, ysup)] += plan
    return P


def _dense_pihat(dd, pi, tail, head, w, nu_old):
    """pi_hat = sum_j sum_{i in N(j)} w_ij pihat_ij with product candidates (eq. flow-update-new-plan)."""
    NN = dd.N * dd.N
    P = np.zeros((NN, NN))
    for a in range(len(tail)):
        i, j = int(tail[a]), int(head[a])
        if w[a] == 0:
            continue
        if i == j:
            rows = dd.cells[i]
            P[rows] += (w[a] / dd.m[i]) * pi[rows]
        else:
            idx, val = nu_old[i]
            xj = dd.cells[j]
            P[np.ix_(xj, idx)] += w[a] * np.outer(dd.mu[xj] / dd.m[j], val / dd.m[i])
    return P


def _kl(dd, P):
    ref = np.outer(dd.mu, dd.nu)
    pos = P > 0
    return float((P[pos] * np.log(P[pos] / ref[pos]) - P[pos]).sum() + ref.sum())


def _cost_matrix(dd):
    C = dd.coords
    return ((C[:, None, :] - C[None, :, :]) ** 2).sum(-1)


def test_singleton_cells_reduce_to_simple_costs():
    dd, eps = _state(N=8, s=1)
    nu_old = list(dd.nu_i)
    res = dd.flow_update(truncate=False)
    tail, head = oracle.neighbourhood(dd.n)
    c = _cost_matrix(dd)
    for a in range(len(tail)):
        i, j = int(tail[a]), int(head[a])
        idx, val = nu_old[i]
        xi, xj = dd.cells[i][0], dd.cells[j][0]
        expect = float(((c[xj, idx] - c[xi, idx]) * val).sum() / dd.m[i])
        assert abs(res["cbar"][a] - expect) < 1e-13


def test_flow_invariants():
    dd, eps = _state(N=8, s=2)
    pi = _dense_pi(dd)
    nu_old = list(dd.nu_i)
    res = dd.flow_update(truncate=False)
    tail, head = oracle.neighbourhood(dd.n)
    w = res["w"]
    # flow feasibility (divergence constraint, eq. div-constraint-single-cell)
    assert np.allclose(np.bincount(tail, weights=w, minlength=len(dd.m)), dd.m, rtol=1e-15, atol=0)
    # in-flow: each of <= 5 incoming arcs carries at most one unit of 2^-40 rounding
    assert np.max(np.abs(np.bincount(head, weights=w, minlength=len(dd.m)) - dd.m)) <= 5 * 2.0 ** -40
    # marginals preserved
    assert dd.y_marginal_error() < 1e-15
    pihat = _dense_pihat(dd, pi, tail, head, w, nu_old)
    assert np.max(np.abs(pihat.sum(1) - pi.sum(1))) <= 5 * 2.0 ** -40
    assert np.max(np.abs(pihat.sum(0) - pi.sum(0))) < 1e-15
    # new cell marginals agree with the dense plan
    for j in range(len(dd.cells)):
        idx, val = dd.nu_i[j]
        dense = np.zeros(dd.N * dd.N)
        dense[idx] = val
        assert np.max(np.abs(dense - pihat[dd.cells[j]].sum(0))) < 1e-15
    # transport cost change = sum w cbar <= 0, strictly negative for a rotated init
    c = _cost_matrix(dd)
    dcost = float((c * pihat).sum() - (c * pi).sum())
    assert abs(dcost - res["value"]) < 1e-13
    assert res["value"] < -1e-4
    # KL non-increase
    assert _kl(dd, pihat) <= _kl(dd, pi) + 1e-13


def test_product_coupling_is_fixed_point():
    N, s = 8, 2
    mu = synth.gaussian_mixture(N, 3, 1e-2, 4)
    nu = synth.gaussian_mixture(N, 3, 1e-2, 5)
    dd = oracle.DomDec(mu, nu, s)  # product coupling nu_i = m_i nu
    # the last composite solve: alpha = beta = 0 gives pi_J = mu_J (x) nu exactly
    eps = 1.0
    dd.iterate("B", eps, fixed_iters=1, balance=False, truncate=False)
    for cs in dd.last["B"]:
        cs.alpha[:] = 0.0
        cs.beta[:] = 0.0
    dd.nu_i = [(np.arange(N * N), mi * dd.nu) for mi in dd.m]
    res = dd.flow_update(truncate=False)
    for j, (idx, val) in enumerate(dd.nu_i):
        dense = np.zeros(N * N)
        dense[idx] = val
        assert np.max(np.abs(dense - dd.m[j] * dd.nu)) < 1e-15
    assert res["value"] <= 0.0


def test_largest_remainder_rounding():
    rng = np.random.default_rng(2)
    m = rng.uniform(0.1, 1.0, 50)
    m /= m.sum()
    T = 1 << 40
    b = oracle.largest_remainder(m, T)
    assert int(b.sum()) == T
    assert np.all(np.abs(b - m * T) < 1.0)


# ---- gluing edge candidates from entropic gamma_ij (Remark "eps-gamma") ----------------------

def _tight_state(N=8, s=2, angle=90.0, scale=1.0, seed=0, uniform=False):
    """A state whose composite plans have exact X-marginals (cell solves to 1e-13), so that the
    candidates' X-marginals are mu_j / m_j to rounding."""
    mu = np.full((N, N), 1.0 / N ** 2) if uniform else synth.gaussian_mixture(N, 3, 1e-2, seed)
    tgt = synth.rotation_map(N, angle, scale, (0.0, 0.0))
    nu, init = synth.map_coupling(mu, tgt)
    dd = oracle.DomDec(mu, nu, s, init)
    eps = (1.0 / N) ** 2
    dd.iterate("A", eps, tol=1e-13, max_iter=100000, balance=False, truncate=False)
    dd.iterate("B", eps, tol=1e-13, max_iter=100000, balance=False, truncate=False)
    return dd, eps


def test_glued_candidate_marginals():
    """Lemma "properties of the gluing edge candidates", item 1: pihat_ij in
    Pi(mu_j / m_j, nu_i / m_i)."""
    dd, eps = _tight_state()
    plans = dd.basic_plans()
    tail, head = oracle.neighbourhood(dd.n)
    for a in range(0, len(tail), 3):
        i, j = int(tail[a]), int(head[a])
        if i == j:
            continue
        ysup, ph = dd.glued_candidate(i, j, 0.3 * eps, plans)
        assert np.abs(ph.sum(1) - dd.mu[dd.cells[j]] / dd.m[j]).max() <= 1e-12
        assert np.abs(ph.sum(0) - plans[i][1].sum(0) / dd.m[i]).max() <= 1e-15


def test_glued_candidate_limits():
    """Remark "eps-gamma": eps_gamma -> infinity gives the product candidate
    mu_j / m_j (x) nu_i / m_i; on a uniform mu, where the optimal map between neighbouring
    cells is the translation, eps_gamma -> 0 gives pi_i translated onto X_j."""
    dd, eps = _tight_state()
    plans = dd.basic_plans()
    i, j = 5, 6  # horizontal neighbours in the 4 x 4 basic-cell grid
    ysup, ph = dd.glued_candidate(i, j, 1e6, plans)
    prod = np.outer(dd.mu[dd.cells[j]] / dd.m[j], plans[i][1].sum(0) / dd.m[i])
    assert np.abs(ph - prod).max() <= 1e-6 * prod.max()
    du, eps = _tight_state(uniform=True)
    plans = du.basic_plans()
    # X_i and X_j are row-major 2 x 2 blocks, X_j = X_i shifted by one cell (the same order);
    # the distance to the translated plan falls as eps_gamma does
    dev = []
    for f in (0.4, 0.2, 0.1):
        ysup, ph = du.glued_candidate(i, j, f / du.N ** 2, plans)
        dev.append(np.abs(ph - plans[i][1] / du.m[i]).max() / ph.max())
    assert dev[0] > dev[1] > dev[2] and dev[2] <= 1e-4, dev


def test_glued_flow_update_does_not_increase_the_objective():
    """Prop. "flow update decreases score" with gluing candidates (Lemma "properties of the
    gluing edge candidates", item 3; Lemma "transport non-increasing"): on the dense plans,
    marginals are kept and E(pihat) <= E(pi)."""
    dd, eps = _tight_state()
    pi = _dense_pi(dd)
    plans = dd.basic_plans()
    tail, head = oracle.neighbourhood(dd.n)
    eps_g = 0.5 * eps
    cands = {}
    for a in range(len(tail)):
        i, j = int(tail[a]), int(head[a])
        if i != j:
            cands[a] = dd.glued_candidate(i, j, eps_g, plans)
    res = dd.flow_update(truncate=False, eps_gamma=eps_g)
    w = res["w"]
    NN = dd.N * dd.N
    P = np.zeros((NN, NN))
    for a in range(len(tail)):
        i, j = int(tail[a]), int(head[a])
        if w[a] == 0:
            continue
        if i == j:
            P[dd.cells[i]] += (w[a] / dd.m[i]) * pi[dd.cells[i]]
        else:
            ysup, ph = cands[a]
            P[np.ix_(dd.cells[j], ysup)] += w[a] * ph
    assert np.abs(P.sum(0) - pi.sum(0)).max() <= 1e-15
    assert np.abs(P.sum(1) - pi.sum(1)).max() <= 5 * 2.0 ** -40 + 1e-13
    c = _cost_matrix(dd)
    E = lambda Q: float((c * Q).sum()) + eps * _kl(dd, Q)  # noqa: E731
    assert res["value"] < 0.0
    assert abs(float((c * P).sum() - (c * pi).sum()) - res["value"]) <= 1e-13
    assert E(P) <= E(pi) + 1e-14
