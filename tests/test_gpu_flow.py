"""GPU parity of the flow update (flow_costs / dd_mcf_solve / flow_apply / flow_update) against
the oracle's brute-force flow update on the same seeded state.

The min-cost flow may have several optimal flows (Remark on non-uniqueness), so parity is
on the edge costs, on the optimal value, and on the new marginals when both sides apply the
same flow (the oracle's).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dense(nu_i, N):
    out = np.zeros((len(nu_i), N * N))
    for k, (idx, val) in enumerate(nu_i):
        out[k, idx] = val
    return out


def _pair(N=16, s=2, seed=0, angle=60.0, prec=None):
    import paper_2405_09400_amd as dd
    mu = synth.gaussian_mixture(N, 4, 1e-2, seed)
    tgt = synth.rotation_map(N, angle, 0.9, (0.0, 0.0))
    nu, init = synth.map_coupling(mu, tgt)
    g = dd.DomDec(mu, nu, s, init, prec=dd.DD_PREC_F64 if prec is None else prec)
    o = oracle.DomDec(mu, nu, s, init)
    eps = 1.0 / N ** 2
    for part in "AB":
        g.iterate(part, eps, fixed_iters=60)
        o.iterate(part, eps, fixed_iters=60)
    return g, o, eps


@pytest.mark.parametrize("N,s", [(16, 2), (32, 2), (32, 4)])
def test_edge_costs_match_brute_force(N, s):
    _need_gpu()
    g, o, _ = _pair(N, s)
    print(f"flow costs N={N} s={s}", flush=True)
    cg = g.flow_costs()
    nu_before = list(o.nu_i)
    res = o.flow_update(truncate=True)
    co = res["cbar"]
    assert cg.shape == co.shape
    assert np.max(np.abs(cg - co)) <= 1e-11 * np.max(np.abs(co)), np.max(np.abs(cg - co))
    # the same flow applied on both sides gives the same new marginals
    g.flow_apply(res["w"])
    G = _dense(g.nu_i_sparse(), N)
    O = _dense(o.nu_i, N)
    # m_i sums differ in their last bit (pairwise vs sequential summation): ~1e-16 relative
    assert np.abs(G - O).sum() <= 1e-13
    g.close()


@pytest.mark.parametrize("N,s,eg", [(16, 2, 0.5), (32, 2, 1.0), (32, 4, 0.5)])
def test_glued_edge_costs_match_brute_force(N, s, eg):
    """Gluing candidates from entropic gamma_ij (Remark "eps-gamma"): the device's edge costs,
    from per-arc conditional moments of gamma_ij and per-pixel moments of pi_i, against the
    oracle's brute force over X_j x supp(pi_i) with its own gamma_ij; then the same flow on both
    sides."""
    _need_gpu()
    g, o, eps = _pair(N, s)
    eps_gamma = eg * eps
    print(f"glued flow costs N={N} s={s} eps_gamma={eps_gamma:.3e}", flush=True)
    cg = g.flow_costs(eps_gamma=eps_gamma)
    res = o.flow_update(truncate=True, eps_gamma=eps_gamma)
    co = res["cbar"]
    assert np.max(np.abs(cg - co)) <= 1e-10 * np.max(np.abs(co)), np.max(np.abs(cg - co))
    # glued and product costs differ (the candidates are not the product)
    assert np.max(np.abs(cg - g.flow_costs())) >= 1e-4 * np.max(np.abs(co))
    g.flow_apply(res["w"])
    G = _dense(g.nu_i_sparse(), N)
    O = _dense(o.nu_i, N)
    assert np.abs(G - O).sum() <= 1e-13
    g.close()


def test_glued_hybrid_schedule_decreases_objective():
    """A, B, flow with gluing candidates: the objective after each B iteration never increases
    (Prop. "flow update decreases score")."""
    _need_gpu()
    g, o, eps = _pair(32, 2, angle=90.0)
    print("glued hybrid N=32 s=2", flush=True)
    E = [g.evaluate()["primal"]]
    for rnd in range(4):
        st = g.flow_update(eps_gamma=0.5 * eps)
        assert st["value"] <= 0.0
        g.iterate("A", eps, fixed_iters=60)
        g.iterate("B", eps, fixed_iters=60)
        E.append(g.evaluate()["primal"])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-9 * abs(E[0])), E
    with pytest.raises(Exception):
        g.flow_costs(eps_gamma=-1.0)
    g.close()


def test_flow_update_invariants_and_value():
    _need_gpu()
    g, o, eps = _pair(32, 2, angle=90.0)
    print("flow update N=32 s=2", flush=True)
    ev0 = g.evaluate()
    cg = g.flow_costs()
    st = g.flow_update()
    ores = o.flow_update()
    assert st["value"] <= 0.0 and st["moved_mass"] > 0.0 and st["n_active_arcs"] > 0
    # optimal values agree (the integer problems differ at most by rounding of the costs)
    assert abs(st["value"] - ores["value"]) <= 1e-9 * abs(ores["value"]) + 1e-15
    ev = g.evaluate()
    assert ev["y_marginal_l1"] <= ev0["y_marginal_l1"] + 1e-13
    assert ev["basic_mass_err"] <= 5 * 2.0 ** -40 + 1e-15
    g.close()


def test_hybrid_schedule_decreases_objective():
    """A, B, flow (Alg. "Hybrid"): the objective after each B iteration never increases."""
    _need_gpu()
    g, o, eps = _pair(32, 2, angle=90.0)
    print("hybrid N=32 s=2", flush=True)
    E = [g.evaluate()["primal"]]
    for rnd in range(4):
        g.flow_update()
        g.iterate("A", eps, fixed_iters=60)
        g.iterate("B", eps, fixed_iters=60)
        E.append(g.evaluate()["primal"])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-9 * abs(E[0])), E
    g.close()


def test_flow_requires_a_b_iteration():
    import paper_2405_09400_amd as dd
    _need_gpu()
    w = synth.workload("small32", N=16)
    g = dd.DomDec(w.mu, w.nu, w.s, prec=dd.DD_PREC_F64)
    with pytest.raises(dd.DomDecError) as e:
        g.flow_update()
    assert e.value.status == dd.DD_ESTATE
    g.iterate("A", w.kappas[0] / 256, fixed_iters=5)
    with pytest.raises(dd.DomDecError):
        g.flow_update()
    g.close()


def test_f32_flow_update_matches_oracle_on_the_gpu_state():
    """The flow workload's configuration at reduced size (512 -> 64, s = 2, map start, kappa = 1):
    float32 cell solves to tol 1e-5 with float64 mass bookkeeping, then a flow update.  The
    oracle replays the flow update from the GPU's own state (basic-cell Y-marginals and the B
    potentials, read through extract_plan and extract_potentials), so float32 rounding of the
    preceding solves drops out: edge costs match brute force, the optimal values agree, the
    oracle's flow applied on both sides gives the same marginals, and the GPU's own update keeps
    every basic cell's mass (sum_y nu_hat_j = m_j) and the Y-marginal."""
    import paper_2405_09400_amd as dd
    _need_gpu()
    w = synth.workload("flow512", N=64)
    print("flow f32 flow512 N=64 s=2", flush=True)
    g = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=dd.DD_PREC_F32)
    eps = w.kappas[-1] / w.N ** 2
    st = g.iterate("A", eps, tol=1e-5, stop_rule=dd.DD_STOP_BATCH, max_iter=20000)
    assert st["sk"]["converged"] == 1
    nu_pre = g.nu_i_sparse()
    st = g.iterate("B", eps, tol=1e-5, stop_rule=dd.DD_STOP_BATCH, max_iter=20000)
    assert st["sk"]["converged"] == 1
    nu_post = g.nu_i_sparse()
    pot = g.extract_potentials("B")
    ev0 = g.evaluate()
    cg = g.flow_costs()

    # the oracle on the same state: nu_i after B, and B's composite solves from its potentials
    cells = oracle.basic_cell_pixels(w.N, w.s)
    xs = np.concatenate([np.full(len(i), cells[k][0], np.int64) for k, (i, _) in enumerate(nu_post)])
    o = oracle.DomDec(w.mu, w.nu, w.s, (xs, np.concatenate([i for i, _ in nu_post]),
                                        np.concatenate([v for _, v in nu_post])))
    solves = []
    for J, basic in enumerate(o.parts["B"]):
        xpix = np.concatenate([o.cells[i] for i in basic])
        ysup, nuJ = oracle.sparse_sum([nu_pre[i] for i in basic])
        keep = nuJ > 0
        ysup, nuJ = ysup[keep], nuJ[keep]
        k1, k2 = np.divmod(xpix, w.N)
        xo = pot["xorig"][J]
        alpha = pot["alpha"][J][(k1 - xo[0]) * pot["xside"] + (k2 - xo[1])]
        y1, y2 = np.divmod(ysup, w.N)
        W2 = pot["ydims"][J][1]
        beta = pot["beta"][pot["ybase"][J] + (y1 - pot["yorig"][J][0]) * W2 + (y2 - pot["yorig"][J][1])]
        assert np.all(np.isfinite(beta))
        solves.append(oracle.CellSolve(basic, xpix, [len(o.cells[i]) for i in basic], ysup, nuJ,
                                       alpha, beta))
    o.last["B"] = solves
    o.last_eps["B"] = eps
    o.last_which = "B"
    res = o.flow_update(truncate=True)
    co = res["cbar"]
    assert np.max(np.abs(cg - co)) <= 1e-11 * np.max(np.abs(co)), np.max(np.abs(cg - co))
    # the oracle's flow keeps the masses: sum_j w_ij = m_i (to rounding), and sum_i w_ij = m_j
    # up to the integer supplies b_i = round(m_i 2^40): w_ij = flow_ij m_i / b_i differs from
    # flow_ij 2^-40 by at most flow_ij 2^-40 / b_i, so with flow_ij <= b_i the in-flow of a
    # cell misses m_j by at most 2^-40 per in-arc (5 arcs: 4.5e-12)
    tail, head = oracle.neighbourhood(w.N // w.s)
    assert np.abs(np.bincount(tail, res["w"], len(o.m)) - o.m).max() <= 1e-15
    assert np.abs(np.bincount(head, res["w"], len(o.m)) - o.m).max() <= 5 * 2.0 ** -40
    # the same flow on the GPU state gives the oracle's new marginals
    g.save()
    g.flow_apply(res["w"])
    G = _dense(g.nu_i_sparse(), w.N)
    O = _dense(o.nu_i, w.N)
    assert np.abs(G - O).sum() <= 1e-13
    # the GPU's own flow update: same optimal value, masses and Y-marginal kept
    # (a fresh context replays the same float32 solves: a restored state needs a new iteration
    # before a flow update)
    g2 = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=dd.DD_PREC_F32)
    g2.iterate("A", eps, tol=1e-5, stop_rule=dd.DD_STOP_BATCH, max_iter=20000)
    g2.iterate("B", eps, tol=1e-5, stop_rule=dd.DD_STOP_BATCH, max_iter=20000)
    assert np.max(np.abs(g2.flow_costs() - co)) <= 1e-11 * np.max(np.abs(co))
    fs = g2.flow_update()
    assert abs(fs["value"] - res["value"]) <= 1e-9 * abs(res["value"]) + 1e-15
    ev = g2.evaluate()
    assert ev["basic_mass_err"] <= 5 * 2.0 ** -40 + 1e-15
    assert ev["y_marginal_l1"] <= ev0["y_marginal_l1"] + 1e-13
    # and the cycle goes on: A, B after the flow, both converged, masses kept
    for part in "AB":
        st = g2.iterate(part, eps, tol=1e-5, stop_rule=dd.DD_STOP_BATCH, max_iter=20000)
        assert st["sk"]["converged"] == 1
    ev = g2.evaluate()
    assert ev["basic_mass_err"] <= 1e-11 and ev["x_marginal_l1"] <= 1e-5 * (1 + 1e-9)
    g.close()
    g2.close()
