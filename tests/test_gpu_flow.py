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
