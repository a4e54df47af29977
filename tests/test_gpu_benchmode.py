"""Parity of the benchmark's own mode against the oracle, at the benchmark's full size.

The GPU runs the 512x512 mixture workload exactly as the benchmark does, from either of its
two set-ups: ms512 (the default: solved coarse to fine, layers 8^2 ... 256^2, then kappa = 2
on the finest layer) or mix512 (Knothe-Rosenblatt start, the eps schedule kappa = 64 ... 2,
4 half-iterations per stage); float32 with the float64 finish, batch stopping rule, tol 1e-5,
tests spaced from check_every = 8.  Then one half-iteration at kappa = 1 from the
previous-iterate start -- the timed step.  That solve
runs on the register-blocked path with all three cell classes (one, four and eight waves per
cell), device-chosen round lengths, the last-workgroup error reduction shared by the classes
and the float64 finish.

The oracle takes the same state just before that step (basic-cell Y-marginals and the
partition's X potentials, read through extract_plan and extract_potentials), and solves a
sample of the same composite cells (the largest boxes, cells of every class and random ones)
for the same number of Sinkhorn iterations (cell problems of one partition are independent,
and a fixed count from the same start reproduces the solve, so the stop rule drops out).
Compared: the new basic-cell Y-marginals, both marginals of each composite plan, and each
cell's objective (eq. entropic-transport restricted to the cell), at the bars of the method:
1e-5 relative on marginals and 1e-6 relative on the objective.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bench_state(name, seed=0):
    """The benchmark's untimed set-up: for mix512 the KR start and the eps schedule down to
    kappa = 2; for ms512 the coarse-to-fine solve (layers 8^2 ... 256^2 with their eps stages
    and refinements), then kappa = 2 on the 512^2 layer."""
    import paper_2405_09400_amd as dd
    w = synth.workload(name, seed=seed)
    levels = w.extra.get("levels", 0)
    g = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=dd.DD_PREC_F32, levels=levels)
    k = 0
    for _ in range(levels):
        for kappa in w.extra["layer_kappas"]:
            for _ in range(w.extra["layer_iters"]):
                g.iterate("AB"[k % 2], kappa / g.N ** 2, tol=TOL, stop_rule=dd.DD_STOP_BATCH,
                          max_iter=20000, check_every=8)
                k += 1
        g.refine()
    for kappa, its in zip(w.kappas[:-1], w.stage_iters[:-1]):
        eps = kappa / w.N ** 2
        for _ in range(its):
            g.iterate("AB"[k % 2], eps, tol=TOL, stop_rule=dd.DD_STOP_BATCH, max_iter=20000,
                      check_every=8)
            k += 1
    return w, g, k


def _oracle_from_state(w, nu_i):
    """An oracle DomDec whose state is the given basic-cell Y-marginals: the coupling puts the
    mass of nu_i on the first pixel of X_i, which the oracle aggregates back into nu_i."""
    cells = oracle.basic_cell_pixels(w.N, w.s)
    xs = np.concatenate([np.full(len(idx), cells[i][0], np.int64) for i, (idx, _) in enumerate(nu_i)])
    ys = np.concatenate([idx for idx, _ in nu_i])
    ms = np.concatenate([v for _, v in nu_i])
    return oracle.DomDec(w.mu, w.nu, w.s, (xs, ys, ms))


def _block_to_xpix(alpha_blk, xorig, xpix, N, xside):
    """GPU block potential (row-major over the 2s x 2s block at xorig) at the oracle's X pixels."""
    k1, k2 = np.divmod(xpix, N)
    return alpha_blk[(k1 - xorig[0]) * xside + (k2 - xorig[1])]


def _cell_objective(o, xpix, ysup, plan, eps):
    """<c, pi> + eps sum pi (log(pi / (mu nu)) - 1) over the cell (the cell's part of E(pi))."""
    d = o.coords[xpix][:, None, :] - o.coords[ysup][None, :, :]
    c = (d ** 2).sum(axis=2)
    ref = o.mu[xpix][:, None] * o.nu[ysup][None, :]
    pos = plan > 0
    return float((c * plan).sum() + eps * (plan[pos] * (np.log(plan[pos] / ref[pos]) - 1.0)).sum())


@pytest.mark.parametrize("name", ["mix512", "ms512"])
def test_benchmark_mode_matches_oracle_at_full_size(name):
    import paper_2405_09400_amd as dd
    _need_gpu()
    # the library's default cell classes, so that all three classes take part
    dd.set_classes(32, 2048)
    try:
        w, g, k = _bench_state(name)
        part = "AB"[k % 2]
        eps = w.kappas[-1] / w.N ** 2
        nu_before = g.nu_i_sparse()
        pre = g.extract_potentials(part, beta=False)
        print(f"bench mode {name} partition {part} after {k} half-iterations", flush=True)
        st = g.iterate(part, eps, tol=TOL, stop_rule=dd.DD_STOP_BATCH, max_iter=20000,
                       check_every=8, init=dd.DD_INIT_PREV)
    finally:
        dd.set_classes(0, 0)
    sk = st["sk"]
    # the benchmark's configuration: register-blocked path, all three classes, batch rule
    assert sk["path"] == 1 and sk["converged"] == 1
    assert sk["n_giant"] > 0 and sk["n_big"] > sk["n_giant"] and sk["ncells"] > sk["n_big"]
    assert sk["iters_min"] == sk["iters_max"] and sk["finish_iters_max"] >= 1
    n_its = sk["iters_max"]  # both phases
    nu_after = g.nu_i_sparse()
    post = g.extract_potentials(part)
    assert post["has_beta"] and abs(post["eps"] - eps) <= 1e-15 * eps
    g.close()

    o = _oracle_from_state(w, nu_before)
    parts = o.parts[part]
    xside = pre["xside"]
    # sample: the 6 largest boxes, 6 cells of each of the two smaller classes, 30 random
    dims = post["ydims"]
    entries = dims[:, 0].astype(np.int64) * dims[:, 1]
    longside = dims.max(axis=1)
    cls = np.where(longside <= 32, 0, np.where(entries > 2048, 2, 1))
    rng = np.random.default_rng(512)
    sample = set(np.argsort(entries)[-6:].tolist())
    for c in (0, 1):
        idx = np.nonzero(cls == c)[0]
        sample |= set(rng.choice(idx, min(6, len(idx)), replace=False).tolist())
    sample |= set(rng.choice(len(parts), 30, replace=False).tolist())
    sample = sorted(sample)
    assert {0, 1, 2} <= set(cls[sample].tolist())
    for J in sample:
        xpix = np.concatenate([o.cells[i] for i in parts[J]])
        o.alpha[part][J] = _block_to_xpix(pre["alpha"][J], pre["xorig"][J], xpix, w.N, xside)
    print(f"oracle: {len(sample)} cells, {n_its} iterations", flush=True)
    o.iterate(part, eps, fixed_iters=n_its, cells=sample)

    # basic-cell Y-marginals of the sampled cells
    worst_nu = 0.0
    for J in sample:
        for i in parts[J]:
            a = np.zeros(w.N * w.N)
            b = np.zeros(w.N * w.N)
            a[nu_after[i][0]] = nu_after[i][1]
            b[o.nu_i[i][0]] = o.nu_i[i][1]
            # entries at the 1e-15 truncation edge may be kept by one side only
            d = (np.abs(a - b).sum() - 64e-15) / o.m[i]
            worst_nu = max(worst_nu, d)
    # composite plans: marginals and objective
    worst_x = worst_y = worst_e = 0.0
    solves = {J: cs for J, cs in zip(sample, o.last[part])}
    for J in sample:
        cs = solves[J]
        xpix, ysup = cs.xpix, cs.ysup
        P_or = oracle.cell_plan(o.coords[xpix], o.mu[xpix], cs.alpha, o.coords[ysup], o.nu[ysup],
                                cs.beta, eps)
        a_g = _block_to_xpix(post["alpha"][J], pre["xorig"][J], xpix, w.N, xside)
        y1, y2 = np.divmod(ysup, w.N)
        W2 = post["ydims"][J][1]
        bidx = post["ybase"][J] + (y1 - post["yorig"][J][0]) * W2 + (y2 - post["yorig"][J][1])
        b_g = post["beta"][bidx]
        assert np.all(np.isfinite(b_g))
        P_g = oracle.cell_plan(o.coords[xpix], o.mu[xpix], a_g, o.coords[ysup], o.nu[ysup], b_g, eps)
        m = P_or.sum()
        worst_x = max(worst_x, np.abs(P_g.sum(1) - P_or.sum(1)).sum() / m)
        worst_y = max(worst_y, np.abs(P_g.sum(0) - P_or.sum(0)).sum() / m)
        e_or = _cell_objective(o, xpix, ysup, P_or, eps)
        e_g = _cell_objective(o, xpix, ysup, P_g, eps)
        worst_e = max(worst_e, abs(e_g - e_or) / abs(e_or))
    print(f"worst relative differences: basic nu_i {worst_nu:.2e}, X-marginal {worst_x:.2e}, "
          f"Y-marginal {worst_y:.2e}, objective {worst_e:.2e}", flush=True)
    assert worst_nu <= 1e-5
    assert worst_x <= 1e-5
    assert worst_y <= 1e-5
    assert worst_e <= 1e-6
