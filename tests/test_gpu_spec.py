"""One wait per domain-decomposition iteration (domdec_iterate): the composite boxes come from
the previous iteration and the float32 solve, its float64 finish and everything behind them
are enqueued whole; when that is not enough the solve is resumed after the wait.  Speculation
changes no arithmetic, so a trajectory with it (DD_SPEC unset) equals one without it
(DD_SPEC=0) bit for bit: basic-cell marginals, both partitions' potentials, iteration counts,
float64-finish counts and batch errors.  Three settings cover the three outcomes: the
benchmark's (the enqueued rounds suffice), rule tests one iteration apart from a zero start
(the float32 rounds are resumed), and no float64-finish iteration enqueued ahead
(DD_SPEC_FINISH=0: every finish is resumed from its start).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STAT_KEYS = ("iters_max", "iters_min", "finish_iters_max", "err", "mass", "cell_iters",
             "converged")


def _run(w, schedule, spec, finish=None, **opts):
    import paper_2405_09400_amd as dd
    old = os.environ.get("DD_SPEC")
    os.environ["DD_SPEC"] = "1" if spec else "0"
    if finish is not None:
        os.environ["DD_SPEC_FINISH"] = str(finish)
    try:
        g = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=dd.DD_PREC_F32)
        stats = []
        k = 0
        for kappa, n in schedule:
            eps = kappa / w.N ** 2
            for _ in range(n):
                stats.append(g.iterate("AB"[k % 2], eps, **opts))
                k += 1
        plan = g.extract_plan()
        pots = [g.extract_potentials(p, beta=False)["alpha"] for p in "AB"]
        g.close()
    finally:
        os.environ.pop("DD_SPEC_FINISH", None)
        if old is None:
            del os.environ["DD_SPEC"]
        else:
            os.environ["DD_SPEC"] = old
    return stats, plan, pots


@pytest.mark.parametrize("case", ["bench", "resume_rounds", "resume_finish"])
def test_speculative_iterations_equal_waiting_ones(case):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_09400_amd as dd
    w = synth.workload("mix256", seed=3, N=128)
    schedule = [(16.0, 2), (4.0, 2), (1.0, 6)]
    opts = {"bench": dict(tol=1e-5, check_every=8, max_iter=20000),
            "resume_rounds": dict(tol=1e-5, check_every=1, max_iter=20000, init=dd.DD_INIT_ZERO),
            "resume_finish": dict(tol=1e-5, check_every=8, max_iter=20000)}[case]
    finish = 0 if case == "resume_finish" else None
    print(f"spec {case} mix256 N=128 {opts}", flush=True)
    dd.set_classes(32, 2048)  # the class tuner would otherwise pick per run
    try:
        s1, plan1, pots1 = _run(w, schedule, True, finish, **opts)
        s0, plan0, pots0 = _run(w, schedule, False, **opts)
    finally:
        dd.set_classes(0, 0)
    for k, (a, b) in enumerate(zip(s1, s0)):
        for key in STAT_KEYS:
            assert a["sk"][key] == b["sk"][key], (k, key, a["sk"][key], b["sk"][key])
        assert a["nu_entries"] == b["nu_entries"], k
        assert b["spec_resumed"] == 0
    for x, y in zip(plan1, plan0):
        assert np.array_equal(x, y)
    for x, y in zip(pots1, pots0):
        assert np.array_equal(x, y)
    waits1 = [st["host_waits"] for st in s1]
    waits0 = [st["host_waits"] for st in s0]
    resumed = [st["spec_resumed"] for st in s1]
    print("host waits with / without speculation:", waits1, waits0, "resumed:", resumed)
    assert s1[0]["sk"]["path"] == 1  # the register-blocked path takes these batches
    # every later iteration plans from the predicted boxes: one wait unless resumed (a resumed
    # solve waits at most once more than one without speculation: the second end of the
    # iteration; with no finish iteration enqueued ahead its first read of the finish's stop
    # flag is one more)
    for k in range(1, len(s1)):
        if not resumed[k]:
            assert waits1[k] == 1, (k, waits1[k])
        assert waits1[k] <= waits0[k] + 1 + (finish == 0), (k, waits1[k], waits0[k])
    if case == "bench":
        # (the first solve enqueues four rounds, later ones one more than the last solve of
        # their partition needed; at kappa = 1 these solves from the kappa = 4 state take ~200
        # iterations in short rounds, more than the four enqueued ones)
        assert not resumed[0] and not all(resumed[:4])
    elif case == "resume_rounds":
        assert any(r and st["sk"]["iters_max"] > 72 for r, st in zip(resumed, s1))
    else:
        # the iterations whose float32 rounds stopped within the enqueued ones resume only
        # their finish
        assert all(resumed[:4])


def test_prediction_is_dropped_when_the_state_changes():
    """restore / refine / flow entry points change the state: the next iteration reads the
    composite boxes back instead of trusting the prediction (two waits), then predicts again."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_09400_amd as dd
    w = synth.workload("mix256", seed=1, N=64)
    eps = 4.0 / w.N ** 2
    g = dd.DomDec(w.mu, w.nu, w.s, w.init, prec=dd.DD_PREC_F32)
    print("spec prediction mix256 N=64", flush=True)
    dd.set_classes(32, 2048)  # the same cell classes for the replay
    try:
        a = g.iterate("A", eps)
        g.save()
        b = g.iterate("B", eps)
        c = g.iterate("A", eps)
        g.restore()  # back to the state after the first iteration
        d = g.iterate("B", eps)
        e = g.iterate("A", eps)
    finally:
        dd.set_classes(0, 0)
    print("waits", [x["host_waits"] for x in (a, b, c, d, e)],
          "resumed", [x["spec_resumed"] for x in (a, b, c, d, e)])
    # the replayed B iteration is the first one again, with one more wait (the boxes read back)
    for key in ("iters_max", "finish_iters_max", "err"):
        assert d["sk"][key] == b["sk"][key], key
        assert e["sk"][key] == c["sk"][key], key
    assert d["spec_resumed"] == b["spec_resumed"] and e["spec_resumed"] == c["spec_resumed"]
    assert d["host_waits"] == b["host_waits"] + 1
    assert e["host_waits"] == c["host_waits"]
    assert a["host_waits"] == b["host_waits"] + 1 or a["spec_resumed"] != b["spec_resumed"]
    g.close()
