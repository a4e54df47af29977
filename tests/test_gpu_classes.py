"""The cell classes of the register-blocked path and their tuner (sinkhorn_set_classes): every
candidate pair of thresholds solves the same iteration -- the plans agree with the default's
to float32 rounding (a cell that changes class changes kernel: the one-wave kernel holds
log nu_J in float32 registers, the others read it in float64) and every candidate's with the
oracle's to the float32 bar -- the statistics report the pair used,
the tuner tries every candidate on consecutive solves of one batch and then settles, and
out-of-range thresholds are rejected.
"""
import numpy as np
import pytest

from cellcases import gpu_plan, oracle_solve, random_cells

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CANDIDATES = [(32, 2048), (32, 1024), (32, 4096), (24, 2048), (24, 1024), (24, 4096)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _cells():
    # boxes from 10 to 80 a side: every class under every candidate (long sides 25..32 move
    # between the one-wave and the four-wave class, 1024..4096 entries between four and eight)
    rng = np.random.default_rng(21)
    return random_cells(rng, 48, 8, 10, 80, 1.0)


def _solve(cells, **kw):
    import paper_2405_09400_amd as dd
    dev = _dev()
    n = len(cells["dims"])
    dims = torch.tensor(cells["dims"], dtype=torch.int32, device=dev).reshape(n, 2).contiguous()
    base = torch.tensor(cells["base"], dtype=torch.int64, device=dev)
    shift = torch.tensor(cells["shift"], dtype=torch.int32, device=dev).reshape(n, 2).contiguous()
    logmu = torch.tensor(cells["logmu"], dtype=torch.float64, device=dev).reshape(n, 64).contiguous()
    lognu = torch.tensor(cells["lognu"], dtype=torch.float64, device=dev)
    a = torch.zeros(n, 64, dtype=torch.float64, device=dev)
    b = torch.zeros_like(lognu)
    it = torch.zeros(n, dtype=torch.int32, device=dev)
    mw1 = int(cells["dims"][:, 0].max())
    mw2 = int(cells["dims"][:, 1].max())
    status, st = dd.sinkhorn_batch(dims, base, shift, logmu, lognu, a, b, cells["kappa"], mw1, mw2,
                                   prec=dd.DD_PREC_F32, cell_iters=it, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), it.cpu().numpy(), st, status


def test_every_candidate_solves_the_same_iteration():
    import paper_2405_09400_amd as dd
    cells = _cells()
    n = len(cells["dims"])
    plans = {}
    try:
        for ws, be in CANDIDATES:
            print(f"classes wave_side={ws} big_entries={be}: 40 iterations", flush=True)
            dd.set_classes(ws, be)
            a, b, it, st, status = _solve(cells, fixed_iters=40)
            assert status == 0 and st["path"] == 1
            assert (st["wave_side"], st["big_entries"]) == (ws, be)
            plans[(ws, be)] = [gpu_plan(cells, c, a, b) for c in range(n)]
    finally:
        dd.set_classes(0, 0)
    ref = plans[CANDIDATES[0]]
    O, oit, _, _ = oracle_solve(cells, fixed_iters=40)
    for key, ps in plans.items():
        worst = max(float(np.abs(p - q).sum() / q.sum()) for p, q in zip(ps, ref))
        assert worst <= 1e-6, (key, worst)
        # every candidate's plans are the oracle's to the float32 bar at the same count
        worst = max(float(np.abs(p - q).sum() / q.sum()) for p, q in zip(ps, O))
        assert worst <= 3e-5, (key, worst)


def test_tuner_tries_every_candidate_then_settles():
    import paper_2405_09400_amd as dd
    cells = _cells()
    dd.set_classes(0, 0)
    seen = []
    # a key of its own: a tolerance solve of this batch (mode, mean area, cell count)
    for k in range(len(CANDIDATES) + 3):
        print(f"tuned solve {k}", flush=True)
        _, _, _, st, status = _solve(cells, tol=1e-5, check_every=8)
        assert status == 0 and st["converged"] == 1 and st["path"] == 1
        seen.append((st["wave_side"], st["big_entries"]))
    assert sorted(set(seen[:len(CANDIDATES)])) == sorted(CANDIDATES)
    settled = seen[len(CANDIDATES):]
    assert len(set(settled)) == 1 and settled[0] in CANDIDATES


def test_out_of_range_classes_are_rejected():
    import paper_2405_09400_amd as dd
    _dev()
    for ws, be in ((7, 2048), (33, 2048), (32, 63), (32, 70000), (0, 2048)):
        with pytest.raises(dd.DomDecError):
            dd.set_classes(ws, be)
    dd.set_classes(0, 0)
