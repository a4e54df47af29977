"""sinkhorn_batch_noalloc (workspace in a fixed device buffer, no device allocation) against
sinkhorn_batch on the same inputs, through the C ABI: two calls in a row, the second with a
smaller batch, and a batch beyond the buffer rejected before anything is written.

The two entry points share their kernels and their arithmetic (every output has its own
fixed-order sums and the batch error is reduced in fixed cell order); only the streams differ
(the cell classes run one after the other on the caller's stream), so the results are
bit-identical.
"""
import numpy as np
import pytest

from cellcases import random_cells

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _tensors(cells, dev):
    n = len(cells["dims"])
    xs = cells["xside"]
    return dict(
        dims=torch.tensor(cells["dims"], dtype=torch.int32, device=dev).reshape(n, 2).contiguous(),
        base=torch.tensor(cells["base"], dtype=torch.int64, device=dev),
        shift=torch.tensor(cells["shift"], dtype=torch.int32, device=dev).reshape(n, 2).contiguous(),
        logmu=torch.tensor(cells["logmu"], dtype=torch.float64, device=dev).reshape(n, xs * xs).contiguous(),
        lognu=torch.tensor(cells["lognu"], dtype=torch.float64, device=dev))


def _solve(cells, t, a0, noalloc, **kw):
    import paper_2405_09400_amd as dd
    n = len(cells["dims"])
    a = a0.clone()
    b = torch.zeros_like(t["lognu"])
    it = torch.zeros(n, dtype=torch.int32, device=a.device)
    er = torch.zeros(n, dtype=torch.float64, device=a.device)
    mw1, mw2 = int(cells["dims"][:, 0].max()), int(cells["dims"][:, 1].max())
    print(f"sinkhorn_batch{'_noalloc' if noalloc else ''} n={n} kw={kw}", flush=True)
    status, st = dd.sinkhorn_batch(t["dims"], t["base"], t["shift"], t["logmu"], t["lognu"], a, b,
                                   cells["kappa"], mw1, mw2, prec=dd.DD_PREC_F32, cell_iters=it,
                                   cell_err=er, noalloc=noalloc, **kw)
    torch.cuda.synchronize()
    return status, st, a.cpu().numpy(), b.cpu().numpy(), it.cpu().numpy(), er.cpu().numpy()


@pytest.mark.parametrize("kw", [dict(tol=1e-5, stop_rule=0, max_iter=20000, check_every=8),
                                dict(tol=1e-5, stop_rule=1, max_iter=20000),
                                dict(fixed_iters=30)])
def test_noalloc_matches_sinkhorn_batch(kw):
    dev = _dev()
    rng = np.random.default_rng(9)
    # a large batch (all three register-blocked classes: boxes up to 80 a side), then a
    # smaller one of small boxes; the second call finds the first one's data in the buffer
    big = random_cells(rng, 300, 8, 4, 80, 1.0)
    small = random_cells(rng, 40, 8, 3, 20, 2.0)
    for cells in (big, small):
        t = _tensors(cells, dev)
        a0 = torch.tensor(rng.normal(0, 0.3, (len(cells["dims"]), 64)), dtype=torch.float64,
                          device=dev)
        ref = _solve(cells, t, a0, False, **kw)
        got = _solve(cells, t, a0, True, **kw)
        assert ref[0] == 0 and got[0] == 0
        for k in (2, 3, 4, 5):  # f, g, per-cell iterations, per-cell errors
            assert np.array_equal(ref[k], got[k]), k
        for key in ("iters_max", "iters_min", "converged", "finish_iters_max", "path", "err"):
            assert ref[1][key] == got[1][key], key


def test_noalloc_rejects_a_batch_beyond_its_buffer():
    import paper_2405_09400_amd as dd
    dev = _dev()
    # 150,000 cells of 2 x 2 boxes need more than the 64 MiB buffer (about 0.6 KB per cell,
    # most of it the second X-potential buffer of 64 doubles)
    n = 150_000
    dims = torch.full((n, 2), 2, dtype=torch.int32, device=dev)
    base = torch.arange(n, dtype=torch.int64, device=dev) * 4
    shift = torch.zeros((n, 2), dtype=torch.int32, device=dev)
    logmu = torch.full((n, 64), -9.0, dtype=torch.float64, device=dev)
    lognu = torch.full((4 * n,), -7.6, dtype=torch.float64, device=dev)
    a = torch.zeros((n, 64), dtype=torch.float64, device=dev)
    b = torch.full((4 * n,), 3.0, dtype=torch.float64, device=dev)
    print("sinkhorn_batch_noalloc oversize n=150000", flush=True)
    status, _ = dd.sinkhorn_batch(dims, base, shift, logmu, lognu, a, b, 1.0, 2, 2, tol=1e-5,
                                  noalloc=True, raise_on_error=False)
    torch.cuda.synchronize()
    assert status == dd.DD_EINVAL
    assert "no-allocation" in dd.lib().domdec_strerror(None, status).decode()
    assert float(a.abs().max()) == 0.0 and float((b - 3.0).abs().max()) == 0.0
