"""GPU parity of global_sinkhorn (the whole-grid Sinkhorn comparison solver) against the
oracle's dense float64 Sinkhorn on the same problem (one cell covering the grid, Y = supp nu):
plans at equal iteration counts, the converged solve against the oracle's global optimum, and
zero-mass pixels and grid sides that leave a ragged last tile.
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


def _problem(N, seed, holes=False):
    mu = synth.gaussian_mixture(N, 3, 1e-3, seed)
    nu = synth.gaussian_mixture(N, 3, 1e-3, seed + 1000)
    if holes:
        nu[: N // 4, : N // 3] = 0.0  # a block of zero mass in nu
        nu /= nu.sum()
    return mu, nu


def _gpu(mu, nu, eps, alpha0=None, **kw):
    import paper_2405_09400_amd as dd
    dev = torch.device("cuda:0")
    N = mu.shape[0]
    m = torch.tensor(mu, dtype=torch.float64, device=dev)
    v = torch.tensor(nu, dtype=torch.float64, device=dev)
    a = torch.zeros((N, N), dtype=torch.float64, device=dev) if alpha0 is None else \
        torch.tensor(alpha0, dtype=torch.float64, device=dev)
    b = torch.zeros_like(a)
    print(f"global_sinkhorn N={N} eps={eps:.3e} kw={kw}", flush=True)
    status, st = dd.global_sinkhorn(m, v, eps, a, b, **kw)
    torch.cuda.synchronize()
    return status, st, a.cpu().numpy().reshape(-1), b.cpu().numpy().reshape(-1)


def _oracle(mu, nu, eps, n_iter, alpha0=None):
    N = mu.shape[0]
    C = oracle.pixel_coords(N)
    m, v = mu.reshape(-1), nu.reshape(-1)
    ys = np.nonzero(v > 0)[0]
    a0 = np.zeros(N * N) if alpha0 is None else alpha0.reshape(-1)
    a, b, it, err, nit = oracle.sinkhorn_cells(np.array([0, N * N]), C, m, np.array([0, len(ys)]),
                                               C[ys], v[ys], v[ys], eps, fixed_iters=n_iter,
                                               alpha=a0)
    return oracle.cell_plan(C, m, a, C[ys], v[ys], b, eps), ys, err


@pytest.mark.parametrize("N,kappa,holes", [(16, 4.0, False), (18, 1.0, True), (32, 2.0, False),
                                           (30, 0.5, True)])
def test_fixed_iterations_match_oracle(N, kappa, holes):
    _need_gpu()
    mu, nu = _problem(N, 3, holes)
    eps = kappa / N ** 2
    rng = np.random.default_rng(N)
    a0 = rng.normal(0, 0.3 * eps, (N, N))
    status, st, a, b = _gpu(mu, nu, eps, alpha0=a0, fixed_iters=40)
    assert status == 0 and st["iters"] == 40
    P, ys, oerr = _oracle(mu, nu, eps, 40, alpha0=a0)
    C = oracle.pixel_coords(N)
    Pg = oracle.cell_plan(C, mu.reshape(-1), a, C[ys], nu.reshape(-1)[ys], b[ys], eps)
    assert np.abs(Pg - P).sum() <= 1e-11 * P.sum(), np.abs(Pg - P).sum()
    assert abs(st["err"] - float(oerr.sum())) <= 1e-12 + 1e-9 * float(oerr.sum())


def test_tolerance_solve_reaches_the_global_optimum():
    _need_gpu()
    N = 24
    mu, nu = _problem(N, 7)
    eps = 2.0 / N ** 2
    status, st, a, b = _gpu(mu, nu, eps, tol=1e-12, max_iter=20000)
    assert status == 0 and st["converged"] == 1 and st["err"] <= 1e-12
    _, _, P, _ = oracle.global_sinkhorn(mu, nu, eps, tol=1e-13)
    C = oracle.pixel_coords(N)
    ys = np.nonzero(nu.reshape(-1) > 0)[0]
    Pg = np.zeros_like(P)
    Pg[:, ys] = oracle.cell_plan(C, mu.reshape(-1), a, C[ys], nu.reshape(-1)[ys], b[ys], eps)
    Eg = oracle.primal_dense(mu, nu, Pg, eps)
    Eo = oracle.primal_dense(mu, nu, P, eps)
    assert abs(Eg - Eo) <= 1e-10 * abs(Eo)
    assert np.abs(Pg - P).sum() <= 1e-10


def test_iteration_cap_reports_notconv():
    import paper_2405_09400_amd as dd
    _need_gpu()
    mu, nu = _problem(16, 1)
    status, st, _, _ = _gpu(mu, nu, 1.0 / 256, tol=1e-14, max_iter=3, raise_on_error=False)
    assert status == dd.DD_NOTCONV and st["converged"] == 0 and st["iters"] == 3
