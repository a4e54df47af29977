"""Pins of the oracle's coarse-to-fine step of multiscale domain decomposition (no GPU).

App. A.2.1 "Multi-scale and eps-scaling" and Sec. 5.3 use a coarse-to-fine scheme whose
refinement step the paper defers to earlier work; the oracle's reading (DomDec.refine) is
pinned by what any such step must satisfy and by closed forms:
  * the refined coupling is feasible: both marginal constraints hold exactly;
  * the refinement of a product coupling m_i nu is the product coupling of the fine layer;
  * the interpolation of the stitched potential reproduces affine functions exactly and keeps
    constants;
  * coarsening sums 2 x 2 blocks (total mass, a hand-computed case);
  * multiscale DD reaches the fine layer's global entropic optimum (Prop. "Convergence of the
    hybrid scheme" covers plain DD from any feasible start).
"""
import numpy as np
import pytest

import oracle
import synth


def _pair(N, seed=0, floor=1e-2):
    mu = synth.gaussian_mixture(N, 3, floor, seed)
    nu = synth.gaussian_mixture(N, 3, floor, seed + 1000)
    return mu, nu


def test_coarsen_sums_blocks():
    a = np.arange(16, dtype=np.float64).reshape(4, 4)
    c = oracle.coarsen(a)
    assert np.array_equal(c, np.array([[0 + 1 + 4 + 5, 2 + 3 + 6 + 7], [8 + 9 + 12 + 13, 10 + 11 + 14 + 15]],
                                      dtype=np.float64))
    mu, _ = _pair(32)
    assert abs(oracle.coarsen(mu).sum() - 1.0) < 1e-15


def test_upsample_reproduces_affine_functions():
    N = 6
    k1, k2 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    h, hf = 1.0 / N, 1.0 / (2 * N)
    x1, x2 = (k1 + 0.5) * h, (k2 + 0.5) * h
    a = 0.3 - 1.7 * x1 + 2.9 * x2
    f1, f2 = np.meshgrid((np.arange(2 * N) + 0.5) * hf, (np.arange(2 * N) + 0.5) * hf, indexing="ij")
    up = oracle.upsample_bilinear(a)
    assert np.abs(up - (0.3 - 1.7 * f1 + 2.9 * f2)).max() < 1e-14
    assert np.abs(oracle.upsample_bilinear(np.full((N, N), -4.25)) + 4.25).max() < 1e-15
    # a product of affine functions is bilinear: reproduced inside the outermost centres
    b = (1 + x1) * (2 - x2)
    inner = slice(1, 2 * N - 1)
    up = oracle.upsample_bilinear(b)
    assert np.abs(up[inner, inner] - ((1 + f1) * (2 - f2))[inner, inner]).max() < 1e-14


def _converged_coarse(N, s, seed, eps, its=12):
    mu_f, nu_f = _pair(N, seed)
    mu_c, nu_c = oracle.coarsen(mu_f), oracle.coarsen(nu_f)
    dd = oracle.DomDec(mu_c, nu_c, s)
    for k in range(its):
        dd.iterate("AB"[k % 2], eps, tol=1e-9, max_iter=5000)
    return dd, mu_f, nu_f


@pytest.mark.parametrize("N,s", [(16, 2), (32, 2), (32, 4)])
def test_refined_coupling_is_feasible(N, s):
    Nc = N // 2
    dd, mu_f, nu_f = _converged_coarse(N, s, 3, (2.0 / Nc) ** 2, its=6)
    fine = dd.refine(mu_f, nu_f)
    assert fine.N == N and len(fine.nu_i) == (N // s) ** 2
    # The coarse state is feasible up to its truncation (entries below 1e-15 dropped); the
    # refinement carries each coarse cell's mass and each coarse pixel's mass over exactly:
    #   sum_y' nu_i'(y') = (m_i' / m_i) sum_y nu_i(y),
    #   sum_i' nu_i'(y') = (nu_f(y') / nu(P(y'))) sum_i nu_i(P(y')).
    Nc, nc, nf = N // 2, N // 2 // s, N // s
    tot_c = np.zeros(Nc * Nc)
    for idx, val in dd.nu_i:
        np.add.at(tot_c, idx, val)
    tot = np.zeros(N * N)
    for i_f, ((idx, val), mi) in enumerate(zip(fine.nu_i, fine.m)):
        assert np.all(val > 0) and np.all(np.diff(idx) > 0)
        i_c = (i_f // nf // 2) * nc + (i_f % nf) // 2
        want = mi / dd.m[i_c] * dd.nu_i[i_c][1].sum()
        assert abs(val.sum() - want) <= 1e-14 * mi
        assert abs(val.sum() - mi) <= 2e-13  # the coarse truncation, shared out
        np.add.at(tot, idx, val)
    k1, k2 = np.divmod(np.arange(N * N), N)
    parent = (k1 // 2) * Nc + k2 // 2
    want = nu_f.reshape(-1) * tot_c[parent] / dd.nu[parent]
    assert np.abs(tot - want).max() <= 1e-14 * nu_f.max()
    assert np.abs(tot - nu_f.reshape(-1)).max() <= 1e-13
    # every composite cell of both fine partitions starts from the interpolated potential
    assert all(a is not None for w in "AB" for a in fine.alpha[w])


def test_refined_product_coupling_is_the_fine_product():
    N, s = 16, 2
    mu_f, nu_f = _pair(N, 5)
    coarse = oracle.DomDec(oracle.coarsen(mu_f), oracle.coarsen(nu_f), s)
    # potentials are needed for the refinement: one fixed-count visit of each partition
    for w in "AB":
        coarse.iterate(w, 1.0, fixed_iters=2, balance=False, truncate=False)
    # the visits moved the coupling: put the product coupling back
    sup = np.nonzero(coarse.nu > 0)[0]
    coarse.nu_i = [(sup.copy(), mi * coarse.nu[sup]) for mi in coarse.m]
    fine = coarse.refine(mu_f, nu_f)
    nf = nu_f.reshape(-1)
    for (idx, val), mi in zip(fine.nu_i, fine.m):
        assert np.array_equal(idx, np.nonzero(nf > 0)[0])
        assert np.abs(val - mi * nf[idx]).max() <= 1e-15 * mi * nf.max()


def test_refine_rejects_inconsistent_layers():
    dd, mu_f, nu_f = _converged_coarse(16, 2, 1, (2.0 / 8) ** 2, its=2)
    with pytest.raises(ValueError):
        dd.refine(mu_f * 1.01, nu_f)


def test_multiscale_dd_reaches_the_fine_global_optimum():
    """Coarse layer 8 x 8, then the fine 16 x 16 layer at its own eps: DD from the refined state
    converges to the fine global entropic optimum."""
    N, s = 16, 4
    eps = (2.0 / N) ** 2
    dd, mu_f, nu_f = _converged_coarse(N, s, 2, eps, its=4)
    fine = dd.refine(mu_f, nu_f)
    a, b, P, _ = oracle.global_sinkhorn(mu_f, nu_f, eps, tol=1e-13)
    Estar = oracle.primal_dense(mu_f, nu_f, P, eps)
    Es = []
    for k in range(60):
        fine.iterate("AB"[k % 2], eps, tol=1e-11, max_iter=5000)
        Es.append(fine.primal(eps))
    assert (Es[-1] - Estar) / Estar < 1e-9
    assert np.all(np.diff(Es[2:]) <= 1e-10 * abs(Es[0]))
