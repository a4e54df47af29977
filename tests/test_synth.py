"""Seeded input generators: determinism, normalisation and exact couplings (no GPU)."""
import numpy as np

import synth


def test_mixture_seeded_and_normalised():
    a = synth.gaussian_mixture(64, 8, 1e-4, 3)
    b = synth.gaussian_mixture(64, 8, 1e-4, 3)
    c = synth.gaussian_mixture(64, 8, 1e-4, 4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert abs(a.sum() - 1.0) < 1e-14 and a.min() > 0


def test_kr_coupling_marginals():
    mu = synth.gaussian_mixture(64, 8, 1e-4, 0)
    nu = synth.gaussian_mixture(64, 8, 1e-4, 1000)
    x, y, m = synth.kr_coupling(mu, nu)
    assert np.all(m > 0)
    px = np.bincount(x, weights=m, minlength=64 * 64)
    py = np.bincount(y, weights=m, minlength=64 * 64)
    assert np.max(np.abs(px - mu.reshape(-1))) < 1e-15
    assert np.max(np.abs(py - nu.reshape(-1))) < 1e-15
    assert len(m) <= 4 * 64 * 64


def test_map_coupling_marginals_and_image():
    N = 64
    mu = synth.gaussian_mixture(N, 8, 1e-4, 0)
    tgt = synth.rotation_map(N, 30.0, 0.36)
    nu, (x, y, m) = synth.map_coupling(mu, tgt)
    assert abs(nu.sum() - 1.0) < 1e-14
    assert np.array_equal(x, np.arange(N * N))
    assert np.array_equal(np.bincount(y, weights=m, minlength=N * N), nu.reshape(-1))
