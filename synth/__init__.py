"""Seeded synthetic inputs for entropic-OT domain decomposition.

This module generates problem data only: the two marginals mu, nu on a regular
N x N grid of [0,1]^2 and, where a workload asks for one, the initial coupling
pi_init handed to the domain-decomposition driver (the input of the paper's
DomDec / Hybrid algorithms, Sec. 2.3 Alg. "DomDec" and Sec. 3.3 Alg. "Hybrid").
It holds none of the method's arithmetic (no Sinkhorn, no partitions, no
cell marginals, no flows); both the oracle and the GPU path consume it.

Grid convention: pixel (k1, k2) has centre ((k1 + 1/2) h, (k2 + 1/2) h) with
h = 1/N; arrays are row-major with k1 the slow axis, flat index k1 * N + k2.

Gaussian-mixture images stand in for the paper's test images (App. A.2.1,
"Test data": Gaussian mixtures with random variances, means and magnitudes),
which are not available.  Recipe: K isotropic Gaussians with means
~ U[0.1, 0.9]^2, std ~ U[0.05, 0.2], weights ~ U[0.5, 1.5]; the density at
pixel centres is divided by its maximum, a constant floor is added, and the
result is normalised to total mass 1.  RNG: numpy PCG64 seeded with `seed`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "gaussian_mixture",
    "Workload",
    "workload",
    "kr_coupling",
    "map_coupling",
    "rotation_map",
    "WORKLOADS",
]


def gaussian_mixture(N: int, K: int, floor: float, seed: int) -> np.ndarray:
    """Normalised K-blob Gaussian-mixture density on the N x N pixel grid (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(0.1, 0.9, size=(K, 2))
    sig = rng.uniform(0.05, 0.2, size=K)
    wts = rng.uniform(0.5, 1.5, size=K)
    t = (np.arange(N, dtype=np.float64) + 0.5) / N
    X1, X2 = np.meshgrid(t, t, indexing="ij")
    rho = np.zeros((N, N), dtype=np.float64)
    for k in range(K):
        d2 = (X1 - means[k, 0]) ** 2 + (X2 - means[k, 1]) ** 2
        rho += wts[k] * np.exp(-d2 / (2.0 * sig[k] ** 2))
    rho = rho / rho.max() + floor
    return rho / rho.sum()


def _nw_corner_1d(a: np.ndarray, b: np.ndarray):
    """North-west-corner coupling of two non-negative 1D vectors of equal total.

    Returns (ia, ib, mass) arrays: the monotone (quantile) coupling, built from the
    merged breakpoints of the two cumulative sums.  Pieces of zero length are dropped.
    """
    ca = np.cumsum(a)
    cb = np.cumsum(b)
    tot = min(ca[-1], cb[-1])
    ca[-1] = tot
    cb[-1] = tot
    brk = np.unique(np.concatenate([[0.0], ca, cb]))
    brk = brk[brk <= tot]
    lo, hi = brk[:-1], brk[1:]
    mass = hi - lo
    keep = mass > 0
    lo, hi, mass = lo[keep], hi[keep], mass[keep]
    mid = 0.5 * (lo + hi)
    ia = np.searchsorted(ca, mid, side="right")
    ib = np.searchsorted(cb, mid, side="right")
    ia = np.minimum(ia, len(a) - 1)
    ib = np.minimum(ib, len(b) - 1)
    return ia, ib, mass


def kr_coupling(mu: np.ndarray, nu: np.ndarray):
    """2D Knothe-Rosenblatt (north-west-corner) coupling as a sparse (x, y, mass) list.

    First the row marginals of mu and nu are coupled monotonically; each matched
    row pair (k1, l1) with mass p then couples the scaled conditional rows
    p * mu[k1, :] / mu_row[k1] and p * nu[l1, :] / nu_row[l1] monotonically.
    The result is a feasible coupling of (mu, nu) up to float64 rounding with
    O(N^2) entries, usable as an initial plan for fine grids where the product
    coupling would be dense.
    """
    N = mu.shape[0]
    mr = mu.sum(axis=1)
    nr = nu.sum(axis=1)
    r_a, r_b, r_m = _nw_corner_1d(mr, nr)
    xs, ys, ms = [], [], []
    for k1, l1, p in zip(r_a, r_b, r_m):
        ra = mu[k1] * (p / mr[k1])
        rb = nu[l1] * (p / nr[l1])
        c_a, c_b, c_m = _nw_corner_1d(ra, rb)
        xs.append(k1 * N + c_a)
        ys.append(l1 * N + c_b)
        ms.append(c_m)
    x = np.concatenate(xs).astype(np.int64)
    y = np.concatenate(ys).astype(np.int64)
    m = np.concatenate(ms)
    return x, y, m


def rotation_map(N: int, angle_deg: float, scale: float, shift=(0.25, 0.0)):
    """Pixel map k -> nearest pixel of T(x), T(x) = c + scale * R(angle) (x - c) + shift, c = (1/2, 1/2)."""
    t = (np.arange(N, dtype=np.float64) + 0.5) / N
    X1, X2 = np.meshgrid(t, t, indexing="ij")
    th = math.radians(angle_deg)
    c, s = math.cos(th), math.sin(th)
    d1, d2 = X1 - 0.5, X2 - 0.5
    T1 = 0.5 + scale * (c * d1 - s * d2) + shift[0]
    T2 = 0.5 + scale * (s * d1 + c * d2) + shift[1]
    k1 = np.clip(np.floor(T1 * N).astype(np.int64), 0, N - 1)
    k2 = np.clip(np.floor(T2 * N).astype(np.int64), 0, N - 1)
    return (k1 * N + k2).reshape(-1)


def map_coupling(mu: np.ndarray, target: np.ndarray):
    """(id, T)_# mu for a pixel map `target` (flat index per pixel): returns (nu, (x, y, mass))."""
    N = mu.shape[0]
    x = np.arange(N * N, dtype=np.int64)
    m = mu.reshape(-1).copy()
    nu = np.bincount(target, weights=m, minlength=N * N).reshape(N, N)
    keep = m > 0
    return nu, (x[keep], target[keep].astype(np.int64), m[keep])


@dataclass
class Workload:
    """One synthetic problem instance: marginals, cell size, eps schedule, init."""

    name: str
    N: int
    s: int
    mu: np.ndarray
    nu: np.ndarray
    kappas: list  # eps / h^2 per stage
    stage_iters: list  # DD iterations per stage
    init: Optional[tuple] = None  # sparse (x, y, mass) or None = product coupling
    seed: int = 0
    extra: dict = field(default_factory=dict)


def _kappa_schedule(k_max: int):
    ks = []
    k = k_max
    while k >= 1:
        ks.append(k)
        k //= 2
    return ks


def workload(name: str, seed: int = 0, N: Optional[int] = None) -> Workload:
    """Named workloads.

    small32   : 32x32, 3 blobs + 1e-3 floor, s=4, eps=(2h)^2, product init, 20 DD iterations.
    mix256    : 256x256, 8 blobs + 1e-4 floor, s=4, eps from (8h)^2 halving to h^2, KR init.
    flow512   : 512x512, mu = 8-blob mixture, nu = T_# mu with T = rotation by 30 deg,
                contraction 0.36 about the centre and translation (0.25, 0); s=2, eps=h^2,
                init (id, T)_# mu; hybrid DD + flow schedule.
    mix512    : the mix256 generator at 512x512 (s=4).
    mix1024   : 1024x1024, 16 blobs + 1e-4 floor, s=4, eps down to h^2, KR init.
    ms256, ms512, ms1024: the mixN marginals on a coarse-to-fine schedule (see the code); the
                extra fields hold the number of coarser layers and their eps stages.
    `N` overrides the grid size (used by tests to shrink a workload).
    """
    if name == "small32":
        n = N or 32
        mu = gaussian_mixture(n, 3, 1e-3, seed)
        nu = gaussian_mixture(n, 3, 1e-3, seed + 1000)
        return Workload(name, n, 4, mu, nu, [4.0], [20], None, seed)
    if name in ("mix256", "mix512", "mix1024"):
        n = N or {"mix256": 256, "mix512": 512, "mix1024": 1024}[name]
        K = 16 if name == "mix1024" else 8
        mu = gaussian_mixture(n, K, 1e-4, seed)
        nu = gaussian_mixture(n, K, 1e-4, seed + 1000)
        ks = [float(k) for k in _kappa_schedule(64)]
        its = [4] * (len(ks) - 1) + [20]
        return Workload(name, n, 4, mu, nu, ks, its, kr_coupling(mu, nu), seed)
    if name in ("ms256", "ms512", "ms1024"):
        # the mixture workloads of the same size and seed, solved coarse to fine: layers of
        # 2 x 2 block sums down to 8 x 8 (product coupling there; with s = 4 its A partition
        # is one cell), eps = 2h^2, h^2, h^2/2 on each coarser layer (h its pixel size), then
        # 2h^2 and h^2 on the finest, 8 half-iterations per stage
        base = workload("mix" + name[2:], seed=seed, N=N)
        levels = int(round(math.log2(base.N // 8)))
        return Workload(name, base.N, base.s, base.mu, base.nu, [2.0, 1.0], [8, 20], None, seed,
                        {"levels": levels, "layer_kappas": [2.0, 1.0, 0.5], "layer_iters": 8})
    if name == "flow512":
        n = N or 512
        mu = gaussian_mixture(n, 8, 1e-4, seed)
        tgt = rotation_map(n, 30.0, 0.36)
        nu, init = map_coupling(mu, tgt)
        return Workload(name, n, 2, mu, nu, [1.0], [100], init, seed, {"flow_every": 2})
    raise KeyError(name)


WORKLOADS = ("small32", "mix256", "flow512", "mix512", "mix1024", "ms256", "ms512", "ms1024")
