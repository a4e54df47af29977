"""Oracle: plain float64 CPU implementation of entropic-OT domain decomposition
with flow updates (Medina & Schmitzer, "Flow updates for domain decomposition of
entropic optimal transport").  TEST INFRASTRUCTURE ONLY: tests, the smoke check
and the benchmark's CPU-baseline leg may use it; the GPU product path never does.

It follows the paper's algorithms step by step in their notation:
  * cell problem and Sinkhorn: Sec. 2.2 eq. (entropic-transport), Prop. "Optimal
    entropic transport couplings", Sec. 2.3 Alg. "DomDecIter" (reference measure
    mu_J (x) nu), dense non-separable log-domain Sinkhorn in oracle.c;
  * basic-cell Y-marginals as the state: Sec. 2.3 eq. (basic-cell-Y-marginal);
  * partitions: Def. "Basic and composite partitions", App. A.2.1 (2x2 groups of
    s x s basic cells, B staggered by one basic cell; B boundary cells truncated);
  * balancing and truncation: App. A Alg. "DomDecIterGPU" (Balance, Truncate),
    truncation threshold 1e-15 (App. A.2.1);
  * flow update with product gluing candidates: Sec. 3.2 Def. "Flow update",
    eq. (edge-cost), eq. (flow-update-cell-marginals), Remark "eps-gamma";
    min-cost flow (MinCostFlow) by successive shortest paths in oracle.c;
  * evaluation: E, D and the primal-dual gap of App. A.2.2 "Solution quality".

Sparse storage: each basic-cell Y-marginal nu_i is a sorted index array plus a
value array on the flattened N*N Y grid.  Readings of points where the paper is
silent are listed in the project's design notes and restated at each function.

Pinned by tests/test_oracle_*.py against closed forms, invariants and brute force.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.POINTER(ctypes.c_int64)
        i32 = ctypes.POINTER(ctypes.c_int32)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_sinkhorn_cells.restype = ctypes.c_int
        L.orc_sinkhorn_cells.argtypes = [ctypes.c_int, i64, d, d, i64, d, d, d, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         d, d, ip, d, ctypes.c_int]
        L.orc_cell_plan.restype = None
        L.orc_cell_plan.argtypes = [ctypes.c_int, d, d, d, ctypes.c_int, d, d, d, ctypes.c_double, d]
        L.orc_mcf_ssp.restype = ctypes.c_int
        L.orc_mcf_ssp.argtypes = [ctypes.c_int, ctypes.c_int, i32, i32, i64, i64, i64, i64, i64]
        _LIB = L
    return _LIB


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------------------
# C entry points
# ---------------------------------------------------------------------------

def sinkhorn_cells(xoff, xc, mu, yoff, yc, nuJ, nuref, eps, tol=1e-5, max_iter=10000,
                   fixed_iters=0, rule=0, alpha=None, nthreads=0):
    """Batch cell Sinkhorn (see oracle.c).  Returns (alpha, beta, iters, err, n_iter)."""
    xoff = np.ascontiguousarray(xoff, dtype=np.int64)
    yoff = np.ascontiguousarray(yoff, dtype=np.int64)
    xc = np.ascontiguousarray(xc, dtype=np.float64)
    yc = np.ascontiguousarray(yc, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    nuJ = np.ascontiguousarray(nuJ, dtype=np.float64)
    nuref = np.ascontiguousarray(nuref, dtype=np.float64)
    nc = len(xoff) - 1
    a = np.zeros(int(xoff[-1]), dtype=np.float64) if alpha is None else np.array(alpha, dtype=np.float64)
    b = np.zeros(int(yoff[-1]), dtype=np.float64)
    iters = np.zeros(nc, dtype=np.int32)
    err = np.zeros(nc, dtype=np.float64)
    n = lib().orc_sinkhorn_cells(nc, _p(xoff, ctypes.c_int64), _p(xc, ctypes.c_double),
                                 _p(mu, ctypes.c_double), _p(yoff, ctypes.c_int64),
                                 _p(yc, ctypes.c_double), _p(nuJ, ctypes.c_double),
                                 _p(nuref, ctypes.c_double), float(eps), float(tol), int(max_iter),
                                 int(fixed_iters), int(rule), _p(a, ctypes.c_double),
                                 _p(b, ctypes.c_double), _p(iters, ctypes.c_int),
                                 _p(err, ctypes.c_double), int(nthreads))
    return a, b, iters, err, n


def cell_plan(xc, mu, alpha, yc, nuref, beta, eps):
    """Dense pi(x,y) = exp((alpha+beta-c)/eps) mu nu for one cell (nx x ny)."""
    xc = np.ascontiguousarray(xc, dtype=np.float64)
    yc = np.ascontiguousarray(yc, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    nuref = np.ascontiguousarray(nuref, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    nx, ny = len(mu), len(nuref)
    out = np.empty((nx, ny), dtype=np.float64)
    lib().orc_cell_plan(nx, _p(xc, ctypes.c_double), _p(mu, ctypes.c_double),
                        _p(alpha, ctypes.c_double), ny, _p(yc, ctypes.c_double),
                        _p(nuref, ctypes.c_double), _p(beta, ctypes.c_double), float(eps),
                        _p(out, ctypes.c_double))
    return out


def mcf_ssp(n, tail, head, cost, sup, dem):
    """Integer bipartite min-cost flow (see oracle.c).  Returns (flow, potentials, status)."""
    tail = np.ascontiguousarray(tail, dtype=np.int32)
    head = np.ascontiguousarray(head, dtype=np.int32)
    cost = np.ascontiguousarray(cost, dtype=np.int64)
    sup = np.ascontiguousarray(sup, dtype=np.int64)
    dem = np.ascontiguousarray(dem, dtype=np.int64)
    m = len(tail)
    flow = np.zeros(m, dtype=np.int64)
    pot = np.zeros(2 * n, dtype=np.int64)
    st = lib().orc_mcf_ssp(int(n), int(m), _p(tail, ctypes.c_int32), _p(head, ctypes.c_int32),
                           _p(cost, ctypes.c_int64), _p(sup, ctypes.c_int64), _p(dem, ctypes.c_int64),
                           _p(flow, ctypes.c_int64), _p(pot, ctypes.c_int64))
    return flow, pot, st


# ---------------------------------------------------------------------------
# Grid, partitions
# ---------------------------------------------------------------------------

def pixel_coords(N: int) -> np.ndarray:
    """(N*N, 2) pixel-centre coordinates ((k1+1/2)/N, (k2+1/2)/N), row-major."""
    t = (np.arange(N, dtype=np.float64) + 0.5) / N
    X1, X2 = np.meshgrid(t, t, indexing="ij")
    return np.stack([X1.reshape(-1), X2.reshape(-1)], axis=1)


def basic_cell_pixels(N: int, s: int) -> List[np.ndarray]:
    """Pixels of basic cell i = r*n + c (n = N/s): the s x s block at rows r*s.., cols c*s.."""
    n = N // s
    out = []
    for r in range(n):
        for c in range(n):
            k1 = np.arange(r * s, (r + 1) * s)
            k2 = np.arange(c * s, (c + 1) * s)
            out.append((k1[:, None] * N + k2[None, :]).reshape(-1).astype(np.int64))
    return out


def composite_partition(n: int, which: str) -> List[List[int]]:
    """Composite cells as ascending lists of basic-cell ids.

    A: 2x2 groups starting at the origin.  B: 2x2 groups shifted by one basic
    cell in both axes, cells at the boundary keep only their in-range members.
    """
    cells = []
    if which == "A":
        for R in range(n // 2):
            for C in range(n // 2):
                cells.append([(2 * R + dr) * n + (2 * C + dc) for dr in (0, 1) for dc in (0, 1)])
    elif which == "B":
        for R in range(n // 2 + 1):
            for C in range(n // 2 + 1):
                ids = []
                for dr in (0, 1):
                    for dc in (0, 1):
                        r, c = 2 * R - 1 + dr, 2 * C - 1 + dc
                        if 0 <= r < n and 0 <= c < n:
                            ids.append(r * n + c)
                cells.append(ids)
    else:
        raise ValueError(which)
    return cells


def neighbourhood(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """4-neighbourhood plus self loops on the n x n basic-cell grid (Def. neighbourhood set).

    Arcs are listed per tail node in ascending head order: (r-1,c), (r,c-1), (r,c), (r,c+1), (r+1,c).
    """
    tails, heads = [], []
    for r in range(n):
        for c in range(n):
            i = r * n + c
            for dr, dc in ((-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)):
                rr, cc = r + dr, c + dc
                if 0 <= rr < n and 0 <= cc < n:
                    tails.append(i)
                    heads.append(rr * n + cc)
    return np.array(tails, dtype=np.int32), np.array(heads, dtype=np.int32)


# ---------------------------------------------------------------------------
# Sparse helpers
# ---------------------------------------------------------------------------

def sparse_sum(parts: List[Tuple[np.ndarray, np.ndarray]]) -> Tuple[np.ndarray, np.ndarray]:
    """Sum of sparse vectors (idx, val) -> sorted union support."""
    if not parts:
        return np.zeros(0, np.int64), np.zeros(0)
    idx = np.concatenate([p[0] for p in parts])
    val = np.concatenate([p[1] for p in parts])
    u, inv = np.unique(idx, return_inverse=True)
    out = np.zeros(len(u))
    np.add.at(out, inv, val)
    return u, out


def largest_remainder(m: np.ndarray, total: int) -> np.ndarray:
    """Integers b_i >= 0 with sum b_i == total, b_i = floor(total * m_i / sum m) + 1 for the
    largest remainders (ties by index)."""
    q = m / m.sum() * total
    b = np.floor(q).astype(np.int64)
    rem = int(total - b.sum())
    if rem > 0:
        frac = q - b
        order = np.lexsort((np.arange(len(m)), -frac))
        b[order[:rem]] += 1
    return b


# ---------------------------------------------------------------------------
# Domain decomposition state
# ---------------------------------------------------------------------------

@dataclass
class CellSolve:
    """What one DD iteration keeps of a composite cell: geometry and potentials."""
    basic: List[int]
    xpix: np.ndarray  # X pixels (flat), basic cells concatenated in `basic` order
    xcount: List[int]  # pixels per basic cell
    ysup: np.ndarray  # support of nu_J (flat Y pixels)
    nuJ: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray


class DomDec:
    """Oracle domain-decomposition state: basic-cell Y-marginals nu_i (sparse, float64).

    mu, nu: (N, N) float64 probability arrays; s: basic cell size; init: None for
    the product coupling nu_i = m_i nu, else a sparse (x, y, mass) list.
    """

    TRUNC = 1e-15

    def __init__(self, mu: np.ndarray, nu: np.ndarray, s: int, init=None, trunc: float = 1e-15):
        self._setup(mu, nu, s, trunc)
        N = self.N
        if init is None:
            sup = np.nonzero(self.nu > 0)[0].astype(np.int64)
            for mi in self.m:
                self.nu_i.append((sup.copy(), mi * self.nu[sup]))
        else:
            x, y, w = init
            cell_of_pix = np.empty(N * N, dtype=np.int64)
            for i, p in enumerate(self.cells):
                cell_of_pix[p] = i
            ci = cell_of_pix[np.asarray(x)]
            key = ci * (N * N) + np.asarray(y, dtype=np.int64)
            u, inv = np.unique(key, return_inverse=True)
            acc = np.zeros(len(u))
            np.add.at(acc, inv, np.asarray(w, dtype=np.float64))
            cid = u // (N * N)
            yy = u % (N * N)
            starts = np.searchsorted(cid, np.arange(len(self.cells) + 1))
            for i in range(len(self.cells)):
                self.nu_i.append((yy[starts[i]:starts[i + 1]].copy(), acc[starts[i]:starts[i + 1]].copy()))

    def _setup(self, mu: np.ndarray, nu: np.ndarray, s: int, trunc: float) -> None:
        """Grid, basic cells and their masses, partitions; no coupling yet."""
        N = mu.shape[0]
        assert mu.shape == (N, N) and nu.shape == (N, N) and N % (2 * s) == 0
        self.N, self.s, self.n = N, s, N // s
        self.h = 1.0 / N
        self.mu = mu.reshape(-1).astype(np.float64)
        self.nu = nu.reshape(-1).astype(np.float64)
        self.coords = pixel_coords(N)
        self.cells = basic_cell_pixels(N, s)
        self.m = np.array([self.mu[p].sum() for p in self.cells])
        if np.any(self.m <= 0):
            raise ValueError("every basic cell needs positive mass")
        self.trunc = trunc
        self.nu_i: List[Tuple[np.ndarray, np.ndarray]] = []
        self.parts = {w: composite_partition(self.n, w) for w in ("A", "B")}
        self.alpha: Dict[str, List[Optional[np.ndarray]]] = {
            w: [None] * len(self.parts[w]) for w in ("A", "B")}
        self.last: Dict[str, List[CellSolve]] = {}
        self.last_eps: Dict[str, float] = {}
        self.last_which: Optional[str] = None

    # -- DomDecIter -----------------------------------------------------------
    def iterate(self, which: str, eps: float, tol: float = 1e-5, max_iter: int = 10000,
                fixed_iters: int = 0, rule: int = 0, nthreads: int = 0, balance: bool = True,
                truncate: bool = True, cells=None) -> dict:
        """One DomDecIter on partition `which` (Alg. "DomDecIter"; App. A Alg. "DomDecIterGPU").

        For each composite cell J: mu_J = mu on X_J, nu_J = sum of its basic nu_i,
        solve the cell problem by Sinkhorn (warm start: the alpha of the previous
        visit of this partition, zero on the first visit), set nu_i(y) =
        sum_{x in X_i} pi_J(x, y), then balance the basic masses inside J and
        truncate entries below 1e-15.

        `cells` (optional) restricts the iteration to those composite cells; the cells of
        one partition are independent problems (disjoint X_J), so the others are unchanged.
        With a subset and the batch stopping rule the stopping test covers the subset only.
        """
        parts = self.parts[which]
        sel = range(len(parts)) if cells is None else sorted(set(int(c) for c in cells))
        xoffs, yoffs = [0], [0]
        xcs, mus, ycs, nuJs, nurefs, als, geo = [], [], [], [], [], [], []
        for J in sel:
            basic = parts[J]
            xpix = np.concatenate([self.cells[i] for i in basic])
            ysup, nuJ = sparse_sum([self.nu_i[i] for i in basic])
            keep = nuJ > 0
            ysup, nuJ = ysup[keep], nuJ[keep]
            a0 = self.alpha[which][J]
            if a0 is None:
                a0 = np.zeros(len(xpix))
            xcs.append(self.coords[xpix])
            mus.append(self.mu[xpix])
            ycs.append(self.coords[ysup])
            nuJs.append(nuJ)
            nurefs.append(self.nu[ysup])
            als.append(a0)
            xoffs.append(xoffs[-1] + len(xpix))
            yoffs.append(yoffs[-1] + len(ysup))
            geo.append((basic, xpix, [len(self.cells[i]) for i in basic], ysup, nuJ))
        a, b, iters, err, nit = sinkhorn_cells(
            np.array(xoffs), np.concatenate(xcs), np.concatenate(mus), np.array(yoffs),
            np.concatenate(ycs), np.concatenate(nuJs), np.concatenate(nurefs), eps, tol, max_iter,
            fixed_iters, rule, np.concatenate(als), nthreads)
        solves = []
        for n, (J, (basic, xpix, xcount, ysup, nuJ)) in enumerate(zip(sel, geo)):
            aJ = a[xoffs[n]:xoffs[n + 1]].copy()
            bJ = b[yoffs[n]:yoffs[n + 1]].copy()
            self.alpha[which][J] = aJ
            solves.append(CellSolve(basic, xpix, xcount, ysup, nuJ, aJ, bJ))
            plan = cell_plan(self.coords[xpix], self.mu[xpix], aJ, self.coords[ysup], self.nu[ysup],
                             bJ, eps)
            row = 0
            new = []
            for k, i in enumerate(basic):
                new.append(plan[row:row + xcount[k]].sum(axis=0))
                row += xcount[k]
            if balance:
                self._balance(basic, new)
            for k, i in enumerate(basic):
                v = new[k]
                if truncate:
                    keep = v >= self.trunc
                    self.nu_i[i] = (ysup[keep].copy(), v[keep].copy())
                else:
                    self.nu_i[i] = (ysup.copy(), v.copy())
        self.last[which] = solves
        self.last_eps[which] = eps
        self.last_which = which
        return {"iters": iters, "err": err, "n_iter": nit,
                "err_total": float(err.sum()), "mass": float(np.concatenate(mus).sum())}

    def _balance(self, basic: List[int], new: List[np.ndarray]) -> None:
        """Restore sum_y nu_i = m_i inside one composite cell, keeping sum_i nu_i fixed.

        Reading (the balancing routine is deferred to another paper): basic cells with
        excess e_i = sum nu_i - m_i > 0 and with deficit e_k < 0 are paired in
        ascending order; t = min(e_i, -e_k) moves from i to k pointwise in proportion
        to nu_i: moved = (t / M_i) nu_i, nu_k += moved, nu_i -= moved.  Each step zeroes
        one excess or deficit, so at most |J|-1 transfers occur; entries stay >= 0.
        """
        M = [float(v.sum()) for v in new]
        e = [M[k] - self.m[i] for k, i in enumerate(basic)]
        while True:
            src = next((k for k in range(len(basic)) if e[k] > 0), None)
            dst = next((k for k in range(len(basic)) if e[k] < 0), None)
            if src is None or dst is None:
                break
            t = min(e[src], -e[dst])
            f = t / M[src]
            moved = f * new[src]
            new[dst] = new[dst] + moved
            new[src] = new[src] - moved
            M[src] -= t
            M[dst] += t
            if e[src] <= -e[dst]:
                e[dst] += e[src]
                e[src] = 0.0
            else:
                e[src] += e[dst]
                e[dst] = 0.0

    # -- batching and clustering (App. A.1 "Batching and clustering") ------------
    def composite_box_dims(self, which: str) -> np.ndarray:
        """(W1, W2) of each composite cell's Y bounding box: the smallest pixel rectangle
        holding the supports of its basic cells' nu_i (rows, then columns)."""
        N = self.N
        out = np.zeros((len(self.parts[which]), 2), dtype=np.int64)
        for J, basic in enumerate(self.parts[which]):
            sup = np.concatenate([self.nu_i[i][0] for i in basic])
            r, c = sup // N, sup % N
            out[J] = (r.max() - r.min() + 1, c.max() - c.min() + 1)
        return out

    def iterate_batched(self, which: str, eps: float, k: int, **kw) -> dict:
        """CreateBatches / CombineBatches: cluster the composite cells of `which` by their
        bounding-box dimensions (kmeans_boxes) and run DomDecIter on one cluster after the
        other, each with its own stopping test.  The clusters are formed from the state
        before the iteration; the cells of one partition are independent, so solving them
        in sequence is the same as one batch apart from the stopping rule's scope."""
        groups = kmeans_boxes(self.composite_box_dims(which), k)
        stats = []
        for g in groups:
            stats.append(self.iterate(which, eps, cells=g, **kw))
        self.last_which = None  # the composite plans were split over the batches
        return {"batches": groups, "stats": stats}

    # -- ε rescaling is implicit: alpha is kept in energy units across eps changes.

    # -- evaluation -----------------------------------------------------------
    def y_marginal_error(self) -> float:
        """L1 error of sum_i nu_i against nu."""
        tot = np.zeros(self.N * self.N)
        for idx, val in self.nu_i:
            np.add.at(tot, idx, val)
        return float(np.abs(tot - self.nu).sum())

    def basic_mass_error(self) -> float:
        """max_i |sum_y nu_i - m_i| (balancing target)."""
        return float(max(abs(v.sum() - mi) for (_, v), mi in zip(self.nu_i, self.m)))

    def cell_plans(self, which: Optional[str] = None):
        """Dense composite plans of the last iteration on `which`: list of (xpix, ysup, plan)."""
        which = which or self.last_which
        eps = self.last_eps[which]
        out = []
        for cs in self.last[which]:
            plan = cell_plan(self.coords[cs.xpix], self.mu[cs.xpix], cs.alpha,
                             self.coords[cs.ysup], self.nu[cs.ysup], cs.beta, eps)
            out.append((cs.xpix, cs.ysup, plan))
        return out

    def x_marginal_error(self, which: Optional[str] = None) -> float:
        """L1 error of the X-marginal of the composite plans of the last iteration."""
        e = 0.0
        for xpix, _, plan in self.cell_plans(which):
            e += float(np.abs(plan.sum(axis=1) - self.mu[xpix]).sum())
        return e

    def primal(self, eps: float, which: Optional[str] = None) -> float:
        """E(pi) = <c, pi> + eps KL(pi | mu (x) nu) of the composite plans (eq. KL, eq.
        entropic-transport): KL = sum_{pi>0} [pi log(pi/(mu nu)) - pi] + sum_{x,y} mu(x) nu(y)."""
        E = 0.0
        for xpix, ysup, plan in self.cell_plans(which):
            d = self.coords[xpix][:, None, :] - self.coords[ysup][None, :, :]
            c = (d ** 2).sum(axis=2)
            ref = self.mu[xpix][:, None] * self.nu[ysup][None, :]
            pos = plan > 0
            E += float((c * plan).sum())
            E += eps * float((plan[pos] * np.log(plan[pos] / ref[pos]) - plan[pos]).sum())
        return E + eps * float(self.mu.sum() * self.nu.sum())

    def stitched_dual(self, eps: float):
        """A global dual point from the composite-cell potentials and its value D.

        The cell potentials alpha_J are each defined up to a constant (Sec. 2.3, the gauge of
        the cell problem).  Offsets s_J are fixed by a breadth-first walk over the graph whose
        nodes are the A and B composite cells and whose edges are their overlaps (one basic
        cell each): starting from A cell 0 with s = 0, an edge through basic cell i sets the
        new cell's offset so that the mu-weighted mean of alpha_A - s_A and alpha_B - s_B on
        X_i agree.  Cells are expanded in FIFO order and neighbours through members taken in
        ascending basic-cell order.  Then alpha^dagger = alpha_J - s_J on the A cells, and
        beta^dagger is its exact Y-update against mu (x) nu,
            beta(y) = -eps log sum_x mu(x) exp((alpha(x) - c(x, y)) / eps),
        so that D(alpha, beta) = <alpha, mu> + <beta, nu> (dual_value's last term vanishes).
        Returns (D, alpha^dagger, beta^dagger); beta is nan off supp nu."""
        alpha = self.stitched_alpha()
        sup = self.nu > 0
        N2 = self.N * self.N
        beta = np.full(N2, np.nan)
        C = self.coords
        for y in np.nonzero(sup)[0]:
            z = (alpha - ((C - C[y]) ** 2).sum(axis=1)) / eps
            pos = self.mu > 0
            zm = z[pos].max()
            beta[y] = -eps * (zm + np.log((self.mu[pos] * np.exp(z[pos] - zm)).sum()))
        D = float((alpha * self.mu).sum() + (beta[sup] * self.nu[sup]).sum())
        return D, alpha, beta

    def stitched_alpha(self) -> np.ndarray:
        """alpha^dagger of stitched_dual: the A cells' potentials (energy units) with the offsets
        of the breadth-first walk over the A/B overlap graph, on every pixel."""
        if any(a is None for a in self.alpha["A"]) or any(a is None for a in self.alpha["B"]):
            raise ValueError("stitched_dual needs both partitions visited")
        N2 = self.N * self.N
        aX = {}
        own = {}
        for which in "AB":
            arr = np.zeros(N2)
            o = np.full(len(self.cells), -1)
            for J, basic in enumerate(self.parts[which]):
                xpix = np.concatenate([self.cells[i] for i in basic])
                arr[xpix] = self.alpha[which][J]
                o[basic] = J
            aX[which], own[which] = arr, o
        d = np.array([float((self.mu[p] * (aX["A"][p] - aX["B"][p])).sum()) / mi
                      for p, mi in zip(self.cells, self.m)])
        sA = np.full(len(self.parts["A"]), np.nan)
        sB = np.full(len(self.parts["B"]), np.nan)
        sA[0] = 0.0
        queue = [("A", 0)]
        head = 0
        while head < len(queue):
            which, J = queue[head]
            head += 1
            for i in sorted(self.parts[which][J]):
                if which == "A":
                    K = own["B"][i]
                    if np.isnan(sB[K]):
                        sB[K] = sA[J] - d[i]
                        queue.append(("B", K))
                else:
                    K = own["A"][i]
                    if np.isnan(sA[K]):
                        sA[K] = sB[J] + d[i]
                        queue.append(("A", K))
        alpha = aX["A"].copy()
        for J, basic in enumerate(self.parts["A"]):
            for i in basic:
                alpha[self.cells[i]] -= sA[J]
        return alpha

    # -- multiscale ---------------------------------------------------------------
    def refine(self, mu_f: np.ndarray, nu_f: np.ndarray) -> "DomDec":
        """The coarse-to-fine step of multiscale domain decomposition (App. A.2.1 "Multi-scale and
        eps-scaling", Sec. 5.3): the state of the next layer, on the 2N x 2N grid whose 2 x 2
        pixel sums are this layer's mu and nu, with the same basic-cell side s.  The paper defers
        the step to earlier work; the reading taken here:
          * coupling: a fine basic cell i' is one of the 2 x 2 children of a coarse basic cell i,
            and a fine pixel y' one of the 2 x 2 children of a coarse pixel y = P(y'); the coarse
            mass nu_i(y) is split among the X children in proportion to their mu mass and among
            the Y children in proportion to the fine nu:
                nu_i'(y') = (m_i' / m_i) nu_i(P(y')) nu_f(y') / nu(P(y')),
            so that sum_y' nu_i'(y') = m_i' and sum_i' nu_i'(y') = nu_f(y') hold exactly;
          * potentials: the stitched global alpha of this layer (energy units,
            stitched_alpha), interpolated bilinearly at the fine pixel centres (linearly
            extrapolated beyond the outermost coarse centres), is the starting alpha of every
            composite cell of both fine partitions (their first visit is a previous-iterate
            start from it)."""
        N, Nf, s = self.N, 2 * self.N, self.s
        mu_f = np.asarray(mu_f, np.float64).reshape(Nf, Nf)
        nu_f = np.asarray(nu_f, np.float64).reshape(Nf, Nf)
        if np.abs(coarsen(mu_f).reshape(-1) - self.mu).max() > 1e-12 or \
                np.abs(coarsen(nu_f).reshape(-1) - self.nu).max() > 1e-12:
            raise ValueError("refine: the fine marginals must sum to this layer's over 2 x 2 blocks")
        alpha_c = self.stitched_alpha().reshape(N, N)
        fine = DomDec.__new__(DomDec)
        fine._setup(mu_f, nu_f, s, self.trunc)
        nf = fine.n
        # coupling
        nu_c = self.nu
        for r in range(nf):
            for c in range(nf):
                i_f = r * nf + c
                i_c = (r // 2) * self.n + (c // 2)
                idx, val = self.nu_i[i_c]
                y1, y2 = np.divmod(idx, N)
                kids, vals = [], []
                for a in (0, 1):
                    for b in (0, 1):
                        yf = (2 * y1 + a) * Nf + (2 * y2 + b)
                        share = nu_f.reshape(-1)[yf] / nu_c[idx]
                        kids.append(yf)
                        vals.append(val * share * (fine.m[i_f] / self.m[i_c]))
                yf = np.concatenate(kids)
                v = np.concatenate(vals)
                order = np.argsort(yf)
                keep = v[order] > 0
                fine.nu_i.append((yf[order][keep], v[order][keep]))
        alpha_f = upsample_bilinear(alpha_c).reshape(-1)
        for which in ("A", "B"):
            for J, basic in enumerate(fine.parts[which]):
                xpix = np.concatenate([fine.cells[i] for i in basic])
                fine.alpha[which][J] = alpha_f[xpix].copy()
        return fine

    def transport_cost(self, which: Optional[str] = None) -> float:
        """<c, pi> of the composite plans."""
        E = 0.0
        for xpix, ysup, plan in self.cell_plans(which):
            d = self.coords[xpix][:, None, :] - self.coords[ysup][None, :, :]
            E += float((((d ** 2).sum(axis=2)) * plan).sum())
        return E

    def dense_plan_from_state(self) -> np.ndarray:
        """For s == 1 only: the plan sum_i delta_{x_i} (x) nu_i as an (N^2, N^2) array."""
        assert self.s == 1
        P = np.zeros((self.N * self.N, self.N * self.N))
        for i, (idx, val) in enumerate(self.nu_i):
            P[self.cells[i][0], idx] = val
        return P

    # -- flow update ------------------------------------------------------------
    def glued_gamma(self, i: int, j: int, eps_gamma: float) -> np.ndarray:
        """gamma_ij of a gluing edge candidate (Def. "Gluing edge candidate", Remark "eps-gamma"):
        the entropic optimal transport plan between mu_i/m_i and mu_j/m_j for the cost
        |x - x'|^2 at regularisation eps_gamma, by the oracle's dense Sinkhorn to 1e-14.
        Rows: the pixels of X_i, columns: those of X_j (both in row-major block order)."""
        xi, xj = self.cells[i], self.cells[j]
        mi = self.mu[xi] / self.m[i]
        mj = self.mu[xj] / self.m[j]
        a, b, _, _, _ = sinkhorn_cells(np.array([0, len(xi)]), self.coords[xi], mi,
                                       np.array([0, len(xj)]), self.coords[xj], mj, mj, eps_gamma,
                                       tol=1e-14, max_iter=200000)
        return cell_plan(self.coords[xi], mi, a, self.coords[xj], mj, b, eps_gamma)

    def basic_plans(self, which: Optional[str] = None):
        """pi_i for every basic cell: the rows of X_i of the composite plan of the last
        iteration, as (ysup, rows [|X_i|, |ysup|]) with rows in the block order of X_i."""
        which = which or self.last_which
        eps = self.last_eps[which]
        out = [None] * len(self.cells)
        for cs in self.last[which]:
            plan = cell_plan(self.coords[cs.xpix], self.mu[cs.xpix], cs.alpha,
                             self.coords[cs.ysup], self.nu[cs.ysup], cs.beta, eps)
            row = 0
            for k, i in enumerate(cs.basic):
                out[i] = (cs.ysup, plan[row:row + cs.xcount[k]])
                row += cs.xcount[k]
        return out

    def glued_candidate(self, i: int, j: int, eps_gamma: float, plans=None):
        """The gluing edge candidate pihat_ij (eq. glued-plan) on X_j x supp(pi_i), densely:
            pihat_ij(x', y) = (1/m_i) sum_{x in X_i} (gamma_ij)_x(x') pi_i(x, y),
        with (gamma_ij)_x = gamma_ij(x, .) / sum_x' gamma_ij(x, x') the disintegration of gamma_ij
        at x, and mu_i(x) (pi_i)_x read as the plan's own row pi_i(x, .) (so the candidate's
        Y-marginal is exactly the plan's nu_i / m_i).  Returns (ysup, pihat)."""
        plans = plans or self.basic_plans()
        ysup, rows = plans[i]
        g = self.glued_gamma(i, j, eps_gamma)
        cond = g / g.sum(axis=1, keepdims=True)
        return ysup, cond.T @ rows / self.m[i]

    def flow_update(self, mass_bits: int = 40, cost_bits: int = 30, truncate: bool = True,
                    eps_gamma: Optional[float] = None) -> dict:
        """Flow update with gluing edge candidates (Def. "Flow update", Def. "Gluing edge
        candidate", Remark "eps-gamma").  eps_gamma None: the product candidates; else the
        candidates glued from entropic plans gamma_ij at regularisation eps_gamma, with
            cbar_ij = <c, pihat_ij> - <c, pi_i>/m_i
        summed by brute force over X_j x supp(pi_i) (glued_candidate).

        pi_i is the restriction to X_i x Y of the composite plan of the immediately
        preceding DD iteration (instantiated from its potentials).  For every arc (i, j)
        of the 4-neighbourhood plus self loops,
            cbar_ij = <c, mu_j/m_j (x) nu_i/m_i> - <c, pi_i>/m_i   (i != j),  cbar_ii = 0,
        summed by brute force over X_j x supp(nu_i) and X_i x supp(pi_i).
        The min-cost flow is solved on integers: masses b_i by largest remainder with
        sum 2^mass_bits, costs round(cbar * 2^cost_bits / max|cbar|); the flow is mapped
        back as w_ij = flow_ij * m_i / b_i.  New marginals nu_hat_j = sum_i w_ij nu_i / m_i
        (eq. flow-update-cell-marginals), then truncated at 1e-15.
        """
        which = self.last_which
        eps = self.last_eps[which]
        n, N = self.n, self.N
        # instantiate pi_i from the last composite solve
        ctotal = np.zeros(len(self.cells))
        for cs in self.last[which]:
            plan = cell_plan(self.coords[cs.xpix], self.mu[cs.xpix], cs.alpha,
                             self.coords[cs.ysup], self.nu[cs.ysup], cs.beta, eps)
            d = self.coords[cs.xpix][:, None, :] - self.coords[cs.ysup][None, :, :]
            cp = ((d ** 2).sum(axis=2)) * plan
            row = 0
            for k, i in enumerate(cs.basic):
                ctotal[i] = float(cp[row:row + cs.xcount[k]].sum())
                row += cs.xcount[k]
        tail, head = neighbourhood(n)
        cbar = np.zeros(len(tail))
        plans = self.basic_plans(which) if eps_gamma is not None else None
        for a in range(len(tail)):
            i, j = int(tail[a]), int(head[a])
            if i == j:
                continue
            if eps_gamma is not None:
                ysup, ph = self.glued_candidate(i, j, eps_gamma, plans)
                d = self.coords[self.cells[j]][:, None, :] - self.coords[ysup][None, :, :]
                cbar[a] = float(((d ** 2).sum(axis=2) * ph).sum()) - ctotal[i] / self.m[i]
                continue
            idx, val = self.nu_i[i]
            xj = self.coords[self.cells[j]]
            d = xj[:, None, :] - self.coords[idx][None, :, :]
            c = (d ** 2).sum(axis=2)
            w = (self.mu[self.cells[j]] / self.m[j])[:, None] * (val / self.m[i])[None, :]
            cbar[a] = float((c * w).sum()) - ctotal[i] / self.m[i]
        res = self.solve_flow(tail, head, cbar, mass_bits, cost_bits)
        self.apply_flow(tail, head, res["w"], truncate=truncate)
        res["cbar"] = cbar
        return res

    def solve_flow(self, tail, head, cbar, mass_bits=40, cost_bits=30) -> dict:
        nI = len(self.cells)
        b = largest_remainder(self.m, 1 << mass_bits)
        cmax = float(np.abs(cbar).max()) if len(cbar) else 0.0
        scale = (float(1 << cost_bits) / cmax) if cmax > 0 else 0.0
        icost = np.rint(cbar * scale).astype(np.int64)
        flow, pot, st = mcf_ssp(nI, tail, head, icost, b, b)
        if st != 0:
            raise RuntimeError("min-cost flow failed")
        w = flow.astype(np.float64) * (self.m[tail] / b[tail].astype(np.float64))
        int_value = sum(int(f) * int(c) for f, c in zip(flow, icost))  # exact (can exceed int64)
        return {"w": w, "flow": flow, "icost": icost, "b": b, "pot": pot,
                "int_value": int_value, "value": float((w * cbar).sum())}

    def apply_flow(self, tail, head, w, truncate: bool = True) -> None:
        """nu_hat_j = sum_{i in N(j)} w_ij nu_i / m_i (eq. flow-update-cell-marginals)."""
        parts: List[List[Tuple[np.ndarray, np.ndarray]]] = [[] for _ in self.cells]
        for a in range(len(tail)):
            i, j = int(tail[a]), int(head[a])
            if w[a] == 0.0:
                continue
            idx, val = self.nu_i[i]
            parts[j].append((idx, (w[a] / self.m[i]) * val))
        new = []
        for j in range(len(self.cells)):
            idx, val = sparse_sum(parts[j])
            if truncate:
                keep = val >= self.trunc
                idx, val = idx[keep], val[keep]
            new.append((idx, val))
        self.nu_i = new


# ---------------------------------------------------------------------------
# Global problems (tiny grids)
# ---------------------------------------------------------------------------

def kmeans_boxes(dims: np.ndarray, k: int) -> List[List[int]]:
    """K-means clustering of bounding-box dimensions (App. A.1 "Batching and clustering";
    App. A.2.1, Fig. "clustering": K-means on the width and height of the composite cells'
    Y-marginal boxes).  Lloyd's algorithm: assign every box to its nearest centre in the
    (W1, W2) plane (ties to the lower centre index), move every centre to the mean of its
    boxes, until no assignment changes.  Reading (the paper does not state an
    initialisation): the k starting centres are the boxes at ranks floor((q + 1/2) n / k),
    q = 0..k-1, of the order by area W1 W2 (stable).  Returns the non-empty clusters as
    ascending cell lists, by decreasing centre area."""
    dims = np.asarray(dims, dtype=np.float64).reshape(-1, 2)
    n = len(dims)
    k = max(1, min(int(k), n))
    area = dims[:, 0] * dims[:, 1]
    order = sorted(range(n), key=lambda i: area[i])
    cent = np.array([dims[order[min(n - 1, int((q + 0.5) * n / k))]] for q in range(k)])
    lab = [-1] * n
    for _ in range(100):
        changed = False
        for i in range(n):
            d = [(dims[i, 0] - cent[q, 0]) ** 2 + (dims[i, 1] - cent[q, 1]) ** 2 for q in range(k)]
            best = min(range(k), key=lambda q: (d[q], q))
            changed |= lab[i] != best
            lab[i] = best
        if not changed:
            break
        for q in range(k):
            mem = [i for i in range(n) if lab[i] == q]
            if mem:
                cent[q] = dims[mem].mean(axis=0)
    groups = [[i for i in range(n) if lab[i] == q] for q in range(k)]
    qs = sorted(range(k), key=lambda q: -cent[q, 0] * cent[q, 1])
    return [groups[q] for q in qs if groups[q]]


def upsample_bilinear(a: np.ndarray) -> np.ndarray:
    """Values of a function known at the pixel centres of an N x N grid, at the pixel centres of
    the 2N x 2N grid: bilinear interpolation between the four nearest coarse centres, linear
    extrapolation beyond the outermost ones.  Fine pixel k lies at coarse index (k - 1/2) / 2."""
    N = a.shape[0]
    u = (np.arange(2 * N) - 0.5) / 2.0
    k0 = np.clip(np.floor(u).astype(np.int64), 0, N - 2)
    t = u - k0
    rows = (1 - t)[:, None] * a[k0, :] + t[:, None] * a[k0 + 1, :]
    return (1 - t)[None, :] * rows[:, k0] + t[None, :] * rows[:, k0 + 1]


def coarsen(a: np.ndarray) -> np.ndarray:
    """The next coarser layer of a measure on an N x N grid: sums over 2 x 2 pixel blocks."""
    N = a.shape[0]
    return a.reshape(N // 2, 2, N // 2, 2).sum(axis=(1, 3))


def global_sinkhorn(mu: np.ndarray, nu: np.ndarray, eps: float, tol: float = 1e-13,
                    max_iter: int = 200000):
    """Entropic OT on the whole grid with the oracle's cell solver (one cell = X, Y = supp nu).

    Returns (alpha, beta) on all pixels (beta = nan off the support), and the dense plan."""
    N = mu.shape[0]
    C = pixel_coords(N)
    m = mu.reshape(-1)
    v = nu.reshape(-1)
    ys = np.nonzero(v > 0)[0]
    a, b, it, err, nit = sinkhorn_cells(np.array([0, N * N]), C, m, np.array([0, len(ys)]), C[ys],
                                        v[ys], v[ys], eps, tol=tol, max_iter=max_iter, rule=0)
    plan = np.zeros((N * N, N * N))
    plan[:, ys] = cell_plan(C, m, a, C[ys], v[ys], b, eps)
    beta = np.full(N * N, np.nan)
    beta[ys] = b
    return a, beta, plan, nit


def dual_value(mu: np.ndarray, nu: np.ndarray, alpha: np.ndarray, beta: np.ndarray, eps: float) -> float:
    """D(alpha, beta) = <alpha, mu> + <beta, nu> + eps <1 - exp((alpha+beta-c)/eps), mu (x) nu>."""
    N = mu.shape[0]
    C = pixel_coords(N)
    m, v = mu.reshape(-1), nu.reshape(-1)
    sup = v > 0
    b = np.where(sup, beta, 0.0)
    c = ((C[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    K = np.exp((alpha[:, None] + b[None, :] - c) / eps) * (m[:, None] * v[None, :])
    K[:, ~sup] = 0.0
    return float((alpha * m).sum() + (b * v).sum() + eps * (m.sum() * v.sum() - K.sum()))


def primal_dense(mu: np.ndarray, nu: np.ndarray, plan: np.ndarray, eps: float) -> float:
    """E(pi) for a dense (N^2, N^2) plan, straight from eq. (KL) and eq. (entropic-transport)."""
    N = mu.shape[0]
    C = pixel_coords(N)
    m, v = mu.reshape(-1), nu.reshape(-1)
    c = ((C[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    ref = m[:, None] * v[None, :]
    pos = plan > 0
    kl = float((plan[pos] * np.log(plan[pos] / ref[pos]) - plan[pos]).sum()) + float(ref.sum())
    return float((c * plan).sum()) + eps * kl
