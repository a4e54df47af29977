"""ctypes binding of libdomdec.so (include/domdec.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libdomdec.so")
_LIB = None

DD_OK, DD_NOTCONV, DD_EINVAL, DD_ENOMEM, DD_EDEVICE, DD_ESTATE, DD_ENUMERIC = 0, 1, -1, -2, -3, -4, -5
DD_PREC_F32, DD_PREC_F64 = 0, 1
DD_STOP_BATCH, DD_STOP_CELL = 0, 1
DD_INIT_ZERO, DD_INIT_PREV, DD_INIT_NET = 0, 1, 2
DD_PART_A, DD_PART_B = 0, 1
DD_CAND_PRODUCT, DD_CAND_GLUED = 0, 1

_NAMES = {0: "DD_OK", 1: "DD_NOTCONV", -1: "DD_EINVAL", -2: "DD_ENOMEM", -3: "DD_EDEVICE",
          -4: "DD_ESTATE", -5: "DD_ENUMERIC"}

# every function include/domdec.h declares
SYMBOLS = ("sinkhorn_batch", "sinkhorn_batch_f64", "domdec_init", "domdec_iterate", "flow_update",
           "flow_costs", "flow_apply", "dd_mcf_solve", "extract_plan", "domdec_evaluate", "domdec_free",
           "domdec_strerror", "dd_net_param_count", "dd_net_create", "dd_net_params", "dd_net_forward", "dd_net_infer",
           "dd_net_train_step", "dd_net_free", "dd_net_strerror", "domdec_set_net", "domdec_net_samples", "domdec_save", "domdec_restore",
           "extract_potentials", "sinkhorn_batch_noalloc", "domdec_refine", "global_sinkhorn",
           "domdec_set_clusters", "sinkhorn_set_classes")


class DomDecError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class SinkhornOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("check_every", ctypes.c_int32), ("init", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("ncells", ctypes.c_int32), ("iters_max", ctypes.c_int32), ("iters_min", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("cell_iters", ctypes.c_int64), ("err", ctypes.c_double),
                ("mass", ctypes.c_double), ("lse_terms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("main_ms", ctypes.c_double),
                ("finish_iters_max", ctypes.c_int32), ("n_big", ctypes.c_int32),
                ("n_giant", ctypes.c_int32), ("lds_kb", ctypes.c_int32 * 2),
                ("tile_small", ctypes.c_int32 * 2), ("tile_big", ctypes.c_int32 * 2),
                ("path", ctypes.c_int32), ("kernel_launches", ctypes.c_int32 * 3),
                ("wave_side", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double * 3), ("kernel_terms", ctypes.c_double * 3),
                ("big_entries", ctypes.c_int32), ("reserved4", ctypes.c_int32)]


# dd_params.dev_alloc / dev_free
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("s", ctypes.c_int32), ("trunc", ctypes.c_double),
                ("prec", ctypes.c_int32), ("levels", ctypes.c_int32), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_ud", ctypes.c_void_p)]


class TorchAllocator:
    """dd_params hooks that take the context's device memory from PyTorch's caching allocator
    on the context's stream (torch.cuda.caching_allocator_alloc / _delete).  `live` counts the
    blocks the library holds, `peak_bytes` the most it held at once."""

    def __init__(self, stream, device=None):
        import torch
        self._torch = torch
        self._stream = stream
        self._device = torch.cuda.current_device() if device is None else device
        self._sizes = {}
        self.live_bytes = 0
        self.peak_bytes = 0
        self.calls = 0
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    @property
    def live(self) -> int:
        return len(self._sizes)

    def _alloc(self, nbytes, _ud):
        try:
            p = int(self._torch.cuda.caching_allocator_alloc(int(nbytes), self._device,
                                                             self._stream))
        except Exception:  # out of memory (or any failure): NULL -> DD_ENOMEM
            return None
        self._sizes[p] = int(nbytes)
        self.live_bytes += int(nbytes)
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        self.calls += 1
        return p

    def _free(self, ptr, _ud):
        if not ptr:
            return
        self.live_bytes -= self._sizes.pop(int(ptr), 0)
        self._torch.cuda.caching_allocator_delete(int(ptr))


class IterStats(ctypes.Structure):
    _fields_ = [("sk", BatchStats), ("partition", ctypes.c_int32), ("max_w1", ctypes.c_int32),
                ("max_w2", ctypes.c_int32), ("grid_n", ctypes.c_int32), ("nu_entries", ctypes.c_int64),
                ("comp_entries", ctypes.c_int64), ("t_b2c_ms", ctypes.c_double),
                ("t_sinkhorn_ms", ctypes.c_double), ("t_c2b_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("t_init_ms", ctypes.c_double),
                ("batches", ctypes.c_int32), ("host_waits", ctypes.c_int32),
                ("peak_comp_entries", ctypes.c_int64), ("spec_resumed", ctypes.c_int32),
                ("reserved4", ctypes.c_int32)]


class FlowStats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_arcs", ctypes.c_int32), ("int_value", ctypes.c_double),
                ("value", ctypes.c_double), ("moved_mass", ctypes.c_double),
                ("n_active_arcs", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_costs_ms", ctypes.c_double), ("t_mcf_ms", ctypes.c_double),
                ("t_assemble_ms", ctypes.c_double)]


class PlanView(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_entries", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int32)), ("dims", ctypes.POINTER(ctypes.c_int32)),
                ("base", ctypes.POINTER(ctypes.c_int64)), ("data", ctypes.POINTER(ctypes.c_double))]


class PotentialsView(ctypes.Structure):
    _fields_ = [("partition", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("xside", ctypes.c_int32),
                ("has_beta", ctypes.c_int32), ("eps", ctypes.c_double), ("n_y", ctypes.c_int64),
                ("xorig", ctypes.POINTER(ctypes.c_int32)), ("alpha", ctypes.POINTER(ctypes.c_double)),
                ("yorig", ctypes.POINTER(ctypes.c_int32)), ("ydims", ctypes.POINTER(ctypes.c_int32)),
                ("ybase", ctypes.POINTER(ctypes.c_int64)), ("beta", ctypes.POINTER(ctypes.c_double))]


class GlobalStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("err", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("lse_terms", ctypes.c_double)]


class Eval(ctypes.Structure):
    _fields_ = [("y_marginal_l1", ctypes.c_double), ("x_marginal_l1", ctypes.c_double),
                ("primal", ctypes.c_double), ("transport", ctypes.c_double),
                ("basic_mass_err", ctypes.c_double), ("total_mass", ctypes.c_double),
                ("dual", ctypes.c_double), ("pd_gap", ctypes.c_double)]


def _struct_dict(s) -> dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        if isinstance(v, ctypes.Structure):
            v = _struct_dict(v)
        elif isinstance(v, ctypes.Array):
            v = list(v)
        out[name] = v
    return out


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libdomdec.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_2405_09400_amd.build` "
                           "(the HIP library is required; there is no CPU path)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32p, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("sinkhorn_batch", "sinkhorn_batch_f64", "sinkhorn_batch_noalloc"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                      ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(SinkhornOpts), vp, vp, vp,
                      ctypes.POINTER(BatchStats)]
    L.domdec_init.restype = ctypes.c_int
    L.domdec_init.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_int64, i64p, i64p, dp, vp,
                              ctypes.POINTER(vp)]
    L.sinkhorn_set_classes.restype = ctypes.c_int
    L.sinkhorn_set_classes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.domdec_set_clusters.restype = ctypes.c_int
    L.domdec_set_clusters.argtypes = [vp, ctypes.c_int32]
    L.domdec_iterate.restype = ctypes.c_int
    L.domdec_iterate.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(SinkhornOpts),
                                 ctypes.POINTER(IterStats)]
    L.flow_update.restype = ctypes.c_int
    L.flow_update.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(FlowStats)]
    L.flow_costs.restype = ctypes.c_int
    L.flow_costs.argtypes = [vp, ctypes.c_int32, ctypes.c_double, dp, i32p]
    L.flow_apply.restype = ctypes.c_int
    L.flow_apply.argtypes = [vp, dp]
    L.dd_mcf_solve.restype = ctypes.c_int
    L.dd_mcf_solve.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p, i64p, i64p, i64p, i64p]
    L.extract_plan.restype = ctypes.c_int
    L.extract_plan.argtypes = [vp, ctypes.POINTER(PlanView)]
    L.global_sinkhorn.restype = ctypes.c_int
    L.global_sinkhorn.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_double, vp, vp,
                                  ctypes.POINTER(SinkhornOpts), vp, ctypes.POINTER(GlobalStats)]
    L.extract_potentials.restype = ctypes.c_int
    L.extract_potentials.argtypes = [vp, ctypes.POINTER(PotentialsView)]
    L.domdec_evaluate.restype = ctypes.c_int
    L.domdec_evaluate.argtypes = [vp, ctypes.POINTER(Eval)]
    L.domdec_free.restype = None
    L.domdec_free.argtypes = [vp]
    L.domdec_strerror.restype = ctypes.c_char_p
    L.domdec_strerror.argtypes = [vp, ctypes.c_int]
    L.dd_net_param_count.restype = ctypes.c_int64
    L.dd_net_param_count.argtypes = []
    fp = ctypes.POINTER(ctypes.c_float)
    L.dd_net_create.restype = ctypes.c_int
    L.dd_net_create.argtypes = [fp, ctypes.POINTER(vp)]
    L.dd_net_params.restype = ctypes.c_int
    L.dd_net_params.argtypes = [vp, fp]
    L.dd_net_forward.restype = ctypes.c_int
    L.dd_net_forward.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    L.dd_net_infer.restype = ctypes.c_int
    L.dd_net_infer.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    L.dd_net_train_step.restype = ctypes.c_int
    L.dd_net_train_step.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_float, vp, dp]
    L.dd_net_free.restype = None
    L.dd_net_free.argtypes = [vp]
    L.dd_net_strerror.restype = ctypes.c_char_p
    L.dd_net_strerror.argtypes = [vp]
    L.domdec_set_net.restype = ctypes.c_int
    L.domdec_set_net.argtypes = [vp, vp]
    for name in ("domdec_save", "domdec_restore", "domdec_refine"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [vp]
    L.domdec_net_samples.restype = ctypes.c_int
    L.domdec_net_samples.argtypes = [vp, vp, vp, vp, ctypes.c_int32, i32p]
    _LIB = L
    return L


def mcf_solve(n, tail, head, cost, supply):
    """Integer bipartite min-cost flow (dd_mcf_solve, host only).  Returns (flow, potentials)."""
    tail = np.ascontiguousarray(tail, dtype=np.int32)
    head = np.ascontiguousarray(head, dtype=np.int32)
    cost = np.ascontiguousarray(cost, dtype=np.int64)
    supply = np.ascontiguousarray(supply, dtype=np.int64)
    flow = np.zeros(len(tail), dtype=np.int64)
    pot = np.zeros(2 * n, dtype=np.int64)
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    st = lib().dd_mcf_solve(int(n), len(tail), tail.ctypes.data_as(i32p), head.ctypes.data_as(i32p),
                            cost.ctypes.data_as(i64p), supply.ctypes.data_as(i64p),
                            flow.ctypes.data_as(i64p), pot.ctypes.data_as(i64p))
    _check(st)
    return flow, pot


def exported_symbols():
    """Names from include/domdec.h that the loaded library exports."""
    L = lib()
    return [n for n in SYMBOLS if hasattr(L, n)]


def _check(st: int, ctx=None, warn_ok=True):
    if st == DD_OK or (warn_ok and st == DD_NOTCONV):
        return st
    msg = lib().domdec_strerror(ctx, st)
    raise DomDecError(st, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _opts(tol, max_iter, fixed_iters, stop_rule, check_every, init=DD_INIT_PREV) -> SinkhornOpts:
    return SinkhornOpts(float(tol), int(max_iter), int(fixed_iters), int(stop_rule), int(check_every),
                        int(init), 0)


def _candidate(eps_gamma):
    return (DD_CAND_PRODUCT, 0.0) if eps_gamma is None else (DD_CAND_GLUED, float(eps_gamma))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def sinkhorn_batch(dims, base, shift, logmu, lognu, a, b, kappa, max_w1, max_w2, *, prec=DD_PREC_F32,
                   tol=1e-5, max_iter=10000, fixed_iters=0, stop_rule=DD_STOP_BATCH, check_every=8,
                   cell_iters=None, cell_err=None, stream=None, raise_on_error=True, noalloc=False):
    """Batched cell Sinkhorn on device tensors (see sinkhorn_batch in include/domdec.h;
    noalloc=True calls sinkhorn_batch_noalloc, float32 only).

    dims int32 [n,2], base int64 [n], shift int32 [n,2], float64 logmu [n, xside^2], lognu packed,
    a [n, xside^2] (f, in/out), b packed (g, out).  prec DD_PREC_F32 -> sinkhorn_batch
    (float32 log-sum-exp terms), DD_PREC_F64 -> sinkhorn_batch_f64.  Returns (status, stats)."""
    import torch
    n = int(dims.shape[0])
    xside = int(round(logmu.shape[1] ** 0.5)) if n else 2
    for t, dt in ((dims, torch.int32), (base, torch.int64), (shift, torch.int32)):
        assert t.dtype == dt and t.is_cuda and t.is_contiguous()
    for t in (logmu, lognu, a, b):
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    # host-side shape checks: the kernels trust base/dims to stay inside the packed buffers
    if n:
        hd = dims.cpu().numpy().astype(np.int64)
        hb = base.cpu().numpy()
        if logmu.dim() != 2 or logmu.shape[1] != xside * xside or tuple(a.shape) != tuple(logmu.shape) \
                or logmu.shape[0] != n or tuple(shift.shape) != (n, 2) or tuple(dims.shape) != (n, 2):
            raise ValueError("sinkhorn_batch: logmu/a must be [n, xside^2], dims/shift [n, 2]")
        if np.any(hd < 1) or np.any(hb < 0) or np.any(hb + hd[:, 0] * hd[:, 1] > lognu.numel()) \
                or b.numel() != lognu.numel():
            raise ValueError("sinkhorn_batch: a Y box lies outside lognu/b")
    if noalloc and prec != DD_PREC_F32:
        raise ValueError("sinkhorn_batch_noalloc is the float32 entry point")
    f = lib().sinkhorn_batch_noalloc if noalloc else (
        lib().sinkhorn_batch if prec == DD_PREC_F32 else lib().sinkhorn_batch_f64)
    st = BatchStats()
    o = _opts(tol, max_iter, fixed_iters, stop_rule, check_every)
    status = f(n, xside, _ptr(dims), _ptr(base), _ptr(shift), _ptr(logmu), _ptr(lognu), _ptr(a), _ptr(b),
               float(kappa), int(max_w1), int(max_w2), ctypes.byref(o), _ptr(cell_iters), _ptr(cell_err),
               _stream_ptr(stream), ctypes.byref(st))
    if raise_on_error:
        _check(status)
    return status, _struct_dict(st)


def global_sinkhorn(mu, nu, eps, alpha, beta, *, tol=1e-5, max_iter=100000, fixed_iters=0,
                    stream=None, raise_on_error=True):
    """Global Sinkhorn on the whole grid (global_sinkhorn in include/domdec.h): mu, nu float64
    [N, N] device tensors, alpha (in/out) and beta (out) float64 [N, N].  Returns (status, stats)."""
    import torch
    N = int(mu.shape[0])
    for t in (mu, nu, alpha, beta):
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and tuple(t.shape) == (N, N)
    st = GlobalStats()
    o = _opts(tol, max_iter, fixed_iters, DD_STOP_BATCH, 0)
    status = lib().global_sinkhorn(N, _ptr(mu), _ptr(nu), float(eps), _ptr(alpha), _ptr(beta),
                                   ctypes.byref(o), _stream_ptr(stream), ctypes.byref(st))
    if raise_on_error:
        _check(status)
    return status, _struct_dict(st)


def set_classes(wave_side: int = 0, big_entries: int = 0) -> None:
    """Cell classes of the register-blocked path (sinkhorn_set_classes): boxes with long side
    <= wave_side one wave, more than big_entries entries eight waves, the rest four; (0, 0)
    hands the choice back to the library's tuner."""
    st = lib().sinkhorn_set_classes(int(wave_side), int(big_entries))
    if st != DD_OK:
        raise DomDecError(st, lib().domdec_strerror(None, st).decode())


class DomDec:
    """A device-resident domain-decomposition state (dd_ctx) on the current HIP device."""

    def __init__(self, mu: np.ndarray, nu: np.ndarray, s: int, init=None, trunc: float = 1e-15,
                 prec: int = DD_PREC_F32, stream=None, levels: int = 0, allocator=None):
        """levels > 0: multiscale; the context starts on the (N / 2^levels)^2 layer and refine()
        moves to the next finer one (self.N is the grid side of the current layer).
        allocator: None (the library's hipMalloc), "torch" (PyTorch's caching allocator on the
        context's stream) or an object with alloc_fn / free_fn hooks (TorchAllocator's shape)."""
        import torch
        self.N = int(mu.shape[0]) >> int(levels)
        self.levels = int(levels)
        self.s = int(s)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        mu64 = np.ascontiguousarray(mu.reshape(-1), dtype=np.float64)
        nu64 = np.ascontiguousarray(nu.reshape(-1), dtype=np.float64)
        p = Params(int(mu.shape[0]), self.s, float(trunc), int(prec), int(levels))
        if allocator == "torch":
            allocator = TorchAllocator(self._stream)
        self.allocator = allocator  # keeps the hooks alive as long as the context
        if allocator is not None:
            p.dev_alloc = allocator.alloc_fn
            p.dev_free = allocator.free_fn
        ctx = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        if init is None:
            n_init, xp, yp, mp = 0, None, None, None
        else:
            x, y, m = init
            self._ix = np.ascontiguousarray(x, dtype=np.int64)
            self._iy = np.ascontiguousarray(y, dtype=np.int64)
            self._im = np.ascontiguousarray(m, dtype=np.float64)
            n_init = len(self._ix)
            xp, yp, mp = (self._ix.ctypes.data_as(i64p), self._iy.ctypes.data_as(i64p),
                          self._im.ctypes.data_as(dp))
        st = lib().domdec_init(ctypes.byref(p), mu64.ctypes.data_as(dp), nu64.ctypes.data_as(dp), n_init,
                               xp, yp, mp, _stream_ptr(self._stream), ctypes.byref(ctx))
        _check(st, None)
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            lib().domdec_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, partition: str, eps: float, *, tol=1e-5, max_iter=10000, fixed_iters=0,
                stop_rule=DD_STOP_BATCH, check_every=8, init=DD_INIT_PREV) -> dict:
        st = IterStats()
        o = _opts(tol, max_iter, fixed_iters, stop_rule, check_every, init)
        part = {"A": DD_PART_A, "B": DD_PART_B}[partition] if isinstance(partition, str) else int(partition)
        status = lib().domdec_iterate(self._ctx, part, float(eps), ctypes.byref(o), ctypes.byref(st))
        _check(status, self._ctx)
        d = _struct_dict(st)
        d["status"] = status
        return d

    def set_clusters(self, k: int) -> None:
        """Solve each later iteration's composite cells in k bounding-box clusters, one batch
        after another (domdec_set_clusters); k = 1: one batch."""
        _check(lib().domdec_set_clusters(self._ctx, int(k)), self._ctx)

    def refine(self) -> None:
        """Move to the next finer layer of a multiscale context (domdec_refine)."""
        _check(lib().domdec_refine(self._ctx), self._ctx)
        self.N *= 2

    def save(self) -> None:
        """Keep a copy of the mutable state (domdec_save)."""
        _check(lib().domdec_save(self._ctx), self._ctx)

    def restore(self) -> None:
        """Return to the saved state (domdec_restore)."""
        _check(lib().domdec_restore(self._ctx), self._ctx)

    def set_net(self, net: Optional["WarmStartNet"]) -> None:
        """Attach a warm-start net for init=DD_INIT_NET (the object must outlive its use)."""
        self._net = net
        _check(lib().domdec_set_net(self._ctx, net._net if net is not None else None), self._ctx)

    def net_samples(self):
        """(x [n,8,32,32], target [n,32,32], weight [n,32,32]) float32 device tensors of the
        cells of the last iteration (features, target correction of the Y potential, weights)."""
        import torch
        n = ctypes.c_int32(0)
        _check(lib().domdec_net_samples(self._ctx, None, None, None, 0, ctypes.byref(n)), self._ctx)
        k = int(n.value)
        dev = torch.device("cuda", torch.cuda.current_device())
        x = torch.empty((k, 8, 32, 32), dtype=torch.float32, device=dev)
        t = torch.empty((k, 32, 32), dtype=torch.float32, device=dev)
        w = torch.empty((k, 32, 32), dtype=torch.float32, device=dev)
        self._stream.synchronize()
        _check(lib().domdec_net_samples(self._ctx, _ptr(x), _ptr(t), _ptr(w), k, ctypes.byref(n)),
               self._ctx)
        return x, t, w

    def flow_update(self, eps_gamma=None) -> dict:
        """Flow update (flow_update): product candidates, or with eps_gamma the candidates glued
        from entropic plans at that regularisation."""
        st = FlowStats()
        cand, eg = _candidate(eps_gamma)
        _check(lib().flow_update(self._ctx, cand, eg, ctypes.byref(st)), self._ctx)
        return _struct_dict(st)

    def flow_costs(self, eps_gamma=None) -> np.ndarray:
        n = ctypes.c_int32()
        cand, eg = _candidate(eps_gamma)
        _check(lib().flow_costs(self._ctx, cand, eg, None, ctypes.byref(n)), self._ctx)
        out = np.zeros(n.value, dtype=np.float64)
        _check(lib().flow_costs(self._ctx, cand, eg,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None),
               self._ctx)
        return out

    def flow_apply(self, w) -> None:
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(lib().flow_apply(self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._ctx)

    def evaluate(self) -> dict:
        ev = Eval()
        _check(lib().domdec_evaluate(self._ctx, ctypes.byref(ev)), self._ctx)
        return _struct_dict(ev)

    def extract_plan(self):
        """Basic-cell Y-marginals: (offsets [I,2], dims [I,2], base [I+1], data) host arrays."""
        v = PlanView()
        _check(lib().extract_plan(self._ctx, ctypes.byref(v)), self._ctx)
        nI, nE = int(v.n_cells), int(v.n_entries)
        off = np.zeros((nI, 2), np.int32)
        dims = np.zeros((nI, 2), np.int32)
        base = np.zeros(nI + 1, np.int64)
        data = np.zeros(max(nE, 1), np.float64)
        v.offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        v.dims = dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        v.base = base.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        v.data = data.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(lib().extract_plan(self._ctx, ctypes.byref(v)), self._ctx)
        return off, dims, base, data[:nE]

    def extract_potentials(self, partition: str, beta: bool = True) -> dict:
        """Composite-cell potentials of one partition in energy units (extract_potentials):
        dict with eps, xorig [n,2], alpha [n, xside^2] and, when the partition's iteration is the
        last one and `beta`, yorig [n,2], ydims [n,2], ybase [n+1], beta (packed boxes)."""
        v = PotentialsView()
        v.partition = {"A": DD_PART_A, "B": DD_PART_B}[partition] if isinstance(partition, str) \
            else int(partition)
        _check(lib().extract_potentials(self._ctx, ctypes.byref(v)), self._ctx)
        n, xs, ny = int(v.n_cells), int(v.xside), int(v.n_y)
        out = {"eps": float(v.eps), "xside": xs, "has_beta": bool(v.has_beta)}
        xorig = np.zeros((n, 2), np.int32)
        alpha = np.zeros((n, xs * xs), np.float64)
        v.xorig = xorig.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        v.alpha = alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if beta and v.has_beta:
            yorig = np.zeros((n, 2), np.int32)
            ydims = np.zeros((n, 2), np.int32)
            ybase = np.zeros(n + 1, np.int64)
            b = np.zeros(max(ny, 1), np.float64)
            v.yorig = yorig.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            v.ydims = ydims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            v.ybase = ybase.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            v.beta = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            out.update(yorig=yorig, ydims=ydims, ybase=ybase, beta=b[:ny])
        _check(lib().extract_potentials(self._ctx, ctypes.byref(v)), self._ctx)
        out.update(xorig=xorig, alpha=alpha)
        return out

    def nu_i_sparse(self):
        """The stored basic-cell Y-marginals as (flat indices, values) lists (host)."""
        off, dims, base, data = self.extract_plan()
        out = []
        for i in range(len(dims)):
            o1, o2 = off[i]
            w1, w2 = dims[i]
            vals = data[base[i]:base[i + 1]].reshape(w1, w2)
            k1 = (o1 + np.arange(w1))[:, None]
            k2 = (o2 + np.arange(w2))[None, :]
            idx = (k1 * self.N + k2).reshape(-1)
            v = vals.reshape(-1)
            keep = v > 0
            out.append((idx[keep].astype(np.int64), v[keep]))
        return out


def net_param_count() -> int:
    return int(lib().dd_net_param_count())


class WarmStartNet:
    """The learned warm-start conv net (dd_net): BF16 weights, FP32 accumulation, trained with
    Adam by hand-written kernels.  `params` is the flat FP32 parameter vector."""

    def __init__(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if p.size != net_param_count():
            raise ValueError(f"expected {net_param_count()} parameters, got {p.size}")
        h = ctypes.c_void_p()
        st = lib().dd_net_create(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h))
        if st != DD_OK:
            raise DomDecError(st, lib().dd_net_strerror(None).decode())
        self._net = h

    def _check(self, st):
        if st != DD_OK:
            raise DomDecError(st, lib().dd_net_strerror(self._net).decode())

    def params(self) -> np.ndarray:
        out = np.zeros(net_param_count(), np.float32)
        self._check(lib().dd_net_params(self._net, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def forward(self, x, stream=None):
        import torch
        n = int(x.shape[0])
        y = torch.empty((n, 32, 32), dtype=torch.float32, device=x.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        self._check(lib().dd_net_forward(self._net, n, _ptr(x.contiguous()), _ptr(y), _stream_ptr(s)))
        return y

    def infer(self, x, stream=None):
        """The DD start's inference (dd_net_infer): 32-channel layers on the matrix cores."""
        import torch
        n = int(x.shape[0])
        y = torch.empty((n, 32, 32), dtype=torch.float32, device=x.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        self._check(lib().dd_net_infer(self._net, n, _ptr(x.contiguous()), _ptr(y), _stream_ptr(s)))
        return y

    def train_step(self, x, target, weight, lr: float, stream=None) -> float:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        loss = ctypes.c_double(0.0)
        self._check(lib().dd_net_train_step(self._net, int(x.shape[0]), _ptr(x), _ptr(target), _ptr(weight),
                                            float(lr), _stream_ptr(s), ctypes.byref(loss)))
        return float(loss.value)

    def close(self):
        if getattr(self, "_net", None):
            lib().dd_net_free(self._net)
            self._net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def net_init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the dd_net parameter layout (seeded)."""
    rng = np.random.default_rng(seed)
    layers = [(8, 32), (32, 32), (32, 32), (32, 32), (32, 4)]
    out = []
    for l, (cin, cout) in enumerate(layers):
        std = np.sqrt(2.0 / (cin * 9)) if l < len(layers) - 1 else np.sqrt(1.0 / (cin * 9))
        out.append(rng.normal(0.0, std, cout * cin * 9))
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)
