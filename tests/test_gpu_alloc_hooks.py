"""dd_params.dev_alloc / dev_free: a context whose device memory comes from PyTorch's caching
allocator gives the same results as one on the library's own hipMalloc, every block it takes
goes back when the context is freed, and a supplier that runs dry fails the call with
DD_ENOMEM without leaking what it had already handed out.
"""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(allocator):
    """Multiscale float64 DD at fixed counts: two half-iterations on the 32^2 layer, refine,
    two on 64^2, a flow update with glued candidates, one more half-iteration; returns the
    basic-cell Y-marginals, the evaluation and the flow statistics."""
    import paper_2405_09400_amd as dd
    w = synth.workload("mix256", N=64)
    g = dd.DomDec(w.mu, w.nu, 4, w.init, prec=dd.DD_PREC_F64, levels=1, allocator=allocator)
    for layer in range(2):
        eps = 2.0 / g.N ** 2
        g.iterate("A", eps, fixed_iters=30)
        g.iterate("B", eps, fixed_iters=30)
        if layer == 0:
            g.refine()
    eps = 1.0 / g.N ** 2
    fs = g.flow_update(eps_gamma=eps)
    g.iterate("A", eps, fixed_iters=30)
    ev = g.evaluate()
    nu_i = g.nu_i_sparse()
    return g, nu_i, ev, fs


def test_torch_allocator_matches_hipmalloc_and_returns_every_block():
    import paper_2405_09400_amd as dd
    _need_gpu()
    print("alloc hooks: multiscale f64 N=64 s=4, hipMalloc vs torch caching allocator", flush=True)
    g0, nu0, ev0, fs0 = _run(None)
    g0.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    alloc = dd.TorchAllocator(torch.cuda.current_stream())
    g1, nu1, ev1, fs1 = _run(alloc)
    torch.cuda.synchronize()
    assert alloc.calls > 0 and alloc.live > 0
    # the context's blocks are PyTorch's: its allocated-bytes counter holds them
    assert torch.cuda.memory_allocated() - before >= alloc.live_bytes
    for (i0, v0), (i1, v1) in zip(nu0, nu1):
        assert np.array_equal(i0, i1)
        assert np.abs(v0 - v1).max(initial=0.0) <= 1e-14
    for k in ("primal", "x_marginal_l1", "y_marginal_l1", "dual"):
        assert abs(ev0[k] - ev1[k]) <= 1e-13 * max(1.0, abs(ev0[k])), k
    assert fs0["int_value"] == fs1["int_value"]
    g1.close()
    torch.cuda.synchronize()
    assert alloc.live == 0 and alloc.live_bytes == 0
    assert torch.cuda.memory_allocated() == before


class _Limited:
    """Hooks over PyTorch's allocator that return NULL from the k-th request on."""

    def __init__(self, k):
        import paper_2405_09400_amd as dd
        self.inner = dd.TorchAllocator(torch.cuda.current_stream())
        self.k = k
        self.n = 0
        self.alloc_fn = dd.binding.ALLOC_FN(self._alloc)
        self.free_fn = self.inner.free_fn

    def _alloc(self, nbytes, ud):
        self.n += 1
        if self.n >= self.k:
            return None
        return self.inner._alloc(nbytes, ud)


@pytest.mark.parametrize("k", [1, 7, 20])
def test_supplier_out_of_memory_fails_init_without_leaks(k):
    import paper_2405_09400_amd as dd
    _need_gpu()
    print(f"alloc hooks: supplier fails from request {k}", flush=True)
    w = synth.workload("mix256", N=32)
    lim = _Limited(k)
    with pytest.raises(dd.DomDecError) as e:
        dd.DomDec(w.mu, w.nu, 4, w.init, prec=dd.DD_PREC_F64, allocator=lim)
    assert e.value.status == dd.DD_ENOMEM
    torch.cuda.synchronize()
    assert lim.inner.live == 0


def test_supplier_out_of_memory_in_iterate_then_close():
    import paper_2405_09400_amd as dd
    _need_gpu()
    print("alloc hooks: supplier runs dry after init", flush=True)
    w = synth.workload("mix256", N=32)
    lim = _Limited(10 ** 9)
    g = dd.DomDec(w.mu, w.nu, 4, w.init, prec=dd.DD_PREC_F64, allocator=lim)
    lim.k = lim.n + 1  # every later request fails
    with pytest.raises(dd.DomDecError) as e:
        g.iterate("A", 1.0 / 32 ** 2, fixed_iters=10)
    assert e.value.status == dd.DD_ENOMEM
    g.close()
    torch.cuda.synchronize()
    assert lim.inner.live == 0


def test_one_hook_without_the_other_is_rejected():
    import paper_2405_09400_amd as dd
    _need_gpu()
    w = synth.workload("mix256", N=32)
    alloc = dd.TorchAllocator(torch.cuda.current_stream())
    p = dd.binding.Params(32, 4, 1e-15, dd.DD_PREC_F64, 0)
    p.dev_alloc = alloc.alloc_fn
    dp = ctypes.POINTER(ctypes.c_double)
    mu = np.ascontiguousarray(w.mu.reshape(-1))
    nu = np.ascontiguousarray(w.nu.reshape(-1))
    ctx = ctypes.c_void_p()
    st = dd.lib().domdec_init(ctypes.byref(p), mu.ctypes.data_as(dp), nu.ctypes.data_as(dp), 0,
                              None, None, None, None, ctypes.byref(ctx))
    assert st == dd.DD_EINVAL and not ctx.value
    assert alloc.calls == 0
