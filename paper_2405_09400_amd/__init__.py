"""MI355X (gfx950) domain decomposition for entropic optimal transport with flow updates.

Thin ctypes binding over the C ABI in include/domdec.h (libdomdec.so, built in-tree by
`paper_2405_09400_amd.build`).  Argument marshalling only: every step of the method runs
in the HIP kernels of the library.  PyTorch supplies device memory and streams.
The binding fails loudly when the library is missing -- there is no CPU fallback.
"""
from .binding import (  # noqa: F401
    DD_OK, DD_NOTCONV, DD_EINVAL, DD_ENOMEM, DD_EDEVICE, DD_ESTATE, DD_ENUMERIC,
    DD_PREC_F32, DD_PREC_F64, DD_STOP_BATCH, DD_STOP_CELL, DD_INIT_ZERO, DD_INIT_PREV, DD_INIT_NET,
    DomDecError, lib, lib_path, exported_symbols, sinkhorn_batch, global_sinkhorn, mcf_solve, DomDec,
    TorchAllocator, set_classes,
    WarmStartNet,
    net_param_count, net_init_params,
)
