"""MI355X (gfx950) superstep engine for GX-Plug-style graph daemons.

Thin Python binding over the C ABI of ``libgx.so`` (declared in
``include/gx.h``).  This module only marshals arguments: every step of a
superstep runs in the library's HIP kernels.  PyTorch provides the device
memory (arenas are ``torch.uint8`` CUDA tensors) and the streams.  If the
library has not been built the import of the binding fails loudly; there is
no CPU fallback.
"""
from .binding import (  # noqa: F401
    GX_CC,
    GX_OK,
    GX_DELTA_ALL,
    GX_DELTA_MASTERS,
    GX_DELTA_REMOTE,
    GX_LP,
    GX_NEED_IN,
    GX_NEED_OUT,
    GX_NEED_SYM,
    GX_PAGERANK,
    GX_PHASES_LOCAL,
    GX_PHASES_MASTERS,
    GX_PPR,
    GX_SSSP,
    INF,
    DeviceGraph,
    GxError,
    Server,
    CpuPart,
    State,
    balance_split,
    Stream,
    pipeline_plan,
    Tune,
    batch_autotune,
    batch_run,
    exported_symbols,
    lib,
    library_path,
)
