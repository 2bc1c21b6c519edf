"""MI355X (gfx950) implementation of the compress/decompress path of LOPC,
the Local-Order-Preserving Compressor (arXiv 2603.26968).

``compress`` / ``decompress`` run entirely in the HIP kernels of
``liblopc.so`` (see ``include/lopc.h``).  The binding is loaded on first use
of any of its names; if the library has not been built
(``python paper_2603_26968_amd/build.py``) that first use raises ImportError.
The ``synth`` submodule (input generators) does not need the library.
"""
import importlib

_BINDING = (
    "LopcError", "compress", "decompress", "context", "lopc_compress_bound",
    "lopc_stream_info", "lopc_workspace_size", "lopc_compress", "lopc_decompress",
    "lopc_ctx_create", "lopc_ctx_destroy", "LOPC_EB_ABS", "LOPC_EB_NOA", "LOPC_F32",
    "LOPC_F64", "Stats", "lopc_ctx_set_timing", "lopc_ctx_last_timings",
    "compress_batch", "decompress_batch", "Job", "BatchStats", "lopc_batch_workspace_size",
    "lopc_compress_batch", "lopc_decompress_batch", "lopc_ctx_last_batch",
    "lopc_ctx_set_option", "lopc_ctx_get_option", "LOPC_OPT_BATCH_GRAPH", "LOPC_OPT_GRAPH_SWEEPS",
    "LOPC_OPT_PERSIST_PCT", "lopc_ctx_last_batch_headers", "lopc_batch_autotune",
    "autotune_compress_batch", "verify", "VerifyReport", "lopc_verify",
    "compress_enqueue", "LOPC_OPT_REPAIR", "LOPC_REPAIR_QUEUE", "LOPC_REPAIR_SWEEPS", "LOPC_REPAIR_HYBRID", "LOPC_REPAIR_AUTO", "LOPC_REPAIR_POINTS", "LOPC_OPT_TILE_3D", "LOPC_OPT_TILE_2D", "LOPC_OPT_SWEEP_ORDER",
)


def __getattr__(name):
    if name in _BINDING:
        return getattr(importlib.import_module(".lopc", __name__), name)
    raise AttributeError(name)


__all__ = list(_BINDING)
