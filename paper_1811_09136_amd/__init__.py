"""MI355X-native REPT semi-triangle counting (arXiv:1811.09136).

The counting pass runs in the HIP library ``librept.so`` (C ABI in ``include/rept.h``);
``rept`` is its ctypes binding, ``batch`` the batched runtime, ``serve`` the serving loop.
"""
from .rept import (  # noqa: F401
    Graph,
    Params,
    ReptError,
    hash_slots,
    lib,
    make_job,
    to_device_edges,
    tuning,
)
