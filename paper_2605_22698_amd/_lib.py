"""ctypes binding of libe3mi.so (the C ABI in include/e3mi.h).

Argument marshalling only: every step of the computation runs in the HIP
library. PyTorch supplies device memory (through the library's allocator
callbacks, so the caching allocator serves the workspace) and the stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libe3mi.so")

E3MI_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "ENAN",
                -6: "EUNSUPPORTED"}
FP32 = 0
BF16_MIX = 1

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_p = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "e3mi_weight_count": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]),
    "e3mi_model_create": (ctypes.c_int, [ctypes.c_char_p, _p, ctypes.c_size_t, ctypes.c_int, ALLOC_FN, FREE_FN, _p,
                                         ctypes.POINTER(_p)]),
    "e3mi_model_destroy": (ctypes.c_int, [_p]),
    "e3mi_build_graph": (ctypes.c_int, [_p, ctypes.c_int, _p, _p, _p, _p, _p, ctypes.c_double, ctypes.c_double, _p,
                                        ctypes.POINTER(_p)]),
    "e3mi_graph_destroy": (ctypes.c_int, [_p]),
    "e3mi_graph_info": (ctypes.c_int, [_p, _i64p, _i64p]),
    "e3mi_graph_copy_edges": (ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
    "e3mi_energy_forces": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p]),
    "e3mi_energy_forces_static": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p]),
    "e3mi_graph_last_edge_count": (ctypes.c_int, [_p, _i64p, _p]),
    "e3mi_param_grad": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p]),
    "e3mi_hessian_vector": (ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
    "e3mi_hessian_vectors": (ctypes.c_int, [_p, _p, _p, ctypes.c_int, _p, _p, _p]),
    "e3mi_model_set_r_chunk_bytes": (ctypes.c_int, [_p, ctypes.c_size_t]),
    "e3mi_model_set_r_keep_bytes": (ctypes.c_int, [_p, ctypes.c_size_t]),
    "e3mi_profile_select": (ctypes.c_int, [_p, ctypes.c_char_p]),
    "e3mi_model_set_weights": (ctypes.c_int, [_p, _p, ctypes.c_size_t]),
    "e3mi_model_set_flags": (ctypes.c_int, [_p, ctypes.c_int]),
    "e3mi_md_create": (ctypes.c_int, [_p, ctypes.c_int, _p, _p, _p, _p, _p, _p, _p, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, _p, ctypes.POINTER(_p)]),
    "e3mi_md_step": (ctypes.c_int, [_p, ctypes.c_int, ctypes.c_double, _p, _p]),
    "e3mi_md_state": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "e3mi_md_stats": (ctypes.c_int, [_p, _i64p, _i64p, _i64p]),
    "e3mi_md_set_langevin": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_double, _p, _p, _p]),
    "e3mi_md_set_barostat": (ctypes.c_int, [_p, ctypes.c_double, ctypes.c_int, ctypes.c_double, _p, _p, _p]),
    "e3mi_md_cells": (ctypes.c_int, [_p, _p, _i64p, _i64p]),
    "e3mi_graph_set_total_charge": (ctypes.c_int, [_p, _p]),
    "e3mi_md_set_total_charge": (ctypes.c_int, [_p, _p, _p]),
    "e3mi_md_destroy": (ctypes.c_int, [_p]),
    "e3mi_footprint_bytes": (ctypes.c_size_t, [_p, ctypes.c_int64, ctypes.c_int64]),
    "e3mi_profile_enable": (ctypes.c_int, [_p, ctypes.c_int]),
    "e3mi_profile_query": (ctypes.c_int, [_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), _i64p]),
    "e3mi_last_error": (ctypes.c_char_p, []),
}

_lib = None
_lock = threading.Lock()


class E3miError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_22698_amd.build`")
            l = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(l, name)
                f.restype = res
                f.argtypes = args
            _lib = l
    return _lib


def check(code: int) -> None:
    if code != E3MI_OK:
        raise E3miError(code, lib().e3mi_last_error().decode())


def ptr(t) -> Optional[int]:
    """Device or host address of a tensor / array (None for None)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous()
    return t.data_ptr()


class TorchAllocator:
    """Serves the library's device allocations from PyTorch's caching allocator."""

    def __init__(self, device):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, p, ctx):
        self.live.pop(p, None)

    @property
    def bytes_live(self) -> int:
        return sum(t.numel() for t in self.live.values())
