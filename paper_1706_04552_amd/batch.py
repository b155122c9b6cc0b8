"""Batched gaskets over the C ABI: a planned batch with a captured hipGraph,
the per-pass entry used by continuous batching, and the launch-shape
autotuner.  Argument marshalling only; the passes run in libsg's kernels."""
import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import sg


@dataclass
class Gasket:
    """`steps` life generations of one gasket from `inp` into `out`
    (`work`: third buffer, needed when more than one pass runs)."""
    r: int
    steps: int
    inp: torch.Tensor
    out: torch.Tensor
    work: Optional[torch.Tensor] = None


def _ptr(t: Optional[torch.Tensor], r: int, name: str):
    if t is None:
        return None
    return sg._dev(t, torch.uint8, (1 << r) * (1 << r), name)


def checked_ptr(t: torch.Tensor, r: int, name: str) -> int:
    """Device address of an n x n uint8 CUDA tensor (checked), for PASS_ITEM arrays."""
    return _ptr(t, r, name).value


def _gasket_array(gaskets: Sequence[Gasket]):
    arr = (sg.sg_gasket * len(gaskets))()
    for i, g in enumerate(gaskets):
        arr[i].in_ = _ptr(g.inp, g.r, "inp")
        arr[i].out = _ptr(g.out, g.r, "out")
        arr[i].work = _ptr(g.work, g.r, "work")
        arr[i].r = g.r
        arr[i].steps = g.steps
    return arr


def make_tune(rho: int = 64, steps_per_pass: int = 32, groups_per_cu: int = 0,
              threads: int = 256) -> "sg.sg_tune":
    return sg.sg_tune(rho, steps_per_pass, groups_per_cu, threads)


def default_tune() -> "sg.sg_tune":
    t = sg.sg_tune()
    sg._check(sg.load().sg_tune_default(ctypes.byref(t)), "sg_tune_default")
    return t


def autotune(gaskets: Sequence[Gasket], stream=None):
    """Fastest launch shape for this batch, and its time in ms."""
    arr = _gasket_array(gaskets)
    best, ms = sg.sg_tune(), ctypes.c_float()
    sg._check(sg.load().sg_batch_autotune(arr, len(gaskets), ctypes.byref(best), ctypes.byref(ms),
                                          sg._stream(stream)), "sg_batch_autotune")
    return best, ms.value


class Batch:
    """A planned batch whose passes are captured in one hipGraph."""

    def __init__(self, gaskets: Sequence[Gasket], tune=None):
        self.gaskets = list(gaskets)  # keeps the tensors alive
        self.tune = tune if tune is not None else default_tune()
        arr = _gasket_array(self.gaskets)
        h = ctypes.c_void_p()
        sg._check(sg.load().sg_batch_create(arr, len(self.gaskets), ctypes.byref(self.tune),
                                            ctypes.byref(h)), "sg_batch_create")
        self._h = h

    def run(self, graph: bool = True, stream=None):
        lib = sg.load()
        fn = lib.sg_batch_run if graph else lib.sg_batch_run_eager
        sg._check(fn(self._h, sg._stream(stream)), "sg_batch_run")

    def stats(self):
        p, c = ctypes.c_uint64(), ctypes.c_uint64()
        sg._check(sg.load().sg_batch_stats(self._h, ctypes.byref(p), ctypes.byref(c)), "sg_batch_stats")
        return {"passes": p.value, "cell_steps": c.value}

    def close(self):
        if self._h:
            sg.load().sg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# numpy layout of sg_pass_item
PASS_ITEM = np.dtype([("src", np.uint64), ("dst", np.uint64), ("r", np.int32),
                      ("steps", np.int32)])
assert PASS_ITEM.itemsize == ctypes.sizeof(sg.sg_pass_item)


def run_static(items: List[tuple], tune, stream=None):
    """One batched pass with no context and no allocation
    (sg_pass_run_static): items (src, dst, r, steps) with src/dst uint8
    device tensors, at most SG_PASS_STATIC_MAX of them."""
    arr = (sg.sg_pass_item * max(1, len(items)))()
    for i, (src, dst, r, steps) in enumerate(items):
        arr[i].src = _ptr(src, r, "src")
        arr[i].dst = _ptr(dst, r, "dst")
        arr[i].r = r
        arr[i].steps = steps
    sg._check(sg.load().sg_pass_run_static(arr, len(items), ctypes.byref(tune),
                                           sg._stream(stream)), "sg_pass_run_static")


class PassContext:
    """Device item table for repeated batched passes over a changing set of
    gaskets (continuous batching)."""

    def __init__(self, capacity: int):
        h = ctypes.c_void_p()
        sg._check(sg.load().sg_pass_ctx_create(capacity, ctypes.byref(h)), "sg_pass_ctx_create")
        self._h = h
        self.capacity = capacity

    def run_array(self, items: np.ndarray, tune, stream=None):
        """items: a C-contiguous PASS_ITEM array of raw device pointers (taken
        from checked tensors by the caller), r and steps."""
        if items.dtype != PASS_ITEM or not items.flags.c_contiguous:
            raise TypeError("items must be a C-contiguous PASS_ITEM array")
        ptr = items.ctypes.data_as(ctypes.POINTER(sg.sg_pass_item))
        sg._check(sg.load().sg_pass_run(self._h, ptr, len(items), ctypes.byref(tune),
                                        sg._stream(stream)), "sg_pass_run")

    def run(self, items: List[tuple], tune, stream=None):
        """items: (src, dst, r, steps) with src/dst uint8 device tensors."""
        arr = (sg.sg_pass_item * max(1, len(items)))()
        for i, (src, dst, r, steps) in enumerate(items):
            arr[i].src = _ptr(src, r, "src")
            arr[i].dst = _ptr(dst, r, "dst")
            arr[i].r = r
            arr[i].steps = steps
        sg._check(sg.load().sg_pass_run(self._h, arr, len(items), ctypes.byref(tune),
                                        sg._stream(stream)), "sg_pass_run")

    def close(self):
        if self._h:
            sg.load().sg_pass_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
