"""Block-space (lambda) thread mapping for embedded Sierpinski gaskets on MI355X.

The compute path is the HIP library ``libsg.so`` (C ABI declared in
``include/sg.h``); :mod:`paper_1706_04552_amd.sg` is its thin ctypes binding
over torch device tensors.  :mod:`paper_1706_04552_amd.inputs` holds the seeded
synthetic input generators.  Submodules are imported on first use so that the
input generators stay usable without a GPU runtime.
"""
import importlib

__all__ = ["sg", "inputs", "build", "batch", "serving"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
