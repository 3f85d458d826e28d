"""MI355X (gfx950) oil-paint filter.

The filter itself runs in hand-written HIP kernels inside liboilpaint.so,
reached through its C-ABI (include/oilpaint.h).  This package is the thin
Python side: `binding` marshals torch tensors into that ABI (the batched
form included: `binding.batch`, `binding.Plan`, `binding.Queue`), `serve`
drives the served form, `tune` picks launch shapes, `synth` draws seeded
inputs.

Submodules are imported lazily so that `synth` can be used without loading
the GPU library.
"""
import importlib

__all__ = ["binding", "synth", "serve", "tune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
