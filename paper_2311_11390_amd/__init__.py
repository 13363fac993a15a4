"""libblockalif: block-wise ALIF simulation and surrogate-gradient training on
one AMD Instinct MI355X (gfx950).

Submodules:
  _lib    ctypes binding of the C ABI (include/blockalif.h)
  alif    torch-facing wrappers: forward/backward, autograd ops, readout
  serving continuous-batching server binding
  synth   seeded synthetic workloads
  build   hipcc build of libblockalif.so
"""
import importlib

__all__ = ["alif", "serving", "synth", "build"]


def __getattr__(name):
    if name in ("alif", "serving", "synth", "build", "_lib"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
