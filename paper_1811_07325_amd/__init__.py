"""MI355X (gfx950) Strassen hot path: C = A * B by Strassen's seven-product
recursion (Algorithm 1 of "Stark", Misra et al.) on HIP kernels.

``paper_1811_07325_amd.stark`` is the ctypes binding of ``libstark.so``
(importing it loads the library and fails loudly if it is not built);
``paper_1811_07325_amd.inputs`` holds the seeded input generators.  Submodules
load lazily so the generators can be used without the GPU library.
"""
import importlib

__all__ = ["stark", "inputs"]


def __getattr__(name):
    if name in ("stark", "inputs", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
