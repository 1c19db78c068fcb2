"""g3pcf: anisotropic 3PCF multipoles on one AMD MI355X (gfx950).

``catalogues`` holds the seeded synthetic inputs; ``api`` is the PyTorch front
end of the HIP library (libg3pcf.so, C ABI in include/g3pcf.h).  Submodules
are imported lazily so that the input generators can be used without a GPU or
a built library.
"""
import importlib

__all__ = ["catalogues", "api", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
