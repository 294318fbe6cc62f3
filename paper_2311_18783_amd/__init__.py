"""MI355X-native two-level GenEO-type Schwarz preconditioner for H(curl).

The library is libgeneo.so (HIP for gfx950, C ABI in include/geneo.h); the
Python binding is `paper_2311_18783_amd.geneo`, imported on first use so that
the package can be imported to build the library."""
import importlib

__all__ = ["geneo", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
