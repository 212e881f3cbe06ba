"""MI355X-native weighted Euler characteristic transform (WECT / WECF).

The compute path is libwect.so (hand-written HIP kernels for gfx950 behind the
C ABI in include/wect.h).  This package only marshals arguments; importing it
does not load the library, the first call does (and fails loudly if it is
missing).
"""
import importlib

__version__ = "0.1"

_SUBMODULES = {"api", "_lib", "build", "tune"}


def __getattr__(name):
    if name in _SUBMODULES or name.startswith("__"):
        return importlib.import_module(f"{__name__}.{name}")
    api = importlib.import_module(f"{__name__}.api")
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)
