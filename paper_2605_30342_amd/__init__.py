"""MI355X-native GAVIS visibility-field path.

The hot path (VF CONST: visibility-field construction; VF QUERY: uncertainty
rasterisation of candidate views; next-best-view argmax) runs in HIP kernels
for gfx950 behind the C ABI of include/gavis.h.  This package holds the
ctypes binding (`_lib`), thin Python wrappers that allocate device memory
with PyTorch (`api`), the seeded input generator (`scenes`) and the build
script (`build`).  Importing the package does not load the library; the
first call that needs it does, and fails loudly if it has not been built.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "api", "build"]


def __getattr__(name):
    if name in ("api", "_lib", "build", "serve"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
