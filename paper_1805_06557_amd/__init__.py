"""MI355X-native REXI time stepping for the shallow-water equations on the
rotating sphere (arXiv:1805.06557): a HIP library (librexi_swe.so, C-ABI in
include/rexi_swe.h) and its thin Python binding.

Submodules are imported on demand so that ``paper_1805_06557_amd.inputs``
(seeded synthetic inputs) can be used without loading the library.
"""

__all__ = ["api", "inputs", "configs"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
