"""MI355X-native evaluation of PDE right-hand sides on 3-D grid blocks with
ghost zones (the data-parallel hot path of Chemora, arXiv:1410.1764).

The compute lives in ``libchemora.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/chemora.h``).  ``paper_1410_1764_amd.chemora``
is the thin ctypes binding; it is imported lazily so that the seeded input
generators in ``paper_1410_1764_amd.inputs`` can be used without a GPU.
"""

__all__ = ["chemora", "inputs"]


def __getattr__(name):
    if name == "chemora":
        from . import chemora as _c
        return _c
    raise AttributeError(name)
