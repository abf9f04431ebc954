"""MI355X-native evaluation of PDE right-hand sides on 3-D grid blocks with
ghost zones (the data-parallel hot path of Chemora, arXiv:1410.1764).

The compute lives in ``libchemora.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/chemora.h``); ``paper_1410_1764_amd.chemora`` is
the thin ctypes binding.  ``paper_1410_1764_amd.inputs`` holds the seeded
input generators and needs no GPU.  Submodules are imported explicitly.
"""
