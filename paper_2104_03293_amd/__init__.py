"""MI355X-native state-vector engine for QAOA layers and approximate quantum annealing.

The compute path lives in ``libsv.so`` (hand-written HIP for gfx950 behind a C ABI,
declared in ``include/sv.h``).  ``paper_2104_03293_amd.sv`` is the thin ctypes binding;
``paper_2104_03293_amd.inputs`` holds the seeded synthetic input generators.

Importing this package loads nothing; import the submodules you need.
"""

__all__ = ["inputs", "sv"]
__version__ = "0.1.0"
