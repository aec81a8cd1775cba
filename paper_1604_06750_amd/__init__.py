"""MI355X-native multi-scale S-fraction reduced-order wavefield simulation.

The compute path is libsfrom.so (HIP for gfx950) behind the C ABI declared in
include/sfrom.h; ``paper_1604_06750_amd.sfrom`` is its ctypes binding and
``paper_1604_06750_amd.problem`` a thin helper that marshals synthetic
workloads into ABI calls.
"""
