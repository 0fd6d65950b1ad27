"""MI355X-native algebraic-distance AMG setup path.

The compute path lives in the HIP library `libalgdist.so` (sources under
csrc/, C ABI in include/algdist.h).  `paper_1106_5990_amd.algdist` is the
thin ctypes binding; it raises on import if the library has not been built.
`paper_1106_5990_amd.workloads` builds seeded synthetic inputs.
"""
