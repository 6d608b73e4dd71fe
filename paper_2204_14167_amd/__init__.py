"""DISCOS slit-channel particle-grid core on MI355X (gfx950).

The compute path is the HIP library `libdiscos.so` (built from csrc/); the
Python module `discos` binds its C ABI with ctypes.  Import
`paper_2204_14167_amd.discos` for the bindings; `workloads` holds the seeded
synthetic inputs.
"""
