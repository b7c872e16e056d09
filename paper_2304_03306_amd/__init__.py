"""MI355X-native time stepping of the confined polar-active-fluid (TTSH)
velocity equation under the damping-mask boundary treatment.

The compute path is the HIP library ``libttsh.so`` (hand-written gfx950
kernels behind a C ABI, declared in ``include/ttsh.h`` and ``include/fno.h``);
this package holds the thin ctypes binding (``paper_2304_03306_amd.ttsh``),
the build step and the seeded workload generators.
"""
