"""MI355X-native hot path of a fully relativistic electromagnetic PIC step.

Field interpolation, relativistic Boris push and charge-conserving current
deposition on a Yee mesh, followed by the FDTD field advance, as hand-written
HIP kernels for gfx950 behind the C ABI declared in ``include/pic.h``
(``libpic.so``).  ``paper_1310_0930_amd.pic`` is the thin ctypes binding;
``paper_1310_0930_amd.inputs`` draws seeded synthetic workloads.

Importing the package loads nothing; the binding loads ``libpic.so`` on first
use and raises if it is missing.
"""
__all__ = ["inputs", "pic"]
