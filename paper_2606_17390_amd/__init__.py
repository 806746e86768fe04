"""MI355X-native finite-strain Hill-48 hex8 residual / tangent / CSR / VJP.

The compute path is the HIP library ``libfem.so`` (C ABI in ``include/fem.h``);
``paper_2606_17390_amd.fem`` is its ctypes binding.  Importing this package
does not load the library; the binding loads it on first use and raises if it
is missing.
"""
__all__ = ["fem", "synth"]
