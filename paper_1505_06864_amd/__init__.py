"""MI355X-native decomposition-method (DM) solver for block-tridiagonal systems.

``B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i`` (arXiv:1505.06864, Sec. 2):
the N block rows are split into P subsystems eliminated independently,
a coupling block-tridiagonal system of P-1 rows is solved by the Thomas
algorithm or by the DM itself, and the subsystem interiors are recovered.

Every step runs in the HIP kernels of ``libbtd.so`` (gfx950), reached
through its C ABI (``include/btd.h``); this package only marshals
arguments.  Importing it loads nothing; the first call into
:mod:`paper_1505_06864_amd.btd` loads the library and raises if it is
missing.
"""
__all__ = ["btd", "inputs"]
