"""MI355X (gfx950) hot path of the Inexact Bregman Sparse Newton method for exact OT.

- ``paper_2603_07156_amd.ibsn``: ctypes binding of libibsn.so (the C ABI in
  include/ibsn.h), argument marshalling only.
- ``paper_2603_07156_amd.workloads``: seeded synthetic instances (inputs only).
- ``paper_2603_07156_amd.build``: builds libibsn.so with hipcc for gfx950.
"""
__all__ = ["ibsn", "workloads", "build"]
