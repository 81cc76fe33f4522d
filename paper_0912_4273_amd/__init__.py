"""SimpleX2 direction-conserving photon transport + hydrogen chemistry on
AMD MI355X (gfx950): HIP kernels behind the C ABI of include/sx.h.

  sx       -- Python binding of libsx.so (marshalling only)
  gridgen  -- seeded synthetic workloads shaped like the paper's tests
  build    -- compiles libsx.so in-tree with hipcc
"""
from . import gridgen  # noqa: F401

__all__ = ["gridgen", "sx", "build"]
