"""libfos_mc: MI355X-native Monte Carlo photon transport for particle-laden
slabs (the transport step of FOS, arXiv 2409.00165).

Submodules
  fos        -- ctypes binding of the C ABI in include/fos_mc.h (HIP library)
  workloads  -- seeded synthetic workload recipes (inputs only)
  build      -- in-tree hipcc build of libfos_mc.so
"""
