"""MI355X-native Surface Octahedral Probe (SOP) query-and-shade library.

Submodules:
  sop       binding of the C ABI (include/sop.h) over torch tensors
  autograd  SopShade autograd.Function
  scenes    seeded synthetic workloads (input generation only)
  build     hipcc build of libsop.so for gfx950

Importing the package does not load the HIP library; the binding loads it on first use and
raises if it is missing.
"""

__all__ = ["sop", "autograd", "scenes", "build"]
