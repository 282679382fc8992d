"""MI355X-native (gfx950) artificial-spin-ice relaxation library.

Implements the flatspin dipole model (Jensen et al., Sec. II): FP64
dipole-dipole fields from neighbour tables, the generalized Stoner-Wohlfarth
switching test, and deterministic single-spin-flip relaxation, as HIP kernels
behind the C ABI of include/asi.h.

  paper_2002_11401_amd.asi        ctypes binding of libasi.so (the product path)
  paper_2002_11401_amd.workloads  seeded synthetic lattices and field protocols
  paper_2002_11401_amd.build      hipcc build of libasi.so

Importing the package loads nothing; the library is loaded on first use.
"""

__all__ = ["asi", "workloads", "build"]
