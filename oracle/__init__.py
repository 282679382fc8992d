"""CPU oracle for the flatspin dipole model (Jensen et al., Sec. II).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library; it
is imported solely by tests/, the package smoke check and the benchmark's
CPU-baseline leg.  The product path never imports, links or calls it, and it
shares no code with the HIP library (only the seeded input generators of
paper_2002_11401_amd.workloads feed both).

  definition.py  tier 0: numpy, every field recomputed from Eq. 3 after every
                 flip, linear argmax (tiny inputs only)
  relax.cpp      tier 1: plain C++ FP64 (no FMA contraction), cell-grid
                 neighbour sets, neighbour rows re-summed from Eq. 3 after a
                 flip, ordered candidate set for the argmax; own Philox
  native.py      ctypes binding of relax.cpp

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, special cases, invariants or brute force (see the pin table in
the design notes).  Nothing here is "parity unpinned".
"""
