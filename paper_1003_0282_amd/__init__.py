"""MI355X-native improved axisymmetric lattice Boltzmann solver (arXiv:1003.0282).

Submodules:
    workloads  seeded problem descriptions (no solver arithmetic)
    lbaxi      ctypes binding of the HIP C-ABI library ``liblbaxi.so``
"""
