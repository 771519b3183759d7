"""FP64 CPU oracle of the improved axisymmetric lattice Boltzmann scheme.

Test infrastructure only: used by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.
"""
