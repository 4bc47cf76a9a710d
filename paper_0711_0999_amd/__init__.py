"""MI355X (gfx950) lattice step of nonequilibrium DMFT for the Falicov-Kimball
model in a uniform field (Freericks, arXiv:0711.0999).

The compute lives in the HIP library libfkdmft.so (C ABI: include/fkdmft.h);
``fkdmft`` is its ctypes binding.  ``configs`` names the benchmark workloads and
``inputs`` holds the seeded synthetic input generators.
"""
