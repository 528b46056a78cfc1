"""MI355X-native matching-based AMG-preconditioned CG.

``paper_2006_16147_amd.amg`` is the thin ctypes binding of the HIP C-ABI
library (include/amg.h); ``paper_2006_16147_amd.inputs`` holds the seeded
synthetic workloads. Importing the package loads nothing; the binding loads
the shared library on first use and fails loudly if it is missing.
"""
