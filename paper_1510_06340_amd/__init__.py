"""MI355X-native MUSTA-FORCE step for ideal relativistic hydrodynamics.

The package holds the HIP library (``csrc/``, built into ``libmf.so``), its
thin ctypes binding (:mod:`.mf`) and the seeded synthetic input generators
(:mod:`.inputs`).  Importing the package loads nothing; the binding loads the
shared library on first use and raises if it has not been built.
"""

__all__ = ["inputs", "mf"]
