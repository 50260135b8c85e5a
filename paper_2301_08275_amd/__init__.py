"""MI355X-native time-splitting spectral (TSSP) Gross-Pitaevskii engine.

The compute path lives in the HIP library ``libgpe.so`` (built from
``csrc/``) behind the C ABI declared in ``include/gpe.h``; ``gpe`` is the thin
ctypes binding over it.  Importing this package loads nothing.
"""
__all__ = ["gpe", "inputs"]
