"""MI355X-native FastMap epipolar adjustment.

The compute path lives in the HIP/C library ``libfastea.so`` (built from
``csrc/``); ``fastea`` is its thin ctypes binding.  Importing this package does
not load the library, so the CPU-only scene generator can be used without it.
"""

__all__ = ["synth", "fastea"]
