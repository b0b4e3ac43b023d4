"""fleetstage: MI355X-native fleet staging of air ambulances (arXiv:2001.05291).

The compute path lives in ``libfleetstage.so`` (hand-written HIP for gfx950,
C ABI declared in ``include/fleetstage.h``); ``fleetstage`` is the thin ctypes
binding over it.  Importing this package loads nothing; the library is loaded
on the first call into the binding.
"""

__all__ = ["fleetstage", "synth"]
