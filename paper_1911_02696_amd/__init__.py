"""MI355X-native positional population count (pospopcnt).

The work runs in hand-written HIP kernels for gfx950 inside ``libpospopcnt.so``
(C-ABI declared in include/pospopcnt.h); this package is the thin Python binding.
"""
