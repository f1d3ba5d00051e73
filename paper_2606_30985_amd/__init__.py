"""MI355X-native Heisenberg-picture tensor-network dynamics for the 2D TFIM.

The compute path is the C-ABI library ``libhpt.so`` (hand-written gfx950 HIP
kernels, see ``include/hpt.h``); ``hpt`` is its thin ctypes binding.
"""
