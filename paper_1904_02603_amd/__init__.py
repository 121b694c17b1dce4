"""MI355X-native VeST hot path: C-ABI HIP library plus a thin ctypes binding.

Submodules:
  vest      -- binding of the C ABI declared in include/vest.h (loads libvest.so)
  schedule  -- host-side pruning schedule (VeST^man / VeST^auto)
  synth     -- seeded synthetic inputs
"""
__all__ = ["vest", "schedule", "synth"]
