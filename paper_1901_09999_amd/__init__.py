"""MI355X-native PSF matching (Alard-Lupton, as formulated by Price & Magnier).

Submodules:
  psfm   -- ctypes binding of the HIP library (include/psfm.h)
  synth  -- seeded synthetic image pairs (inputs only)
"""
__all__ = ["psfm", "synth"]
