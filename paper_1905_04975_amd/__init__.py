"""MI355X-native (gfx950) FP64 Schur-reduction engine.

The product path is the HIP library ``libschur_mi355x.so`` (C ABI in
``include/schur.h``) with the thin ctypes binding in ``schur.py``;
``inputs.py`` holds the seeded synthetic input generators.
"""
