"""MI355X-native RecSplit minimal perfect hash construction.

The construction runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/recsplit.h``; :mod:`.recsplit` is a thin ctypes binding
to that library and :mod:`.keygen` draws seeded synthetic fingerprints.
"""
