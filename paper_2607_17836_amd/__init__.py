"""MI355X-native Lagrangian particle hot path (gfx950 HIP behind a C ABI).

Importing the package does not load the native library; the first use of
``paper_2607_17836_amd.lpt`` does, and raises if ``liblpt.so`` is missing.
"""
