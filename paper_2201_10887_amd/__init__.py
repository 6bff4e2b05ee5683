"""MI355X-native adaptive heightfield renderer (Cornel, Horvath, Waser 2022).

The compute path lives in ``libhfr.so`` (hand-written HIP for gfx950 behind
the C ABI in ``include/hfr.h``); ``api`` binds it with the same names.
Importing this package does not load the library; the first call does.
"""
