"""MI355X-native warp-primitive library (CUDA 32-lane warp-function semantics
on gfx950 wave64).

Importing the package loads nothing native.  ``paper_2112_10034_amd.cox``
is the thin ctypes binding over ``libcox.so`` (the C-ABI library declared in
``include/cox.h``); it raises if the library has not been built.
``paper_2112_10034_amd.inputs`` holds the seeded input recipes.
"""
