"""MI355X-native fast block-structured AMG for Toeplitz-like-plus-Cross
systems (arXiv 2202.11288).

* ``paper_2202_11288_amd.binding`` -- ctypes binding of ``libamg.so`` (the C
  ABI declared in ``include/amg.h``); importing it raises if the library has
  not been built.
* ``paper_2202_11288_amd.build`` -- compiles ``csrc/`` for gfx950 into
  ``libamg.so`` in this directory.
"""
