"""MI355X-native scalar spherical harmonic synthesis after the Wavemoth paper
(Seljebotn, arXiv:1110.4874).

Submodules:
  sht        ctypes binding of libsht.so (include/sht.h): plans, synthesis,
             private test entry points.  Fails loudly if the library is not
             built.
  synthetic  seeded synthetic inputs (random draws only).
  build      builds libsht.so for gfx950 in-tree.
"""
