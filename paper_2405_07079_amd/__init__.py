"""Out-of-band-metadata allocators (first, next, best and segregated fit)
replayed on AMD Instinct MI355X (gfx950).

* ``hda`` -- binding of the C ABI in ``include/hda.h`` (libhda.so)
* ``workloads`` -- seeded synthetic request streams
* ``build`` -- compiles libhda.so with hipcc
"""
