"""MI355X (gfx950) Frequency Selective Extrapolation.

Submodules: ``fse`` (ctypes binding of libfse.so), ``synth`` (seeded
synthetic inputs), ``build`` (hipcc build of the library).  Nothing is
imported eagerly, so ``synth`` can be used without the built library.
"""
