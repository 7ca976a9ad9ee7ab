"""Wilson-Dirac operator and Krylov solves on AMD Instinct MI355X (gfx950).

``paper_1112_5280_amd.wilson`` binds the HIP library ``libwilson.so`` (C ABI in
``include/wilson.h``); ``paper_1112_5280_amd.synth`` draws seeded synthetic
gauge fields and sources. Importing the package itself loads nothing, so the
input generators work on machines without the library; importing ``wilson``
raises if the library is not built.
"""
__all__ = ["synth", "wilson", "build"]
