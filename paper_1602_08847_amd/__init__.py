"""MI355X-native MUFFIN primal-dual reconstruction.

``paper_1602_08847_amd.muffin`` is the Python binding of the HIP library
``libmuffin.so`` (C-ABI declared in ``include/muffin.h``); ``synth`` draws
seeded synthetic cubes.  Importing the package loads nothing: the library is
loaded, and must be present, when ``muffin`` is imported.
"""
