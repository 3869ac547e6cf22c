"""MI355X-native matrix-free elemental spectral/hp operators.

Submodules: ``shp`` (binding of libshp.so, the HIP operator library) and
``workloads`` (seeded synthetic meshes and coefficients).  Importing the package
loads nothing; ``shp`` loads the library on first use and raises if it is
missing.
"""
