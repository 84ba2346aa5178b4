"""MI355X-native lattice spring model (LSM) hot path.

``paper_2201_04565_amd.lsm`` is the Python binding of the C-ABI library
``liblsm.so`` (hand-written HIP kernels for gfx950); ``inputs`` holds the
seeded image generators.  Importing the package does not load the library.
"""
