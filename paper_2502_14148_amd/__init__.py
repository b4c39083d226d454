"""MI355X-native hot path of the Oceananigans nonhydrostatic ocean model.

The compute path lives in the HIP library built from ``csrc/`` (``liboc.so``);
``oc`` is its thin ctypes binding and ``inputs`` holds the seeded synthetic
input generators.  Importing the package does not load the library.
"""
