"""MI355X-native hot path of the multi-resolution fast lattice Green's function method.

The solver lives in the HIP/C++ shared library built from ``csrc/`` (C ABI declared in
``include/lgf.h``); ``lgf`` is its thin Python binding.  ``workloads`` generates seeded
synthetic inputs.  Importing this package does not load the library; ``lgf.load()`` does.
"""
