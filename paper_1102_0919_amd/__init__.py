"""MI355X-native self-learning algebraic multigrid for extremal singular triplets and eigenpairs.

The numeric work runs in ``libslamg.so`` (HIP kernels for gfx950 behind the C ABI in
``include/slamg.h``); ``api`` is the Python binding and ``workloads`` builds seeded synthetic inputs.
"""
