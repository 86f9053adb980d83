"""MI355X (gfx950) augmented Population Annealing Monte Carlo.

The library itself is ``libpamc.so`` (C ABI in ``include/pamc.h``); the
``pamc`` submodule is its ctypes binding.  Build with ``build.build()``.
"""
