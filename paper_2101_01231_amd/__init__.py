"""MI355X-native RIDG (regionally-implicit discontinuous Galerkin) hot path.

The compute path lives in ``libridg.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/ridg.h``); ``ridg.py`` is a thin ctypes binding and
``inputs.py`` prepares seeded synthetic initial data.
"""
