"""One-reduce (lagged-normalization, compact-WY) MGS-GMRES on AMD MI355X.

The solver lives in a C-ABI shared library of HIP kernels for gfx950
(``libgmres_hip.so``, interface in ``include/gmres.h``); ``native`` is a thin
ctypes binding to it. ``problems`` builds seeded synthetic inputs.
"""

__version__ = "0.1.0"
