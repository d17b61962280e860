"""MI355X (gfx950) solver for scenario-tree stochastic MPC by accelerated dual
proximal gradient (Sampathirao et al., arXiv 1604.01074).

The solver lives in ``libsmpc.so`` (HIP kernels + float64 host setup) behind
the C ABI of ``include/smpc.h``; ``smpc`` is its ctypes binding and ``solver``
a thin object layer.  Importing ``smpc`` fails if the library is not built.
"""

__all__ = ["smpc", "solver", "build"]
