"""MI355X (gfx950) solver for one backward-Euler step of hybridized
three-field poromechanics (Q1 displacement, RT0-hybridized face pressure, P0
cell pressure) with macro-element stabilization and a block triangular AMG
preconditioner inside flexible GMRES.

The computation lives in the HIP library ``libporomech.so`` behind the C ABI
of ``include/poromech.h``; ``solver.PoroSolver`` is the Python binding and
``autograd`` provides the differentiable step and the checkpointed
multi-step driver.  Importing ``solver`` fails if the library is not built.
"""

__all__ = ["solver", "autograd"]
