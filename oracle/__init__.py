"""FP64 CPU oracle of the hybridized, stabilized Q1-RT0-P0 poromechanics step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything here.  The
HIP library never calls it, and it never calls the HIP library: the two share
no code (only the seeded input generators in ``synth``).

It is a plain, slow, obviously-correct restatement of the paper (Frigo,
Castelletto, Ferronato, White, "Efficient solvers for hybridized three-field
mixed finite element coupled poromechanics"):

* ``mesh``      structured hexahedral topology and numbering (Sec. 2)
* ``element``   Q1 elasticity / coupling and RT0 mass element integrals
                (Appendix A, eq. MFE_matrix and MHFE_matrix)
* ``system``    static condensation (eq. hmfeSys, A_33H), macro-element
                pressure-jump stabilization (eq. J_def, stab_A), Dirichlet
                treatment, right-hand side (eq. MHFE_vector, f~_n of Sec. 2.1)
* ``solve``     direct sparse solve of the exact system, the block upper
                triangular preconditioner with exact inner solves (eq.
                hybridPrec, variant M_I^(h)), B~_p (eq. app_Bp), C~_pi, FGMRES,
                flux reconstruction and conservation residuals
* ``mfe``       the non-hybridized mixed system (eq. mfeSys, MFE_matrix,
                MFE_vector) with the stabilized pressure block, C~_p and the
                block triangular preconditioner of eq. prec (variant M_I^(m));
                pinned to the hybrid oracle by the equivalence of the two
                formulations
* ``adjoint``   transposed solve and per-cell gradients w.r.t. log kappa and
                log E (an extension: the paper has no adjoint)
* ``terzaghi``  one-dimensional consolidation closed form (pin only)

Parity status of each function is stated in its docstring; functions that
nothing independent pins say "parity unpinned".
"""
