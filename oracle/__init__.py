"""Plain, slow FP64 CPU oracle for the discrete-ordinates RTE solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver product imports, links or
executes anything here: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path;
both sides receive their inputs from the seeded generators in ``rte_inputs``.

Modules
  discretisation  setup (scattering kernel, scaling, RHS) and the operator L
  network         MGN1 reader, convolutions written out tap by tap,
                  CoeffNet and the MgNet V-cycle
  krylov          flexible GMRES with modified Gram-Schmidt and Givens
  solve           end-to-end build + FGMRES driver
  direct          independent solvers used only to pin the rest (dense LU,
                  transport sweeps, source iteration, the isotropic limit)
  atfps           the adaptive scheme of Sec. 2.3: selection, face bases,
                  compressed system, layer reconstruction, the filtered loss
  tfps            the tailored finite point scheme of Sec. 2.2 (2D): per-cell
                  eigen-bases, midpoint continuity and inflow conditions, the
                  assembled system and its sparse solve

Functions whose result is not pinned by any test say "parity unpinned" in
their docstring.
"""
from . import atfps, direct, discretisation, krylov, network, solve, tfps  # noqa: F401
