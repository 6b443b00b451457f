"""Plain FP64 CPU oracle for the inexact-Krylov linear-response method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: its only common dependency is the seeded input description in
``workloads``.

Every function is written from the paper (Herbst & Sun, "Efficient Krylov
methods for linear response in plane-wave electronic structure
calculations") and cites the section / equation / algorithm it follows.
Where the paper is silent or ambiguous, the reading taken is stated in the
function's docstring.

Modules
  system      plane-wave bases, grids, F / F^-1, the model Hamiltonian
              (dense and FFT-applied)                       [Sec. 2.3.1, eq. (Hamiltonian)]
  groundstate eigenpairs, occupations, Fermi level, density [eq. (KS), (density)]
  response    chi0 by sum over states, finite differences and Sternheimer;
              Hxc kernel; dielectric adjoint                 [eq. (chi0), (op_discretised)]
  gmres       inexact GMRES(m) and the CG-tolerance strategies
                                                             [Alg. 1, Tables 1 and 3]

Parity status: every function is pinned by a ``-m "not gpu"`` test except
those whose docstring says "parity unpinned".
"""
