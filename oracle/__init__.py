"""FP64 CPU oracle for the explicit velocity-difference (EVD) multicomponent
lattice Boltzmann method with forcing (Lourenco, Constantino & Tavares,
"Forcing mass transfer approach in multicomponent miscible mixtures using the
lattice Boltzmann method", Chem. Eng. Sci. 2025, arXiv 2504.07059).

This package is TEST INFRASTRUCTURE, not part of the product.  Only the test
suite (``tests/``), ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in it.  The HIP library in
``paper_2504_07059_amd`` shares no code with it and never calls it.

Modules
-------
lattice      D2Q9 / D3Q19 direction tables and weights (Sec. 2, eq. for e_alpha^i).
evd          the method itself, vectorised over nodes with torch float64:
             constants, initialisation, moments, cross-relaxation solve,
             collision with forcing, pull streaming with second-order
             interpolation, the impermeable-wall scheme, observables.
scalar       an independent per-node pure-Python implementation (push-form
             streaming, hand-written elimination for the tau system), used
             only as a brute-force cross-check on tiny lattices.
stability    the linear-stability matrix of the velocity-difference relaxation.
closed_forms analytic results the method must reproduce (binary erf profile,
             hypsometric/centrifugal equilibrium, Luo-Girimaji and ternary
             closed forms of the tau relation).
make_workloads  writes the accepted diffusivity draws used by the workloads.

Every function cites the section / equation of the paper it follows.  Where
the paper is silent the reading taken is stated at the function.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(``tests/test_oracle_*.py``), except the D3Q19 extension (the paper is 2-D
only), which is pinned by invariants and the dimension-free closed forms only.
"""
