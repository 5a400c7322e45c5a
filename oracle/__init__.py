"""Plain FP64 CPU oracle for the hyper-reduced Lagrangian-hydro ROM.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the HIP library and its Python binding) never
imports, calls or links anything here, and this package never imports the
product path: the two share no code, no tables and no constant generators.

Modules, in the order of the paper's method:

* ``fe``       -- Q2 kinematic / Q1 thermodynamic spaces on uniform Cartesian
                  meshes, Gauss-Legendre quadrature (Sec. 2.1, spatial
                  discretisation).
* ``problems`` -- initial conditions of the benchmark problems (Sec. 6.1).
* ``fom``      -- mass matrices, the force matrix contractions F.1 and F^T.v,
                  the time-step estimate and the RK2-average integrator with
                  adaptive step control (eq. fom, eq. forceOneforceTv,
                  eq. RK2-avg, eq. adaptive-timestep).
* ``windows``  -- time windows and per-window snapshot matrices (Sec. 4.4, 4.5).
* ``pod``      -- POD by thin SVD and the energy criterion (eq. SVD,
                  eq. energy_criteria).
* ``deim``     -- oversampled greedy DEIM, pseudo-inverse, element closure
                  (Sec. 3.7, 3.3).
* ``rom``      -- SNS hyper-reduced ROM with RK2-average and windows
                  (eq. RK2-avg-rom-hr, eq. rom-hr-sns, eq. ic-tw, eq. relerrors).
* ``mlp``      -- the MLP surrogate of the reduced force coefficients (not
                  in the paper): bfloat16-operand forward and backward, Adam,
                  training targets from the DEIM chain, and the surrogate ROM
                  run with DEIM audits and fallback.

Everything is float64 NumPy/SciPy.
"""
