"""Plain FP64 CPU oracle of the weight-adjusted smoothly-varying SC-PML DGTD step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the package smoke check and the
``cpu_baseline`` leg of the benchmark use it.  It shares no code with the HIP
library; both receive the same seeded inputs (mesh, cubature rule, initial
fields, source parameters) from ``paper_2006_02551_amd.inputs``.

Modules, in the order the method is built:

* ``refel``   reference tetrahedron: nodes, Lagrange operators, cubature
              interpolation V_q and projection P_q (Sec. II-A, eqs. (14)-(21)).
* ``mesh``    affine geometry, outward normals, face matching (Sec. II-A,
              text after eq. (17)).
* ``pml``     SC-PML profiles and the tensor entries of eq. (9).
* ``rhs``     semi-discrete right-hand side, eqs. (26)-(29), with the upwind
              curl operator of eqs. (10)-(17).
* ``brute``   the direct stored-mass-matrix scheme, eqs. (10)-(15)
              (the paper's "SV-paved" method), for comparison.
* ``ec``      element-constant coefficients (the paper's "EC-paved"
              configuration, Sec. III).
* ``lserk``   five-stage fourth-order low-storage Runge-Kutta.
* ``readout`` energy and point probes.
* ``run``     assembles a whole simulation from inputs.

Every floating-point computation is float64.  Parity status of every function
is recorded in its module docstring; all are pinned by the CPU tests.
"""
