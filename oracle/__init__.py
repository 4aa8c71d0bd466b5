"""Plain FP64 CPU oracle for the repulsive-curves hot path (test infrastructure).

This package is test infrastructure, not part of the product.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the HIP library: it is written directly from the
paper's definitions (Sec. 4 "Discretization", Sec. 7.1 "Constraints and
Potentials", App. B "Acceleration Scheme"), evaluated in float64 with numpy
and scipy, and is deliberately slow and simple.

Modules
-------
``tpe``          discrete tangent-point energy and its exact differential
                 (Sec. 4.1, eqs. DiscreteEnergy / DiscreteKernel), plus the
                 edge-midpoint variant that Barnes-Hut approximates (App. B.1).
``sobolev``      the Sobolev-Slobodeckij Gram matrices B and B0 (Sec. 4.2),
                 their quadratic forms and the kernel-matrix form (App. B.3.4).
``constraints``  barycenter, total-length and edge-length constraints with
                 exact Jacobians (Sec. 7.1).
``solve``        dense saddle-point solves for the projected gradient and the
                 constraint projection, and the backtracking step (Sec. 4.3,
                 4.4, App. B.3.3-B.3.4).
``obstacle``     sphere-obstacle surface potential in closed form (Sec. 7.1).
``penalties``    total-length, length-difference and field penalties (Sec. 7.1).
``ccd``          first collision time of a curve moving along a direction
                 (Sec. 4.4, time stepping).
``learned``      the learned multigrid smoother weights: network, features,
                 targets and loss (not in the paper; its hierarchy follows
                 App. B.3.1-B.3.2).
"""
