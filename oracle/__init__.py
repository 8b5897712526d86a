"""Plain FP64 CPU oracle for the channel-flow DNS step (TEST INFRASTRUCTURE).

This package is the reference that the HIP path is checked against.  It is
slow on purpose: dense Chebyshev matrices, ``numpy.fft`` on the padded grid
and batched LAPACK solves of the dense tau systems, written in the order in
which the method is described, with no blocking or fusion.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product library never calls it and shares no
code with it.

Method (Guastoni et al., "Deep reinforcement learning for turbulent drag
reduction in channel flows"):

* §3.1 "Simulation setup": Fourier (x, z) x Chebyshev (y) pseudo-spectral DNS
  of incompressible channel flow, grids N_x x N_y x N_z with N_y Chebyshev
  modes, Crank--Nicolson for the linear terms and third-order Runge--Kutta for
  the non-linear terms.  The paper only cites its solver; the velocity--
  vorticity form, the influence-matrix wall correction and the three-stage
  low-storage RK3/CN coefficients are the standard published choices
  (Kim, Moin & Moser 1987; Spalart, Moser & Rogers 1991), written out in
  ``channel.py``.
* §3.2 "Reinforcement-learning environment and algorithm": wall-normal
  blowing/suction as the control, a linear ramp from the old to the new
  action over the actuation interval, clipping to [-u_tau, u_tau], an
  observation plane at a height rounded up to a Chebyshev node, and a reward
  built from the wall-shear stress averaged between two actions.
* §4.1 "Validation and baseline": opposition control, v_w = -alpha (v(y_s) -
  <v(y_s)>), zero net mass flux.

Parity status of each function is stated in its docstring; functions whose
result is pinned by a test against an independent fact say which test.
"""
