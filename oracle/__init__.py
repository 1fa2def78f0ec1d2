"""Plain FP64 CPU oracle for the preconditioned GLBE with forcing and the
preconditioned vector lattice kinetic equation (LKE) for magnetic induction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table
or helper with the HIP library; the two meet only through seeded inputs.

The oracle is deliberately slow and literal:

* the moment transform is the dense 19x19 matrix built from the row polynomials
  of the orthogonal D3Q19 basis and applied with a matrix product; its inverse
  is ``numpy.linalg.inv`` (orthogonality is a tested property, not an
  assumption);
* equilibrium moments and moment-space sources are written out as the paper
  lists them (Sec. 3, D3Q19 preconditioned equilibria and sources; App. A);
* streaming is ``numpy.roll`` plus halfway bounce-back substitution;
* the implicit Lorentz-force coupling is solved as a plain 3x3 linear system
  per node with ``numpy.linalg.solve``.

Every array routine accepts complex128 as well as float64 so that complex-step
derivatives of the whole time march can be taken (no ``abs``, ``max`` or
comparisons on state values inside a step).

Modules
-------
lattice  D3Q19 / D3Q7 velocity sets, weights, moment basis (Sec. 2, Sec. 4, App. A)
glbe     preconditioned GLBE collide/stream step, fields, residual (Sec. 2-3, Sec. 5)
mhd      preconditioned vector LKE with chi-scaling and Lorentz coupling (Sec. 4, 4.1)
adjoint  complex-step and dense-Jacobian gradients of the steady flow rate
rounding stochastic rounding to BF16 with counter-based random bits (a storage
         option of the library, not part of the paper)
"""
