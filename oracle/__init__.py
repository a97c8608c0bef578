"""FP64 CPU oracle of the level-set LLG forward/adjoint path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
package: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; the two meet only
through the seeded input arrays of ``paper_2411_19109_amd.workloads`` (which
holds no arithmetic of the method).

Plain, slow, obviously-correct NumPy in float64.  Every function accepts
complex arrays too, so that complex-step differentiation can pin the adjoint
against the forward map to machine precision.

Modules
  newell     cell-averaged demagnetisation tensor (Newell closed form near,
             Gauss-Legendre quadrature of the tent-weighted dipole kernel far)
  micromag   effective field, LLG right-hand side, RK4, energies
  adjoint    discrete adjoint of the RK4 map, objectives (energy + area, port
             m_y^2, spectral port, magnetisation curve) and gradients
  levelset   smoothed Heaviside map phi -> psi and its derivative
  rbf        RBF cones and their p-norm level set (amplitudes -> phi), its
             vector-Jacobian product, and the Adam update of the amplitudes
  shape      size and centre-of-mass constraints of the regularised objective
  dopri      adaptive Dormand-Prince 5(4) integration and the adjoint of its
             accepted steps
  continuous the continuous adjoint (the adjoint equation integrated backwards
             on the kept forward states), for comparison with the discrete one
"""
