"""Plain, slow, FP64 CPU oracle of the wavelet-collocation vortex method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path; both sides see
only the seeded inputs of the `workloads` module.

Modules
  dd      exact DD subdivision weights and collocation-derivative filters
  mra     dyadic pyramid: forward / inverse transform, threshold, prolongation
  ops     collocation derivatives, Poisson solve, Smagorinsky viscosity,
          advection-diffusion residual and its Jacobian-vector product
  krylov  Arnoldi + phi_1 exponential step with regrid, diagnostics
  implicit  theta-scheme step by Newton iterations with GMRES
  scalar  passive scalar (vapor) transported by the vortex flow
  track   vortex centres and the convective time
  brute   pure-Python loop twins for tiny grids (used to pin the above)

Everything here follows the method of Walsh & Alam, "Fujiwhara interaction of
tropical cyclone scale vortices using a weighted residual collocation method"
(arXiv:1604.08159); each function cites the section or equation it follows.
Where the paper is silent the documented readings of the design notes apply.
"""
