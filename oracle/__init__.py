"""FP64 CPU oracle for SH soft-shadow visibility and shading.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path (the
HIP library and its Python binding) never does, and shares no code, tables or
constants with it.

The oracle is a plain, slow, step-by-step restatement of the method of
"Efficient and Differentiable Shadow Computation for Inverse Problems"
(Lyu et al., ICCV 2021), written in torch float64 on the CPU so that gradients
come from autograd rather than from a hand-derived adjoint:

  sh        real orthonormal SH basis, Legendre polynomials, Funk-Hecke
            coefficients, exact spherical quadrature, the triple-product
            tensor C_ijk (Sec. 3.2, Eqs. 3-7)
  method    pair geometry -> log-cap zonal coefficients -> rotation -> sum
            over spheres -> SH exponential -> clamped-cosine transfer ->
            shading (Sec. 3.3.2, Eqs. 8, 10-13), and its gradients
  brute     reference integrals used only to pin the above (Eq. 2 with the
            binary blocker function, exact function-space exponential)
  deform    the scene parameterisation upstream of the spheres: rigid pose
            and embedded deformation driven by the spheres (Sec. 3.3.1,
            Sec. 3.5)
"""
from . import sh, method, brute, deform  # noqa: F401
