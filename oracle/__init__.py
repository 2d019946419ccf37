"""Plain, slow FP64 CPU oracle of the SIMP compliance hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import anything in this package.  It shares
no code with the GPU library: it never imports ``paper_2005_05436_amd`` and the
library never imports it.  Every function follows one passage of
Ferrari & Sigmund, "A new generation 99 line Matlab code for compliance
Topology Optimization and its extension to 3D" (arXiv:2005.05436); the
passage is named in each docstring (equations numbered in order of appearance
as typeset: (1) projection, (2) filter, (6) SIMP, (7)-(8) sensitivities,
(9) projection derivative, (10)-(11) OC rule, (14) reduced index set,
(15) full-matrix recovery, (17) volume-preserving threshold, (18) its
derivative, (19) multiplier estimate).

Modules
  mesh        numbering, connectivity, loads, supports, initial design
  element     Q4 / Hex8 element stiffness by Gauss quadrature
  sparse      reduced index set, lower CSR pattern, permutation, assembly
  filt        cone density filter, forward and adjoint, both boundary rules
  projection  Heaviside projection, volume-preserving threshold by Newton
  solve       dense Cholesky (tiny meshes) and Jacobi-PCG (larger meshes)
  sensitivity element energies, compliance
  oc          optimality-criteria update with bisection on sqrt(lambda)
  continuation parameter continuation
  topopt      one redesign iteration and the whole loop
"""
