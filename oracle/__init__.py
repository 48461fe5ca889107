"""Reference oracle for the matrix-free finite-strain tangent operator and its
geometric-multigrid preconditioned CG.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct CPU
finite-element code written from the paper (Davydov, Pelteret, Arndt,
Steinmann, "A matrix-free approach for finite-strain hyperelastic problems
using geometric multigrid").  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_1904_13131_amd``) never imports, links or calls anything here, and
nothing here imports the product path: the two share only the seeded input
generators in ``workloads``, which hold none of the method's arithmetic.

Everything is FP64.  The oracle assembles the sparse tangent in the
*referential* route (second Piola-Kirchhoff stress S and the referential
tangent C = 4 d2psi/dC2 of Sec. 2.3, chained through P = F S), which is a
different route from the spatial formulas (tau, J*c) the device kernels use,
so agreement also checks the paper's push-forward algebra.

Modules
-------
basis     1-D Gauss-Lobatto-Legendre support points, Gauss-Legendre rules,
          Lagrange bases (Sec. 5, tensor-product discussion).
material  compressible Neo-Hookean energy, S, referential tangent, tau, J*c
          (Sec. 2.3).
fe        structured Q_p lattice on the unit box, per-quadrature-point
          material ids, element residual and tangent, global CSR assembly,
          Dirichlet handling, sampled rows (Sec. 3, eq. mf_vmult in Sec. 5).
gmg       transfers, diagonal, Chebyshev smoother, Lanczos eigenvalue
          estimate, coarse LU solve, V-cycle, PCG (Sec. 6 and Sec. 7).
newton    Newton-Raphson load-stepping driver with cut-backs and a step
          length that keeps J > 0 (Sec. 3, Sec. 7).
spmv      OpenMP CSR product of the assembled tangent on all host cores
          (spmv.c, built by ``build()``): the matrix-based CPU baseline.
rng       the counter-based generator (SplitMix64) that both sides implement
          independently for the eigenvalue-estimate start vector.
"""
