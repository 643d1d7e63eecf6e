"""Plain FP64 CPU oracle for the geometry-split ARK-IMEX DG / HDG scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP path: it reads the
seeded workload description and nothing else from the package.

It follows the paper (Ellmenreich, Shehadi, Lederer, "IMEX Schemes for
Compressible Flow using Hybridizable Discontinuous Galerkin Methods") term by
term, with full (not sum-factorised) interpolation matrices, Jacobians by the
complex-step method and a monolithic sparse direct solve of each Newton step.

Modules
-------
basis    Gauss-Legendre quadrature, nodal Q^k basis, element matrices (Sec. 3.1, Sec. 5)
mesh     tensor-product meshes, facet tables, the implicit/explicit split (Sec. 3.1, Sec. 4)
physics  fluxes, quasi-linear viscous flux, characteristic splitting, numerical fluxes (Sec. 2, 3.2-3.5, App. A-B)
dg       explicit DG-IP residual incl. interface and far-field terms (Sec. 3.3, 4.1.1, App. B.1)
hdg      HDG-IP / HDG-MX stage system and its Newton solve (Sec. 3.4, 3.5, 4.1.2, 4.3, App. B.2-B.3)
ark      ARS tableaux and the IMEX step (Sec. 4.2, App. C)

Parity status: every function is pinned by tests under ``tests/test_oracle_*``
except the absolute field values of the synthetic workloads, which the paper
does not print (those are pinned only through invariants and limits).
"""
