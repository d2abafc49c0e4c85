"""Plain FP64 CPU oracle of the moment-fitting Vlasov hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

Every function follows one passage of the paper (arXiv 2109.06743, "An Energy
Conserving Vlasov Solver That Tolerates Coarse Velocity Space Resolutions")
or of a scheme the paper names (the PFC scheme, CWENO-3, SSP-RK3, Yee FDTD),
and says which.  Where the paper is silent the reading used is stated in the
docstring.  The code is deliberately slow and literal: flux sums are written
as sums, limiters in their ratio form, moments as explicit quadratures.
"""
