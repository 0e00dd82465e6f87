"""CPU FP64 oracle for the upwind-SBP elastic solver (Duru, Fung & Williams,
arXiv:2011.02600).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code, tables or
constant generators with the HIP library: it derives its own SBP operators
(exact rational arithmetic), its own metric terms and its own SAT terms from
the paper, and it is deliberately plain and slow (dense 1D operators applied
along each axis with a matrix product, float64 everywhere).

Modules
-------
sbp_operators  upwind diagonal-norm dual-pair SBP operators (Sec. 4.1,
               Definition of the dual pair, eq. upw_SBP/acc, Table tab:upwind)
lsrk           five-stage 2N-storage fourth-order Runge-Kutta (Sec. 7 uses
               Carpenter & Kennedy 1994)
elastic        metric terms, material, semi-discrete RHS (eq.
               gen_hyp_transformed_discrete_SAT), SAT terms (eq.
               SAT_free_surface, eq. SAT_General with App. A hat variables),
               point source (eq. momententor_pointsource), discrete energy,
               time stepping and receiver recording
kron_form      the same semi-discrete operator assembled literally as sparse
               Kronecker products with the rotated (n, m, l) boundary frame;
               used only as a brute-force pin of ``elastic`` on tiny grids
adjoint        discrete adjoint of the fully discrete scheme (explicit sparse
               transpose of ``kron_form``'s operator, reverse Runge-Kutta
               sweep) and the misfit gradient with respect to the nodal
               rho, lambda, mu (complex-step derivatives of ``elastic.rhs``);
               an extension, not in the paper

Array convention: every grid function is a numpy array of shape (ns, nr, nq)
(C order, q fastest), so the q-derivative acts on axis 2, r on axis 1 and s
on axis 0.  The nine fields are ordered (vx, vy, vz, sxx, syy, szz, sxy, sxz,
syz) as in eq. elastic_sys.
"""
