"""Plain CPU FP64 oracle for the polynomial-filtered interior eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package; only the test-suite, the smoke check of the
entry module and the CPU-baseline leg of the benchmark use it.  It shares no
code with the HIP library: it is written directly from the paper
(Accaputo, Derlet, Arbenz, "Solving large-scale interior eigenvalue problems
to investigate the vibrational properties of the boson peak regime in
amorphous materials", 2019) with numpy/scipy/LAPACK as the only primitives,
plus one plain C loop (cbsr.c) for the block-sparse product at large sizes.

Modules
-------
hessian     mass weighting H_ij = K_ij / sqrt(m_i m_j) (Sec. 1, eq. intro.2)
filters     piecewise-quadratic target p (Sec. 2.6, eq. fct_f), its Chebyshev
            coefficients by the exact integrals of Appendix A, Jackson and
            Lanczos damping (Sec. 2.3), the degree rule (eq. thresh), the
            Dirac-delta filter (Sec. 2.5, eq. cheby-delta.1)
chebyshev   Algorithm 2, y = p_d(H) x by the three-term recurrence
lanczos     a few Lanczos steps for the extremal-eigenvalue bounds (Alg. 3)
cbsr        H @ X by the textbook block-CSR loop in C (OpenMP over rows), a
            drop-in for the scipy matrix when n is in the hundreds of thousands
dense       the plain definition: all eigenpairs of H in a closed window
subspace    filtered subspace iteration with Rayleigh-Ritz (Alg. 4, adapted)
count       stochastic trace estimate of the eigenvalue count (eq.
            eigval_count_estimator)
adjoint     reverse-mode derivative of y = p_d(H) x (no counterpart in the
            paper; defined from Algorithm 2 by the chain rule)
"""
