"""FP64 CPU oracle for the well-conditioned low-rank SDP interior-point method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under this package: only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with
the HIP library; the two are independent implementations of the same paper
(Chiu & Zhang, "Well-conditioned primal-dual interior-point method for
accurate low-rank semidefinite programming", arXiv 2407.14013).

Contents
--------
notation   svec / smat / Psi_n / symmetric Kronecker product (Notations).
operators  the constraint operator A and its adjoint (Introduction,
           eq. sdp-pd), dense and entry-sampling forms.
nt         Nesterov-Todd scaling (Introduction, eq. newt).
reform     the low-rank plus well-conditioned decomposition (Section 3,
           eq. EQSigdef), the augmented system and recovery (eq. augrec),
           the indefinite preconditioner (Section 6) and the matrix-free
           product formulas (Section 5).
krylov     PCG as in Definition pcg, the indefinite-preconditioned solve of
           Corollary pcg, and MINRES as in Corollary minres.
ipm        a plain primal-dual NT path-following IPM whose Newton systems
           are solved directly through the m x m Schur complement
           (the direct approach described in the Introduction).
certify    KKT certificate of a returned (X, y, S).
brute      tiny brute-force instances with closed-form or enumerated optima.

Parity status: every function listed above is pinned by the not-gpu tests
(tests/test_oracle_*.py) against identities, closed forms or brute force.
"""
