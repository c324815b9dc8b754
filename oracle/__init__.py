"""FP64 / exact-integer CPU oracle for the Polya interior-point method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

Written from the paper (Kamyar, Peet & Peet, "Solving Large-Scale Robust
Stability Problems by Exploiting the Parallel Structure of Polya's Theorem",
IEEE TAC 2013):

* ``polya``  exponent sets, lexicographic index, the beta and H coefficient
  recursions of Section III-A (eq. beta_init/beta, H_init/H), their closed
  forms and a brute-force polynomial expansion, homogenisation (Section II).
* ``sdp``    the SDP elements C, B_i, a of Section III-B (eq. C, Cj, K, Ai,
  Aij, a), the operators B and B^T (eq. AT), dense materialisation for tiny
  cases, and the Schur complement (Alg. 2, eq. T2) in definition and
  expanded form.
* ``ipm``    the predictor-corrector primal-dual method of Section IV-A and
  Alg. 2 with the readings listed in the design notes, the line-search
  ladder, the certificate check, the Farkas ray rule and the phase-I margin
  SDP; plus a dense textbook primal-dual solver used to check Theorem 3.
* ``stability``  the homogeneous representation of A on a translated
  simplex (Section II and the regions of Section V, Examples 1 and 2) and
  the bisection over the region's size; a brute-force spectral boundary.
* ``discrete``  the discrete-time form (x+ = A(alpha) x) as an instance of
  the generalized LMI of Section III-C: 2n x 2n derivative blocks
  [[b P, P H], [H^T P, b P]] with basis matrices blockdiag(E_b, E_b).
* ``mlp``    the FP64 network of the learned warm start.

Parity pins live under ``tests/`` (marker ``not gpu``).  Functions whose
result is not pinned by an independent fact say so in their docstring
("parity unpinned").
"""
