"""Plain, slow, obviously-correct FP64 CPU oracle for sketch-preconditioned least squares
(Lacotte & Pilanci, "Faster Least Squares Optimization", arXiv 1911.02675).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it.  The GPU library never calls into it and shares no code,
header, table or constant generator with it: both sides implement the random draws from the
published Philox definition and the sketch/solver definitions from the paper independently.

Modules
  philox      Philox4x64-10 counter-based generator (Salmon et al., SC'11), plain uint64 numpy.
  draws       the draw specification: SRHT signs and row subset, SJLT targets/signs, Gaussian entries.
  sketch      explicit S (or S@A) for the SRHT, SJLT and Gaussian embeddings (Section 2).
  householder Householder QR and triangular back-substitution (textbook, Golub & Van Loan 5.2).
  solve       direct least-squares solve, error metrics.
  pcg         PCG with a fixed sketch preconditioner (Section 1.2).
  ihs         IHS / Polyak-IHS with fixed or refreshed sketches (Section 1.1).
  theory      inverse moments theta_1, theta_2 (Section 2), closed-form expected errors
              (Theorems 3.3, 4.1, the Polyak-IHS moment recursion in the proof of Theorem 4.3),
              the PCG extreme-eigenvalue bound (Section 3.1).
"""
