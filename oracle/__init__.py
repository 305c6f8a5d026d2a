"""Plain FP64 CPU oracle for Levenberg-Marquardt bundle adjustment.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports this package;
only the test suite, the smoke check and the CPU-baseline leg of the benchmark
call it.  It shares no code with the HIP path: the GPU computes Jacobians in
closed form and solves the reduced camera system with preconditioned conjugate
gradients, while this oracle differentiates with forward-mode dual numbers and
solves the full damped normal equations exactly with a block Cholesky
factorisation.

Method (Graphite, arXiv 2509.26581):
  * objective: half the sum of robustified squared Mahalanobis residuals
    (Background, Eq. 1-2; Huber kernel Eq. 7);
  * LM step: (J^T W J + lambda D^T D) dx = -J^T W r with D^T D the clamped
    diagonal of J^T W J (Background, Eq. 4-6; Sec. IV-D diagonal clamp);
  * camera model: the BAL camera (the paper's BA benchmark, Sec. V), which the
    paper does not spell out; the reading used here is stated in camera.py.

Modules:
  dual      forward-mode dual numbers (Sec. IV-C idea, used on the CPU)
  camera    Rodrigues rotation and BAL projection
  robust    squared / Huber kernels and IRLS weights
  lm        generic LM loop (step acceptance, Nielsen damping update)
  ba        bundle-adjustment normal equations + block Cholesky solve
  pcg       preconditioned CG on the reduced camera system (Sec. IV-D stop rules)
  dense     dense generic least-squares problems (circle example, linear LS)
  align     similarity (Umeyama) alignment for gauge-free comparisons

Every function here is pinned by tests marked "not gpu" against closed forms,
library routines (scipy), brute-force dense algebra or finite differences.
"""
