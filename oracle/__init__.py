"""Plain FP64 CPU oracle for recycled-Krylov hypergradient solves.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library and never imports it.

Every function follows the paper (Ehrhardt, Gazzola, Scott, "Efficient
gradient-based methods for bilevel learning via recycling Krylov subspaces",
arXiv 2412.08264) step by step in NumPy float64, favouring obviously-correct
code over speed.  Citations name the section / equation / algorithm.

Modules
  ops      forward operators: Gaussian blur A, forward differences D, filter correlations K
  problem  lower-level objectives (smoothed TV, fields-of-experts filters): Phi, grad, HVP, J
  lbfgs    L-BFGS lower-level solver
  krylov   plain CG, recycled CG (Galerkin counterpart of RMINRES), stop tests, reference solve
  rminres  RMINRES (Algorithm 3) with the explicit residual of Appendix A, stop tests
  recycle  orthonormalisation, projected GSVD (two routes), Ritz-GSV selection, refresh
  upper    gradient descent with backtracking (frozen-trajectory generator)
"""
