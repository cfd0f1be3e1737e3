"""CPU oracle for LU_PRRP and CALU_PRRP -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy implementation of what the GPU library computes,
written from the paper (Khabou, Demmel, Grigori, Gu, "LU factorization with
panel rank revealing pivoting and its communication avoiding version").  It
shares no code with the HIP path and is never called by the product: only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark import
it.

Modules
  rules    -- the deterministic tie rule used for every pivot decision
  srrqr    -- QR with column pivoting of a panel's transpose and the strong
              RRQR exchange loop (Appendix A, Algorithm "Strong RRQR")
  lu       -- GEPP, LU_PRRP (Section 2.1, Algorithm "LU_PRRP factorization")
              and CALU_PRRP (Section 3.1, tournament pivoting)
  block_lu -- block parallel and block pairwise LU_PRRP (Section 5,
              Appendix E): an update at every tree node, and their solve
  solve    -- triangular solves and iterative refinement with an exactly
              rounded residual
  metrics  -- growth factors, backward errors, HPL tests, growth bounds and
              flop counts

Every function names the passage it follows.  Parity status of each function
is listed in the module docstrings; all functions are pinned by the CPU tests
under tests/ (no function is "parity unpinned").
"""
from . import rules, srrqr, lu, block_lu, solve, metrics  # noqa: F401
