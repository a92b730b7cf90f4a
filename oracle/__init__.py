"""Plain FP64 CPU oracle of the Heisenberg Lanczos hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
benchmark's cpu_baseline leg import this package.  It shares no code with the
HIP library (paper_0706_3293_amd): the count table, encoding, decoding,
successor and row-gather product live in oracle/oracle.c, written from Secs. 3
and 4 of the paper; the Lanczos recurrence, the tridiagonal eigensolve
(scipy), the stored-basis Ritz vector and the bond correlations live in
oracle/lanczos.py; magnetization sectors and thermodynamic sums live in
oracle/sectors.py, the block recurrence in oracle/block.py; oracle/brute.py holds independent brute-force references
used to pin the oracle.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  count_table        pinned: enumeration, closed form, paper's boundary values
  unrank/rank        pinned: enumeration, paper's worked encoding example
  successor          pinned: enumeration, paper's worked successor example
  apply/apply_rows   pinned: dense Kronecker Hamiltonian restricted to H(M)
  lanczos (E0)       pinned: dense eigenvalues, closed forms (dimer,
                     ferromagnet, complete graph, Majumdar-Ghosh ring)
  ground_state       pinned: dense eigenvector (|overlap| = 1), Marshall sign
  bond_correlations  pinned: dense <psi|s.s|psi>, finite differences, sum rule
  sector_energies    pinned: saturation closed form, one-magnon Laplacian
                     spectrum, SU(2) nesting of the sector spectra
  exact_thermodynamics  pinned: two-site closed form, full Kronecker spectrum
  ftl_thermodynamics pinned: exact with canonical start vectors, T -> infinity
                     sum rule, T -> 0 limit
  block_lanczos      pinned: p = 1 equals the scalar recurrence, lowest levels
                     (degenerate pairs included) equal the dense spectrum,
                     V^T V = I and V^T H V = T, full spectrum when exhausted
"""
from .core import Subspace, count, count_table, max_threads  # noqa: F401
from .lanczos import (bond_correlations, ground_state, lanczos,  # noqa: F401
                      ritz, ritz_all)
