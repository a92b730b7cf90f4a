"""MI355X-native Lanczos hot path for Heisenberg spin systems in H(M).

The product path is libhm.so (HIP kernels for gfx950 behind the C ABI in
include/hm.h); this package is its thin Python binding:

  Basis            subspace H(M), host/device encoding and decoding, H x,
                   Lanczos, ground-state recompute, bond correlations
  GroundStateEnergy  torch.autograd.Function for E0(J) with dE0/dJ = -<s.s>
  lanczos_batched  many instances and start vectors in one persistent launch
  magnetization_curve, ftl_thermodynamics
                   E0(M) over all sectors and finite-temperature Lanczos sums
"""
from .api import (Basis, LanczosResult, block_tridiag_eigenvalues, count,  # noqa: F401
                  last_timing, set_timing, tridiag_lowest, tridiag_ritz)
from .autograd import GroundStateEnergy, ground_state, ground_state_energy  # noqa: F401,E402
from .batched import BatchedProblem, BatchedResult, lanczos_batched  # noqa: F401,E402
from .sectors import (MagnetizationCurve, ftl_thermodynamics,  # noqa: F401,E402
                      magnetization_curve)
