"""FP64 CPU reference for regularized dipole sums (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it and shares no code
with it.  See ``dps_oracle.c`` for what is computed and which passage of the
paper each part follows.
"""
from .oracle import (  # noqa: F401
    build, load, direct, direct_adjoint, Tree, rho, psi, rho_series,
    psi_series, rho_closed, radial, chi, chi_series, radial_nu, radial_eps, direct_mono,
    direct_mono_adjoint, round_bf16, STORAGE_MODES,
)
from . import rays  # noqa: F401,E402
