"""MI355X-native electrostatic potential of a QM/MM environment.

V(r) = sum_A Z_A/|r - R_A| - sum_{mu nu} P_{mu nu} [mu nu | r], evaluated at
QMC electron positions by hand-written HIP kernels for gfx950 behind a C ABI
(``include/env_potential.h``).  The sub-modules are imported lazily so that
the input generator (``synth``) can be used without loading the native
library.
"""
__all__ = ["synth", "envpot"]
