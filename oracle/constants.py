"""Physical constants used by the oracle (SI).

mu0 is taken as exactly 4*pi*1e-7 T m/A (the paper gives no value); the
library uses the same definition so FP64 parity is not limited by a 5e-10
relative difference between conventions.
"""
import math

MU0 = 4.0e-7 * math.pi          # T m / A
MU_B = 9.2740100783e-24         # J / T
QE = 1.602176634e-19            # C
