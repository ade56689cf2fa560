"""Physical constants (SI) and the time convention.

Time dependence exp(+j w t); the free-space Green's function is
G(R) = exp(-j k R) / (4 pi R). Test infrastructure only.
"""

import math

C0 = 299_792_458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = MU0 * C0


def wavenumber(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz / C0


def wavelength(freq_hz: float) -> float:
    return C0 / freq_hz
