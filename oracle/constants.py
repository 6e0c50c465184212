"""Free-space constants (SI) and the harmonic time convention.

Time dependence e^{j w t}, so the Green's function of eq. (3) is taken as
G = exp(-j k R) / (4 pi R).  (The printed eq. (3) has exp(+jkR) together with a
"+ j/(w eps)" scalar term in eq. (2); the two signs do not belong to one
convention.  Magnitudes |x| and the RCS do not depend on the choice.)
"""

import math

C0 = 299792458.0                 # speed of light, m/s
MU0 = 4.0e-7 * math.pi           # permeability, H/m
EPS0 = 1.0 / (MU0 * C0 * C0)     # permittivity, F/m
ETA0 = MU0 * C0                  # free-space impedance, ohm


def wavenumber(freq_hz):
    return 2.0 * math.pi * freq_hz / C0


def omega(freq_hz):
    return 2.0 * math.pi * freq_hz
