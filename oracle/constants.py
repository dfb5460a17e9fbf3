"""Physical constants in SI units.

The speed of light and the elementary charge are exact in the 2019 SI; the vacuum
permittivity is the CODATA 2018 recommended value.
"""
C_LIGHT = 299792458.0            # m/s (exact)
E_CHARGE = 1.602176634e-19       # C   (exact)
EPS0 = 8.8541878128e-12          # F/m (CODATA 2018)
