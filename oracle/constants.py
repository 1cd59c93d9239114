"""Physical constants in CGS units (CODATA 2018 exact or recommended values).

Part of the test-only oracle.  Derived constants are computed here, never
typed in, so that a test can compare them against textbook values.
"""
import math

C_LIGHT = 2.99792458e10            # cm s^-1 (exact)
H_PLANCK = 6.62607015e-27          # erg s (exact)
K_BOLTZ = 1.380649e-16             # erg K^-1 (exact)
E_CHARGE = 1.602176634e-19 * 2.99792458e9   # statC: e[C] * c[m/s] * 10 (exact)
M_ELECTRON = 9.1093837015e-28      # g
AMU = 1.66053906660e-24            # g
EV = 1.602176634e-12               # erg (exact)
M_HYDROGEN_AMU = 1.008             # standard atomic weight of H
CHI_HYDROGEN_EV = 13.598434599702  # ionisation energy of H I (NIST ASD)
U_HYDROGEN = (2.0, 1.0)            # partition functions of H I (ground state) and H II

#: pi e^2 / (m_e c): integrated cross-section per oscillator [cm^2 s^-1]
PI_E2_MC = math.pi * E_CHARGE ** 2 / (M_ELECTRON * C_LIGHT)
#: (2 pi m_e k / h^2)^(3/2): Saha constant [cm^-3 K^-3/2]
SAHA_CONST = (2.0 * math.pi * M_ELECTRON * K_BOLTZ / H_PLANCK ** 2) ** 1.5
#: h c / k with lambda in nm [nm K]
HC_K_NM = H_PLANCK * C_LIGHT / K_BOLTZ * 1e7
