"""Physical constants in the paper's normalised units (test infrastructure only).

Units: time in 1/omega_0, length in c/omega_0, momentum in m_e c, fields in
m_e c omega_0 / e (the normalisation the paper states below Eqs. (2)-(3)).

E_S   The Schwinger field in those units is m_e c^2 / (hbar omega_0), which depends
      on the laser wavelength.  The paper gives no wavelength; its Fig. 1 triples
      (b0, gamma_e, chi_e) = (200, 206, 0.1), (2000, 206, 1), (2000, 2060, 10) force
      E_S ~ gamma * b0 / chi ~ 4.12e5, which is the value at lambda_0 = 1 um.
ALPHA The fine-structure constant; the paper writes alpha ~ 1/137 (text under
      Eq. 1).  CODATA 2018 is used.

Pinned by: tests/test_oracle_pins.py::test_fig1_triples (the Fig. 1 triples give
chi within 0.04 % of the paper's 0.1 / 1 / 10).
"""
import math

M_E_C2_EV = 510998.95                 # electron rest energy [eV], CODATA 2018
HC_EV_UM = 1.239841984                # h c [eV um], CODATA 2018
LAMBDA0_UM = 1.0                      # laser wavelength implied by Fig. 1
E_S = M_E_C2_EV / (HC_EV_UM / LAMBDA0_UM)   # Schwinger field, m_e c omega_0 / e
ALPHA = 1.0 / 137.035999084           # fine-structure constant
RATE_UNIT = ALPHA * E_S               # alpha m_e c^2 / hbar in units of omega_0

# Thresholds of the method.
PHOTON_XI_MIN_GAMMA = 2.0   # infrared cutoff: xi_min * eps_e = 2 m_e c^2 (text under Eq. 7)
PAIR_GAMMA_MIN = 2.0        # a photon below 2 m_e c^2 cannot make a pair

GAMMA_2_3 = math.gamma(2.0 / 3.0)
