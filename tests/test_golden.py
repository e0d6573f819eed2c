"""Numbers the paper prints, recomputed from the definitions the oracle and the input
generator use (tests/golden/paper_printed_values.json holds them with their places in the
paper).  Physical constants: k_B = 1.380649e-23 J/K (exact, SI 2019), argon atomic mass
39.948 u, u = 1.66053906660e-27 kg.  CPU only."""
import json
import math
import os

import numpy as np

from oracle import closure, moments as mo, scheme as sc

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'paper_printed_values.json')))
KB = 1.380649e-23
M_AR = 39.948 * 1.66053906660e-27


def test_jet_speed_from_the_mach_definition():
    """The oracle's jet Maxwellian (|u| = M sqrt(5/3 T) with the gas constant absorbed) in
    SI units for argon at 300 K."""
    g = GOLDEN['jet_speed_m_s']
    T_nd = KB * g['inputs']['T_K'] / M_AR            # k T / m in m^2/s^2
    W = sc.jet_prim(sc.Setup(jet_mach=g['inputs']['mach'], jet_T=T_nd), 0.0)
    speed = float(np.hypot(W[1], W[2]))
    assert abs(speed - g['value']) < 0.5, speed      # printed to 4 digits


def _jet_density(d):
    n = 1.0 / (math.sqrt(2.0) * d['sigma_m2'] * d['kn'] * d['L_jet_m'])
    return n * M_AR


def test_jet_density_from_the_knudsen_definition():
    for key in ('jet_density_kn1_kg_m3', 'jet_density_euler_appendix_kg_m3'):
        g = GOLDEN[key]
        rho = _jet_density(g['inputs'])
        assert abs(rho / g['value'] - 1.0) < 5e-3, (key, rho)   # printed to 3 digits


def test_equilibrium_fourth_moment():
    g = GOLDEN['equilibrium_R_coefficient']
    rho, p = np.array([0.7, 2.0]), np.array([1.3, 0.4])
    W = mo.maxwellian_prim14(rho, np.zeros((2, 3)), p)
    assert np.allclose(W[13] * rho / p**2, g['value'], rtol=1e-15)
    # the dimensionless form the closure sees
    Rs = closure.nondim14(W)[6]
    assert np.allclose(Rs, g['value'], rtol=1e-14)
