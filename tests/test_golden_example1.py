"""Pins against the numbers the manual prints for its first worked example
(infrared FEL; ch. 5 "Examples", table "example1"), stored in
tests/golden/example1_infrared_fel.txt.

The oracle's frame constants must reproduce the printed radiation
wavelength (resonance of the boosted frame, sec. "Lorentz Transformation")
and its undulator field the printed peak field (sec. "Static Undulator
Field"); the 1-D FEL parameter used to size the synthetic bunches must
reproduce the printed FEL parameter, gain length and cooperation length.
The table's own internal consistency (density, current) is checked first,
so that a mistyped fixture fails here rather than in a physics pin."""
import math
import os

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2009_13645_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
MC2_EV = 0.51099895e6


def golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "example1_infrared_fel.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, value, _unit = line.split()
        out[name] = float(value)
    return out


G = golden()
GAMMA = G["bunch_energy"] / MC2_EV  # total energy over rest energy


def test_fixture_is_self_consistent():
    vol = G["bunch_size_x"] * G["bunch_size_y"] * G["bunch_size_z"]
    n_e = G["bunch_charge"] / W.Q_E / vol
    assert n_e == pytest.approx(G["electron_density"], rel=0.01)
    current = G["bunch_charge"] * W.C_LIGHT / G["bunch_size_z"]
    assert current == pytest.approx(G["bunch_current"], rel=0.01)


def example1_oracle():
    """A small oracle run with the example's undulator and beam energy."""
    w = W.Workload(name="example1-frame", nx=8, ny=8, nz=16, gamma=GAMMA, K=G["undulator_parameter"],
                   lambda_u=G["undulator_period"], n_periods=10, und_type=W.PLANAR, n_particles=1,
                   sigma_cells=(1.0, 1.0, 1.0), seed=3, tile=(4, 4, 4))
    return w, Oracle(w.descriptor())


def test_oracle_resonance_matches_printed_radiation_wavelength():
    w, o = example1_oracle()
    c = o.consts()
    g0, b0 = c["gamma0"], c["beta0"]
    lam_star = G["undulator_period"] / (g0 * b0)       # boosted-frame undulator period
    lam_lab = lam_star / (g0 * (1.0 + b0))            # Doppler back to the lab
    o.close()
    assert lam_lab == pytest.approx(G["radiation_wavelength"], rel=0.03)


def test_oracle_undulator_peak_field_matches_printed_field():
    w, o = example1_oracle()
    c = o.consts()
    g0, b0 = c["gamma0"], c["beta0"]
    d = w.descriptor()
    ku = 2.0 * math.pi / d["lambda_u"]
    # on axis, a quarter period inside the entrance at t = 0: sin(ku z') = 1
    zq = d["z_entrance"] + (0.25 * d["lambda_u"] + 3 * d["lambda_u"]) / g0
    E, B = o.external_field(np.array([0.0, 0.0, zq]), 0.0)
    o.close()
    # boosted B_y = gamma0 B'_y (sec. "Lorentz Transformation", E' = 0)
    assert B[1] / g0 == pytest.approx(G["undulator_field"], rel=0.01)
    assert E[0] == pytest.approx(-g0 * b0 * W.C_LIGHT * B[1] / g0, rel=1e-12)


def test_fel_parameter_gain_and_cooperation_lengths():
    rho = W.fel_rho_1d(GAMMA, G["undulator_parameter"], G["undulator_period"], G["electron_density"],
                       helical=False)
    assert rho == pytest.approx(G["fel_parameter"], rel=0.1)
    lg = G["undulator_period"] / (4.0 * math.pi * math.sqrt(3.0) * rho)
    assert lg == pytest.approx(G["gain_length_1d"], rel=0.05)
    lc = G["radiation_wavelength"] / (4.0 * math.pi * rho)
    assert lc == pytest.approx(G["cooperation_length"], rel=0.1)
