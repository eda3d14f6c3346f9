"""Pins of the reference velocity autocorrelation curves (tests/vacf_theory.py)
against closed forms that do not go through their quadratures: the
incompressible limit of the translational friction, causality of the
one-sided transform, the Green-Kubo sum rules (Stokes-Einstein translational
and rotational friction), the hydrodynamic long-time tail and the rotational
initial value."""
import math

import numpy as np
import pytest

import vacf_theory as V

R = 3.0
MS = 4.0 * math.pi * R ** 3 * V.RHO0 / 3.0
IS = 2.0 * MS * R * R / 5.0


def test_incompressible_limit_is_the_stokes_boussinesq_friction():
    w = np.array([1e-3, 0.3, 2.0, 50.0])
    x = R * np.sqrt(-1j * w / V.NU0)
    ref = 6.0 * math.pi * V.ETA0 * R * (1.0 + x + x * x / 9.0)
    assert np.abs(V.gamma_t(w, R, c0=1e9) / ref - 1.0).max() < 1e-10
    assert abs(V.gamma_t(np.array([1e-9]), R)[0] / (6.0 * math.pi * V.ETA0 * R) - 1.0) < 1e-3


def test_translational_curve_is_causal_and_obeys_the_sum_rule():
    neg = V.ct_theory([-0.5, -2.0, -5.0], R)
    assert np.abs(neg).max() < 1e-5  # nothing before t = 0 (C_T(0+) ~ 5e-3)
    tt = np.concatenate([np.linspace(0.0, 10.0, 201)[1:], np.linspace(10.0, 300.0, 146)[1:]])
    c = V.ct_theory(tt, R)
    c0p = 2.0 * V.ct_theory([0.0], R)[0]  # the one-sided transform gives C(0+)/2 at 0
    tail = 1.0 / (4.0 * V.RHO0 * (math.pi * V.NU0) ** 1.5)
    integral = np.trapezoid(np.concatenate([[c0p], c]), np.concatenate([[0.0], tt])) + 2.0 * tail / math.sqrt(tt[-1])
    assert integral == pytest.approx(3.0 / (6.0 * math.pi * V.ETA0 * R), rel=5e-3)  # 3 D, Stokes-Einstein
    # long-time tail kT / (4 rho (pi nu t)^{3/2}) (three components)
    for t in (200.0, 300.0):
        assert V.ct_theory([t], R)[0] == pytest.approx(tail * t ** -1.5, rel=0.05)


def test_rotational_curve_initial_value_and_sum_rule():
    c = V.cr_theory([1e-6], R)[0]
    assert c == pytest.approx(3.0 / IS, rel=0.02)
    tr = np.concatenate([np.linspace(0.0, 5.0, 101)[1:], np.linspace(5.0, 100.0, 96)[1:]])
    cr = V.cr_theory(tr, R)
    integral = np.trapezoid(np.concatenate([[3.0 / IS], cr]), np.concatenate([[0.0], tr]))
    assert integral == pytest.approx(3.0 / (8.0 * math.pi * V.ETA0 * R ** 3), rel=0.01)
