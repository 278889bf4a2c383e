"""Pins of the complex-step build of the oracle (the FP64 reference gradient of the adjoint).

The same C source compiled with a complex scalar type gives dJ/dtheta = Im J(theta + i h)/h
for J = D_o + D_i / 2 after a few coupled steps.  Pinned here against things other than
itself: the real oracle's value of J, Richardson-extrapolated central differences of the
real oracle (an independent way to the same derivative, whose own error is its rounding),
the exact zeros at H0 = 0 (the Kelvin force is quadratic in H0, so neither H0 nor the field
angle can move J there), and the independence of the result from h.
"""
import math

import numpy as np
import pytest

from fcd_inputs import Workload, channel_drive, h0_from_bond
from oracle import OracleSim
from oracle.oracle import THETA_NAMES, complex_step_gradient, complex_step_run

NSTEPS = 10
W = (1.0, 0.5)


def small(H0=None):
    """48 x 16 channel, ferrofluid shell, three different surface tensions, field at 30 deg."""
    ny, tau3, u = 16, 0.8, 0.01
    s12, s13, s23 = 0.008, 0.012, 0.01
    rc, rs = 3.0, 6.0
    h0 = h0_from_bond(1.0, "shell", 1.0, rc, rs, s12, s23) if H0 is None else H0
    return Workload(name="cs_48x16", nx=48, ny=ny, tau=(tau3, tau3, tau3), chi=(0.0, 1.0, 0.0),
                    sigma12=s12, sigma13=s13, sigma23=s23, xi=4.0, H0=h0, alpha=math.radians(30.0),
                    drive_G=channel_drive(u, 1.0, tau3, ny), xc=20.0, yc=7.3, r_core=rc, r_shell=rs, u_ref=u)


def real_J(w, theta):
    H0, alpha, u, s12, s13, s23 = theta
    ww = w.replace(H0=H0, alpha=alpha, u_ref=u, sigma12=s12, sigma13=s13, sigma23=s23,
                   drive_G=channel_drive(u, w.rho[2], w.tau[2], w.ny))
    s = OracleSim(ww)
    s.init_droplet(solve=False)
    assert s.step(NSTEPS) == 0
    d = s.diagnostics()
    return W[0] * d[0] + W[1] * d[1]


def theta_of(w):
    return [getattr(w, n) for n in THETA_NAMES]


@pytest.fixture(scope="module")
def cs():
    w = small()
    J, g = complex_step_gradient(w, NSTEPS, W)
    return w, J, g


def test_real_part_is_the_real_oracle(cs):
    w, J, _ = cs
    J_real = real_J(w, theta_of(w))
    # complex quotients round their real part differently from real ones
    assert abs(J - J_real) <= 1e-13 * abs(J_real), (J, J_real)


def test_matches_richardson_central_differences_of_the_real_oracle(cs):
    w, J, g = cs
    th = theta_of(w)
    for k in range(6):
        h = 1e-3 * abs(th[k])

        def cd(hh):
            tp, tm = list(th), list(th)
            tp[k] += hh
            tm[k] -= hh
            return (real_J(w, tp) - real_J(w, tm)) / (2 * hh)

        fd = (4 * cd(h / 2) - cd(h)) / 3
        # the difference quotient's own error is rounding: a few hundred ulps of J over
        # 2h, largest relative to the smallest sensitivity (u_ref: 2e-7 measured)
        assert abs(g[k] - fd) <= 1e-6 * abs(fd) + 1e-9 * abs(J), (THETA_NAMES[k], g[k], fd)


def test_zero_field_gradients_are_exactly_zero():
    w = small(H0=0.0)
    J, g = complex_step_gradient(w, NSTEPS, W)
    assert g[0] == 0.0 and g[1] == 0.0
    assert np.all(g[2:] != 0.0)


def test_independent_of_the_step():
    """Im J(theta + i h)/h carries no difference of nearby values, so h from 1e-12 to
    1e-100 gives the same derivative to rounding (its second-order error is h^2)."""
    w = small()
    k = THETA_NAMES.index("sigma23")
    vals = []
    for h in (1e-12, 1e-20, 1e-100):
        d = complex_step_run(w, NSTEPS, k, h)
        vals.append((W[0] * d[0] + W[1] * d[1]).imag / h)
    assert max(vals) - min(vals) <= 1e-12 * abs(vals[0]), vals
