"""Pins of the oracle's isotropic stencils (Eq. 34-35), permeability mixing (Eq. 8)
and magnetic-potential solve (Eq. 5-7)."""
import ctypes as C
import math

import numpy as np
import pytest

from fcd_inputs import Workload, random_phase_fields
from oracle.oracle import OracleSim, OracleSolver, lib, params_from_workload, ptr


def stencils(a):
    ny, nx = a.shape
    gx, gy, lap = np.zeros_like(a), np.zeros_like(a), np.zeros_like(a)
    lib().orc_stencils(nx, ny, ptr(np.ascontiguousarray(a)), ptr(gx), ptr(gy), ptr(lap))
    return gx, gy, lap


def test_stencils_exact_on_quadratics():
    ny, nx = 12, 16
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    c = [0.3, -1.2, 0.7, 0.05, -0.02, 0.11]
    a = c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    gx, gy, lap = stencils(a)
    sl = np.s_[1:-1, 1:-1]
    np.testing.assert_allclose(gx[sl], (c[1] + 2 * c[3] * x + c[4] * y)[sl], atol=1e-12)
    np.testing.assert_allclose(gy[sl], (c[2] + c[4] * x + 2 * c[5] * y)[sl], atol=1e-12)
    np.testing.assert_allclose(lap[sl], 2 * (c[3] + c[5]), atol=1e-12)


def test_stencils_on_periodic_wave():
    ny, nx = 6, 24
    k = 2 * math.pi * 3 / nx
    x = np.arange(nx, dtype=float)
    a = np.tile(np.sin(k * x), (ny, 1))
    gx, gy, lap = stencils(a)
    # central-difference closed forms, valid across the periodic seam too
    np.testing.assert_allclose(gx, np.tile(math.sin(k) * np.cos(k * x), (ny, 1)), atol=1e-14)
    np.testing.assert_allclose(lap, np.tile(2 * (math.cos(k) - 1) * np.sin(k * x), (ny, 1)), atol=1e-14)
    np.testing.assert_allclose(gy, 0.0, atol=1e-15)


def test_stencil_wall_rule_is_zero_normal_gradient():
    ny, nx = 8, 8
    prof = np.linspace(0.1, 0.9, ny) ** 2
    a = np.tile(prof[:, None], (1, nx))
    gx, gy, lap = stencils(a)
    # mirror ghost rows: the centred difference sees a(-1) = a(0) and a(ny) = a(ny-1)
    assert gy[0, 3] == pytest.approx((prof[1] - prof[0]) / 2, abs=1e-15)
    assert gy[-1, 3] == pytest.approx((prof[-1] - prof[-2]) / 2, abs=1e-15)
    assert lap[0, 3] == pytest.approx(prof[1] - prof[0], abs=1e-15)


def test_permeability_is_harmonic_mean():
    w = Workload(name="m", nx=4, ny=1, chi=(2.0, 1.0, 0.0))
    p = params_from_workload(w)
    phi1 = np.array([[1.0, 0.0, 0.5, 0.0]])
    phi2 = np.array([[0.0, 1.0, 0.0, 0.5]])
    mur = np.zeros_like(phi1)
    lib().orc_mu_r(p, ptr(phi1), ptr(phi2), ptr(mur))
    np.testing.assert_allclose(mur[0], [3.0, 2.0, 1.0 / (0.5 / 3 + 0.5), 1.0 / (0.5 / 2 + 0.5)], rtol=1e-15)


def apply_L(p, mur, u):
    out = np.zeros_like(u)
    lib().orc_apply_L(p, ptr(np.ascontiguousarray(mur)), ptr(np.ascontiguousarray(u)), ptr(out))
    return out


def test_operator_symmetric_negative_definite():
    ny, nx = 10, 14
    w = Workload(name="L", nx=nx, ny=ny)
    p = params_from_workload(w)
    rng = np.random.default_rng(5)
    mur = 1.0 + 2.0 * rng.random((ny, nx))
    u, v = rng.standard_normal((2, ny, nx))
    assert (v * apply_L(p, mur, u)).sum() == pytest.approx((u * apply_L(p, mur, v)).sum(), rel=1e-12)
    assert (u * apply_L(p, mur, u)).sum() < 0.0


def test_operator_constant_mu_is_scaled_eq35():
    ny, nx = 9, 12
    w = Workload(name="L", nx=nx, ny=ny)
    p = params_from_workload(w)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    u = 0.4 * x * x - 0.3 * x * y + 0.2 * y * y + x
    out = apply_L(p, np.full((ny, nx), 2.5), u)
    np.testing.assert_allclose(out[1:-1, 1:-1], 2.5 * 2 * (0.4 + 0.2), atol=1e-11)


def test_operator_converges_to_div_mu_grad():
    """Second-order consistency with div(mu grad u) (Eq. 6) for smooth mu and u."""
    errs = []
    for n in (32, 64):
        nx, ny = n, n
        w = Workload(name="L", nx=nx, ny=ny)
        p = params_from_workload(w)
        y, x = np.mgrid[0:ny, 0:nx].astype(float)
        kx, ky = 2 * math.pi / nx, math.pi / (ny + 1)
        u = np.sin(kx * x) * np.sin(ky * (y + 1))  # vanishes on the ghost rows
        mu = 1.5 + 0.5 * np.cos(kx * x + 0.3) * np.cos(ky * y)
        ux, uy = kx * np.cos(kx * x) * np.sin(ky * (y + 1)), ky * np.sin(kx * x) * np.cos(ky * (y + 1))
        mux = -0.5 * kx * np.sin(kx * x + 0.3) * np.cos(ky * y)
        muy = -0.5 * ky * np.cos(kx * x + 0.3) * np.sin(ky * y)
        exact = mu * (-(kx ** 2 + ky ** 2) * u) + mux * ux + muy * uy
        got = apply_L(p, mu, u)
        sl = np.s_[1:-1, :]
        errs.append(np.abs(got - exact)[sl].max() / np.abs(exact[sl]).max())
    assert errs[0] < 1e-2
    assert 3.5 < errs[0] / errs[1] < 4.5


def droplet_phi(nx, ny, a, xi):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    d = np.hypot(x - (nx - 1) / 2, y - (ny - 1) / 2)
    return 0.5 * (1 + np.tanh(2 * (a - d) / xi)), np.zeros((ny, nx))


def solve(p, phi1, phi2, solver=None, psi=None):
    psi = np.zeros_like(phi1) if psi is None else psi
    sw, res = C.c_int32(), C.c_double()
    rc = lib().orc_solve_potential_phi(p, ptr(phi1), ptr(phi2), solver or OracleSolver.direct(),
                                       ptr(psi), None, None, C.byref(sw), C.byref(res))
    assert rc == 0
    return psi, sw.value, res.value


@pytest.mark.parametrize("mu_in,a,xi", [(2.0, 8, 2.0), (2.0, 16, 2.0), (3.0, 8, 2.0), (3.0, 16, 2.0),
                                        (3.0, 16, 4.0)])
def test_permeable_cylinder_interior_field(mu_in, a, xi):
    """Interior field of a permeable cylinder in a uniform field: H = 2 H0/(1 + mu_r).
    The box is 8a wide, periodic in x with potential walls in y; the periodic and wall
    images raise the applied field by K pi^2 a^2/(2 L^2) to first order, K = (mu-1)/(mu+1).
    What is left is the O(xi/a) error of the diffuse interface."""
    L = 8 * a
    w = Workload(name="cyl", nx=L, ny=L, chi=(mu_in - 1, 0, 0), H0=1.0, alpha=0.0, xi=xi)
    p = params_from_workload(w)
    phi1, phi2 = droplet_phi(L, L, a, xi)
    psi, _, res = solve(p, phi1, phi2)
    assert res < 1e-12
    c = L // 2
    Hc = 1.0 - 0.5 * (psi[c, c + 1] - psi[c, c - 1])
    K = (mu_in - 1) / (mu_in + 1)
    expect = 2.0 / (1.0 + mu_in) * (1.0 + K * math.pi ** 2 * a ** 2 / (2 * L ** 2))
    assert abs(Hc / expect - 1.0) < 0.1 * xi / a
    # the field inside is uniform and along the applied field
    Hy = -0.5 * (psi[c + 1, c] - psi[c - 1, c])
    assert abs(Hy) < 1e-3


def test_no_ferrofluid_means_no_perturbation():
    nx, ny = 40, 20
    w = Workload(name="p9", nx=nx, ny=ny, chi=(0.0, 0.0, 0.0), H0=0.3, alpha=0.7, xi=4.0,
                 xc=20, yc=9.5, r_core=4, r_shell=7)
    s = OracleSim(w)
    s.init_droplet()
    # mu_r = 1 up to the rounding of phi1 + phi2 + (1 - phi1 - phi2)
    assert np.abs(s.psi).max() < 1e-14 * 0.3
    m = s.moments()
    np.testing.assert_allclose(m["Hx"], 0.3 * math.cos(0.7), rtol=0, atol=1e-14)
    np.testing.assert_allclose(m["Hy"], 0.3 * math.sin(0.7), rtol=0, atol=1e-14)
    fr = s.forces()
    assert np.abs(fr["Fm_x"]).max() < 1e-16 and np.abs(fr["Fm_y"]).max() < 1e-16


def test_linearity_in_h0():
    nx, ny = 48, 24
    phi1, phi2, _, _, _ = random_phase_fields(nx, ny, seed=2)
    pa = params_from_workload(Workload(name="l", nx=nx, ny=ny, chi=(2.0, 1.0, 0.0), H0=0.1, alpha=0.4))
    pb = params_from_workload(Workload(name="l", nx=nx, ny=ny, chi=(2.0, 1.0, 0.0), H0=0.3, alpha=0.4))
    a, _, _ = solve(pa, phi1, phi2)
    b, _, _ = solve(pb, phi1, phi2)
    np.testing.assert_allclose(b, 3.0 * a, rtol=0, atol=1e-14 * np.abs(b).max())


def test_sor_agrees_with_direct():
    nx, ny = 48, 24
    phi1, phi2, _, _, _ = random_phase_fields(nx, ny, seed=4)
    p = params_from_workload(Workload(name="s", nx=nx, ny=ny, chi=(2.0, 1.0, 0.0), H0=0.2, alpha=1.1))
    d, _, _ = solve(p, phi1, phi2)
    s, sweeps, res = solve(p, phi1, phi2, OracleSolver.sor(1.7, 1e-13, 100000, 4))
    assert res <= 1e-13 * 0.2 and sweeps > 10
    np.testing.assert_allclose(s, d, rtol=0, atol=1e-11)
