"""Physics pins of the oracle's coupled step: closed forms and invariants the paper's
equations imply (Poiseuille flow, Laplace law, stationary flat interface, layered
flow with density contrast, Kelvin-force symmetry, conservation)."""
import math

import numpy as np
import pytest
from scipy.integrate import cumulative_trapezoid

from fcd_inputs import Workload, channel_drive, h0_from_bond, single_channel_small
from oracle import OracleSim, OracleSolver

SOR = OracleSolver.sor(1.8, 1e-10, 200000, 4)


def rest_fields(ny, nx):
    z = np.zeros((ny, nx))
    return z, z.copy(), z.copy(), z.copy()


def test_poiseuille_exact_at_magic_relaxation():
    """Halfway bounce-back + unit rates for the odd moments: the steady profile is the
    exact parabola when Lambda = tau * 1/2 = 3/16, i.e. tau = 3/8."""
    ny, nx, tau = 16, 4, 3.0 / 8.0
    G = channel_drive(0.01, 1.0, tau, ny)
    s = OracleSim(Workload(name="p", nx=nx, ny=ny, tau=(tau,) * 3, drive_G=G, xi=4.0))
    s.init_fields(*rest_fields(ny, nx))
    s.step(30000)
    m = s.moments()
    y = np.arange(ny, dtype=float)
    exact = G / (2 * tau / 3) * (y + 0.5) * (ny - 0.5 - y)
    np.testing.assert_allclose(m["ux"], np.tile(exact[:, None], (1, nx)), rtol=0, atol=1e-10 * exact.max())
    assert np.abs(m["uy"]).max() < 1e-14


def test_poiseuille_slip_at_tau_08():
    """Away from the magic value the halfway wall slips by the known TRT amount
    u_s = G/(2 nu) (16 Lambda - 3)/12 with Lambda = tau/2; profile shape stays parabolic."""
    ny, nx, tau = 16, 4, 0.8
    G = channel_drive(0.01, 1.0, tau, ny)
    s = OracleSim(Workload(name="p", nx=nx, ny=ny, tau=(tau,) * 3, drive_G=G, xi=4.0))
    s.init_fields(*rest_fields(ny, nx))
    s.step(30000)
    u = s.moments()["ux"][:, 0]
    y = np.arange(ny, dtype=float)
    scale = G / (2 * tau / 3)
    slip = u - scale * (y + 0.5) * (ny - 0.5 - y)
    assert np.ptp(slip) < 1e-9 * scale * ny ** 2
    assert slip.mean() / scale == pytest.approx((16 * tau / 2 - 3) / 12, rel=0.01)


@pytest.mark.parametrize("xi", [4.0, 8.0])
def test_flat_interface_is_stationary(xi):
    """A tanh interface of width xi is the rest solution of Eq. 23; the discrete profile
    drifts from it by O(1/xi^2) only."""
    nx, ny = 128, 4
    x = np.arange(nx, dtype=float)
    phi = 0.5 * (np.tanh(2 * (x - 32) / xi) - np.tanh(2 * (x - 96) / xi))
    phi1 = np.tile(phi, (ny, 1))
    s = OracleSim(Workload(name="flat", nx=nx, ny=ny, xi=xi))
    z = np.zeros((ny, nx))
    s.init_fields(phi1, z, z, z)
    s.step(4000)
    drift = np.abs(s.moments()["phi1"] - phi1).max()
    assert drift < 0.1 / xi ** 2 * 1.1
    assert np.abs(s.moments()["phi2"]).max() < 1e-15


def _pressure(m):
    return m["pstar"] / 3.0  # p = rho c_s^2 p*, rho = 1 (Eq. 21)


def test_laplace_single_droplet():
    """Delta p = sigma/R (2-D Laplace law).  With xi = 4 the interface is resolved by a
    few nodes; the O(1/xi^2) discretisation error is several percent."""
    n, R = 64, 16
    w = Workload(name="lap", nx=n, ny=n, xi=4.0, tau=(0.8,) * 3, xc=(n - 1) / 2, yc=(n - 1) / 2,
                 r_core=R, r_shell=R)
    s = OracleSim(w)
    s.init_droplet()
    s.step(3000)
    m = s.moments()
    p = _pressure(m)
    c = n // 2
    dp = p[c - 2:c + 2, c - 2:c + 2].mean() - p[:3, :].mean()
    assert dp == pytest.approx(0.01 / R, rel=0.10)
    assert np.abs(m["phi2"]).max() < 1e-13  # absent phase stays absent


def test_laplace_compound_droplet_unequal_tensions():
    """Core/shell and shell/ambient pressure jumps follow sigma12/r1 and sigma23/r2."""
    n, r1, r2 = 64, 10, 22
    w = Workload(name="cmp", nx=n, ny=n, xi=4.0, sigma12=0.006, sigma13=0.01, sigma23=0.01,
                 tau=(0.8,) * 3, xc=(n - 1) / 2, yc=(n - 1) / 2, r_core=r1, r_shell=r2)
    s = OracleSim(w)
    s.init_droplet()
    s.step(3000)
    p = _pressure(s.moments())
    y, x = np.mgrid[0:n, 0:n]
    d = np.hypot(x - (n - 1) / 2, y - (n - 1) / 2)
    p1, p2, p3 = p[d < 4].mean(), p[(d > 15.5) & (d < 16.5)].mean(), p[:3, :].mean()
    assert p1 - p2 == pytest.approx(0.006 / r1, rel=0.12)
    assert p2 - p3 == pytest.approx(0.01 / r2, rel=0.12)


def test_layered_flow_with_density_and_viscosity_contrast():
    """Steady two-layer channel flow solves d/dy(rho nu du/dy) = -G.  This needs the
    viscous force F_mu = nu (grad u + grad u^T).grad rho of the velocity-based model and
    the linear viscosity mix; without F_mu the profile would be off by ~8%."""
    ny, nx, xi = 64, 4, 4.0
    rho1, tau1, rho3, tau3 = 4.0, 0.3, 1.0, 0.8
    G = channel_drive(0.01, 1.0, tau3, ny)
    w = Workload(name="layer", nx=nx, ny=ny, xi=xi, rho=(rho1, 1.0, rho3), tau=(tau1, 0.8, tau3),
                 drive_G=G)
    yy = np.arange(ny, dtype=float)
    phi = 0.5 * (1 + np.tanh(2 * (yy - 31.5) / xi))
    z = np.zeros((ny, nx))
    s = OracleSim(w)
    s.init_fields(np.tile(phi[:, None], (1, nx)), z, z, z)
    s.step(30000)
    u = s.moments()["ux"][:, 0]
    ys = np.linspace(-0.5, ny - 0.5, 20001)
    ph = 0.5 * (1 + np.tanh(2 * (ys - 31.5) / xi))
    mu = (rho1 * ph + rho3 * (1 - ph)) * (tau1 * ph + tau3 * (1 - ph)) / 3.0
    i1 = cumulative_trapezoid(1 / mu, ys, initial=0)
    i2 = cumulative_trapezoid(ys / mu, ys, initial=0)
    exact = np.interp(yy, ys, G * i2[-1] / i1[-1] * i1 - G * i2)
    assert np.abs(u - exact).max() < 0.01 * np.abs(exact).max()


@pytest.mark.parametrize("alpha,sign", [(0.0, -1), (math.pi / 2, +1)])
def test_ferrofluid_droplet_elongates_along_field(alpha, sign):
    n, R = 48, 10
    H0 = h0_from_bond(2.0, "core", 1.0, R, R, 0.01, 0.01)
    w = Workload(name="fer", nx=n, ny=n, xi=4.0, chi=(1.0, 0, 0), H0=H0, alpha=alpha,
                 tau=(0.8,) * 3, xc=(n - 1) / 2, yc=(n - 1) / 2, r_core=R, r_shell=R)
    s = OracleSim(w, SOR)
    s.init_droplet()
    assert abs(s.diagnostics()[1]) < 1e-12
    s.step(400)
    D = s.diagnostics()[1]
    assert sign * D > 0.01


def test_kelvin_force_has_no_net_component():
    """In a uniform applied field the Kelvin force on a droplet integrates to zero."""
    n, R = 48, 10
    H0 = h0_from_bond(2.0, "core", 1.0, R, R, 0.01, 0.01)
    w = Workload(name="fer", nx=n, ny=n, xi=4.0, chi=(1.0, 0, 0), H0=H0, alpha=math.radians(30),
                 xc=(n - 1) / 2, yc=(n - 1) / 2, r_core=R, r_shell=R)
    s = OracleSim(w)
    s.init_droplet()
    F = s.forces()
    total = np.hypot(F["Fm_x"], F["Fm_y"]).sum()
    assert total > 0
    assert abs(F["Fm_x"].sum()) < 1e-12 * total and abs(F["Fm_y"].sum()) < 1e-12 * total


def small_channel(alpha):
    w = single_channel_small()
    return w.replace(nx=80, ny=32, xc=30.0, yc=15.5, r_core=4.0, r_shell=9.0, alpha=alpha,
                     drive_G=channel_drive(0.01, 1.0, 0.8, 32))


def test_mass_conservation_coupled():
    s = OracleSim(small_channel(math.radians(30)))
    s.init_droplet()
    d0 = s.diagnostics()
    s.step(300)
    d1 = s.diagnostics()
    assert abs(d1[2] - d0[2]) < 1e-12 * d0[2]
    assert abs(d1[3] - d0[3]) < 1e-12 * d0[3]


@pytest.mark.parametrize("alpha", [0.0, math.pi / 2])
def test_mirror_symmetry_about_midplane(alpha):
    """A droplet on the mid-plane y = (ny-1)/2 with the field along x or y keeps the
    mirror symmetry of the set-up: phi, p*, u_x even; u_y odd; psi' and H follow the
    parity of the applied potential (even for a field along x, odd along y)."""
    s = OracleSim(small_channel(alpha))
    s.init_droplet()
    s.step(200)
    m = s.moments()
    even = ["phi1", "phi2", "pstar", "ux"]
    odd = ["uy"]
    if alpha == 0.0:
        even += ["psi", "Hx"]
        odd += ["Hy"]
    else:
        even += ["Hy"]
        odd += ["psi", "Hx"]
    for k in even:
        a = m[k]
        assert np.abs(a - a[::-1, :]).max() < 1e-12 * max(np.abs(a).max(), 1e-30), k
    for k in odd:
        a = m[k]
        assert np.abs(a + a[::-1, :]).max() < 1e-12 * max(np.abs(a).max(), 1e-30), k


def test_deformation_metric():
    from oracle.oracle import lib, ptr
    n = 200
    y, x = np.mgrid[0:n, 0:n].astype(float)
    circ = ((x - 137.3) ** 2 + (y - 100.0) ** 2 < 40 ** 2).astype(float)
    assert abs(lib().orc_deformation_w(n, n, ptr(circ))) < 2e-3
    a, b = 50.0, 30.0  # semi-axes along x, y
    ell = (((x - 100) / a) ** 2 + ((y - 100) / b) ** 2 < 1).astype(float)
    assert lib().orc_deformation_w(n, n, ptr(ell)) == pytest.approx((b - a) / (b + a), abs=3e-3)
    # centroid by circular mean: a shape straddling the periodic seam is measured whole
    seam = (((x - 5) / a) ** 2 + ((y - 100) / b) ** 2 < 1) | (((x - 205) / a) ** 2 + ((y - 100) / b) ** 2 < 1)
    assert lib().orc_deformation_w(n, n, ptr(seam.astype(float))) == pytest.approx((b - a) / (b + a), abs=3e-3)


def test_initial_state():
    w = small_channel(0.0)
    s = OracleSim(w)
    phi1, phi2 = s.init_droplet()
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)[:, None, None]
    np.testing.assert_allclose(s.g1.sum(0), phi1, atol=1e-15)
    np.testing.assert_allclose(s.g2.sum(0), phi2, atol=1e-15)
    np.testing.assert_allclose(s.f.sum(0), 0.0, atol=1e-16)
    y = np.arange(w.ny, dtype=float)
    upois = w.drive_G / (2 * 0.8 / 3) * (y + 0.5) * (w.ny - 0.5 - y)
    np.testing.assert_allclose((s.f * ex).sum(0), np.tile(upois[:, None], (1, w.nx)), atol=1e-16)
    assert phi1.max() > 0.95 and (phi1 + phi2).max() < 1.0 + 1e-15 and phi2.min() > -1e-15
    # tanh profiles cross 1/2 at the radii
    i = int(w.xc + w.r_shell)
    prof = (phi1 + phi2)[int(w.yc + 0.5), :]
    assert prof[i - 1] > 0.5 > prof[i + 1]
