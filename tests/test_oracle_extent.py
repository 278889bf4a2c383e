"""Extent-based deformation index of Eq. 42 in the oracle: T = (l_y - l_x) / (l_y + l_x)
from the interface w = 1/2 of the outer (phi1 + phi2) and inner (phi1) droplets, pinned by
closed forms: a circle gives T = 0 and extents 2r, an ellipse with semi-axes a, b gives
2a, 2b and (b - a) / (b + a); the periodic seam, wall-to-wall bands and empty channels."""
import numpy as np

from fcd_inputs import Workload
from oracle import OracleSim


def sim_with(phi1, phi2):
    ny, nx = phi1.shape
    s = OracleSim(Workload(name="ext", nx=nx, ny=ny, xi=4.0))
    z = np.zeros_like(phi1)
    s.init_fields(phi1, phi2, z, z, solve=False)
    return s


def ellipse_w(nx, ny, xc, yc, a, b, xi=4.0):
    """1/2 exactly on the ellipse (x/a)^2 + (y/b)^2 = 1 (periodic x), tanh across it."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx = (x - xc + nx / 2) % nx - nx / 2
    rho = np.sqrt((dx / a) ** 2 + ((y - yc) / b) ** 2)
    return 0.5 * (1.0 + np.tanh(2.0 * (1.0 - rho) * min(a, b) / xi))


def test_circle_and_ellipse_closed_forms():
    nx, ny = 160, 61
    wo = ellipse_w(nx, ny, 70.0, 30.0, 18.0, 18.0)
    wi = ellipse_w(nx, ny, 70.0, 30.0, 8.0, 8.0)
    T = sim_with(wi, wo - wi).extent_deformation()
    assert abs(T[0]) < 2e-3 and abs(T[1]) < 2e-3, T
    assert abs(T[2] - 36.0) < 0.1 and abs(T[3] - 36.0) < 0.1 and abs(T[4] - 16.0) < 0.1 and abs(T[5] - 16.0) < 0.1, T
    a, b = 24.0, 12.0  # outer stretched along x, inner along y
    wo = ellipse_w(nx, ny, 70.0, 30.0, a, b)
    wi = ellipse_w(nx, ny, 70.0, 30.0, 5.0, 9.0)
    T = sim_with(wi, wo - wi).extent_deformation()
    assert abs(T[0] - (b - a) / (b + a)) < 3e-3, T
    assert abs(T[1] - (9.0 - 5.0) / 14.0) < 3e-3, T
    assert abs(T[2] - 2 * b) < 0.1 and abs(T[3] - 2 * a) < 0.1, T


def test_periodic_seam_even_height_walls_and_empty_channel():
    nx, ny = 120, 40  # even ny: the centreline is the mean of rows 19 and 20
    wo = ellipse_w(nx, ny, 60.0, 19.5, 15.0, 10.0)
    wi = ellipse_w(nx, ny, 60.0, 19.5, 6.0, 4.0)
    T_mid = sim_with(wi, wo - wi).extent_deformation()
    # the same droplet centred on the seam x = 0
    T_seam = sim_with(np.roll(wi, 60, axis=1), np.roll(wo - wi, 60, axis=1)).extent_deformation()
    assert np.allclose(T_mid, T_seam, rtol=0, atol=1e-12), (T_mid, T_seam)
    assert abs(T_mid[3] - 30.0) < 0.1 and abs(T_mid[2] - 20.0) < 0.1, T_mid
    # a band across the whole channel: l_y runs wall to wall
    band = np.zeros((ny, nx))
    band[:, 50:70] = 1.0
    T = sim_with(np.zeros((ny, nx)), band).extent_deformation()
    assert T[2] == ny and abs(T[3] - 20.0) < 1e-12 and T[4] == 0.0 and T[5] == 0.0, T
    # nothing above 1/2: all extents and indices vanish
    T = sim_with(np.zeros((ny, nx)), np.full((ny, nx), 0.3)).extent_deformation()
    assert np.all(T == 0.0), T
