"""Pins of the oracle's lattice, equilibria, forcing and MRT collision.

Each expectation comes from a fact the paper or the mathematics fixes (moment
identities of a second-order Maxwellian, the published Lallemand-Luo moment
polynomials, conservation laws of the collision), not from re-typing the oracle.
"""
import ctypes as C
import math

import numpy as np
import pytest

from oracle.oracle import lib, ptr

CS2 = 1.0 / 3.0


def lattice():
    ex = (C.c_int32 * 9)()
    ey = (C.c_int32 * 9)()
    w = np.zeros(9)
    lib().orc_lattice(ex, ey, ptr(w))
    return np.array(ex[:], float), np.array(ey[:], float), w


def test_velocities_follow_eq20():
    ex, ey, w = lattice()
    # Eq. 20: alpha = 1-4 on the axes at (alpha-1) pi/2, alpha = 5-8 on the diagonals
    # at (2 alpha - 9) pi/4 with length sqrt(2); Eq. 17 weights.
    for a in range(1, 5):
        ang = (a - 1) * math.pi / 2
        assert ex[a] == pytest.approx(math.cos(ang), abs=1e-15)
        assert ey[a] == pytest.approx(math.sin(ang), abs=1e-15)
        assert w[a] == 1.0 / 9.0
    for a in range(5, 9):
        ang = (2 * a - 9) * math.pi / 4
        assert ex[a] == pytest.approx(math.sqrt(2) * math.cos(ang), abs=1e-14)
        assert ey[a] == pytest.approx(math.sqrt(2) * math.sin(ang), abs=1e-14)
        assert w[a] == 1.0 / 36.0
    assert ex[0] == 0 and ey[0] == 0 and w[0] == 4.0 / 9.0


def test_lattice_isotropy():
    ex, ey, w = lattice()
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert abs((w * ex).sum()) < 1e-16 and abs((w * ey).sum()) < 1e-16
    assert (w * ex * ex).sum() == pytest.approx(CS2, abs=1e-15)
    assert (w * ey * ey).sum() == pytest.approx(CS2, abs=1e-15)
    assert abs((w * ex * ey).sum()) < 1e-16
    # fourth-order isotropy: sum w e_i e_j e_k e_l = c_s^4 (d_ij d_kl + d_ik d_jl + d_il d_jk)
    assert (w * ex ** 4).sum() == pytest.approx(3 * CS2 ** 2, abs=1e-15)
    assert (w * ex ** 2 * ey ** 2).sum() == pytest.approx(CS2 ** 2, abs=1e-15)


def test_moment_matrix_is_lallemand_luo():
    m = np.zeros(81)
    minv = np.zeros(81)
    lib().orc_mrt_matrices(ptr(m), ptr(minv))
    M = m.reshape(9, 9)
    Minv = minv.reshape(9, 9)
    ex, ey, _ = lattice()
    e2 = ex ** 2 + ey ** 2
    # Published moment polynomials (Lallemand & Luo 2000, D2Q9).
    rows = [np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 ** 2, ex, (-5 + 3 * e2) * ex,
            ey, (-5 + 3 * e2) * ey, ex ** 2 - ey ** 2, ex * ey]
    for k in range(9):
        np.testing.assert_allclose(M[k], rows[k], atol=1e-14)
    np.testing.assert_allclose(Minv @ M, np.eye(9), atol=1e-14)
    np.testing.assert_allclose(M @ Minv, np.eye(9), atol=1e-14)


def gamma(u):
    out = np.zeros(9)
    lib().orc_gamma(ptr(np.array(u, float)), ptr(out))
    return out


def feq(p, u):
    out = np.zeros(9)
    lib().orc_feq(p, ptr(np.array(u, float)), ptr(out))
    return out


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.03, -0.02), (-0.1, 0.07)])
def test_gamma_moments(u):
    ex, ey, _ = lattice()
    G = gamma(u)
    ux, uy = u
    assert G.sum() == pytest.approx(1.0, abs=1e-15)
    assert (G * ex).sum() == pytest.approx(ux, abs=1e-15)
    assert (G * ey).sum() == pytest.approx(uy, abs=1e-15)
    assert (G * ex * ex).sum() == pytest.approx(CS2 + ux * ux, abs=1e-15)
    assert (G * ey * ey).sum() == pytest.approx(CS2 + uy * uy, abs=1e-15)
    assert (G * ex * ey).sum() == pytest.approx(ux * uy, abs=1e-15)


def test_printed_eq18_last_term_would_break_normalisation():
    # The reading of Eq. 18 (u.u/(2 c_s^2)) is the only coefficient giving sum = 1.
    ex, ey, w = lattice()
    u = np.array([0.05, 0.02])
    eu = ex * u[0] + ey * u[1]
    printed = w * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - (u @ u) / CS2)
    assert abs(printed.sum() - 1.0) > 1e-3
    assert abs(gamma(u).sum() - 1.0) < 1e-15


@pytest.mark.parametrize("p,u", [(0.0, (0.0, 0.0)), (0.013, (0.02, -0.01)), (-0.2, (-0.05, 0.04))])
def test_feq_moments(p, u):
    ex, ey, _ = lattice()
    f = feq(p, u)
    assert f.sum() == pytest.approx(p, abs=1e-15)
    assert (f * ex).sum() == pytest.approx(u[0], abs=1e-15)
    assert (f * ey).sum() == pytest.approx(u[1], abs=1e-15)


def test_forcing_moments():
    ex, ey, _ = lattice()
    F = np.array([1.3e-4, -2.1e-4])
    rho = 1.7
    out = np.zeros(9)
    lib().orc_forcing(ptr(F), rho, ptr(out))
    assert abs(out.sum()) < 1e-19
    assert (out * ex).sum() == pytest.approx(F[0] / rho, rel=1e-14)
    assert (out * ey).sum() == pytest.approx(F[1] / rho, rel=1e-14)


@pytest.mark.parametrize("tau", [0.2, 0.8, 1.0])
def test_collision_conserves_and_relaxes(tau):
    rng = np.random.default_rng(7)
    ex, ey, _ = lattice()
    f = feq(0.01, (0.02, -0.01)) + 1e-3 * rng.standard_normal(9)
    F = np.array([2e-4, -1e-4])
    rho = 1.3
    pstar = f.sum()
    u = np.array([(f * ex).sum() + F[0] / (2 * rho), (f * ey).sum() + F[1] / (2 * rho)])
    out = np.zeros(9)
    lib().orc_collide_f(ptr(f), pstar, ptr(u), ptr(F), rho, tau, ptr(out))
    # mass kept, momentum gains the full force (Eq. 12, 15, 19, 22)
    assert out.sum() == pytest.approx(pstar, abs=1e-15)
    assert (out * ex).sum() == pytest.approx(u[0] + F[0] / (2 * rho), abs=1e-15)
    assert (out * ey).sum() == pytest.approx(u[1] + F[1] / (2 * rho), abs=1e-15)
    # the stress moments of the non-equilibrium part decay by (1 - s_nu), s_nu = 1/(tau + 1/2)
    Fa = np.zeros(9)
    lib().orc_forcing(ptr(F), rho, ptr(Fa))
    fbar = feq(pstar, u) - 0.5 * Fa
    s = 1.0 / (0.5 + tau)
    for poly in (ex ** 2 - ey ** 2, ex * ey):
        before = (poly * (f - fbar)).sum()
        after = (poly * (out - fbar - Fa)).sum()
        assert after == pytest.approx((1 - s) * before, abs=1e-16)
    # every other non-conserved moment relaxes fully (unit rates)
    e2 = ex ** 2 + ey ** 2
    for poly in (-4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 ** 2, (-5 + 3 * e2) * ex, (-5 + 3 * e2) * ey):
        assert abs((poly * (out - fbar - Fa)).sum()) < 1e-16
