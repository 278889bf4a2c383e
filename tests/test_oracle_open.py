"""Open channel in the oracle (Sec. 2.5: Eq. 37 velocity inlet, convective outlet).

Pins: the inlet closure gives the distribution exactly the first moment Eq. 37 prescribes
(a dropped or mis-signed term in any of the three closed populations changes it); a fluid
at rest with no inflow stays at rest; a droplet on the centre line keeps the channel's
mirror symmetry (a transverse term of the closure with the wrong sign breaks it); the
phase masses are conserved while the droplet is away from both ends, the inflow carries
none, and a droplet leaves through the outlet with bounded order parameters; the
quasi-steady empty-channel flow satisfies continuity column by column."""
import numpy as np

from fcd_inputs import open_channel_small
from oracle import OracleSim


def inlet_profile(w):
    s = (np.arange(w.ny) + 0.5) / w.ny
    return 4.0 * w.u_inlet * s * (1.0 - s)


def empty_channel(w):
    sim = OracleSim(w)
    ny, nx = w.ny, w.nx
    ux = np.tile(inlet_profile(w)[:, None], (1, nx))
    zero = np.zeros((ny, nx))
    sim.init_fields(zero, zero, ux, zero)
    return sim


def first_moments(f, i):
    jx = f[1, :, i] + f[5, :, i] + f[8, :, i] - f[3, :, i] - f[6, :, i] - f[7, :, i]
    jy = f[2, :, i] + f[5, :, i] + f[6, :, i] - f[4, :, i] - f[7, :, i] - f[8, :, i]
    return jx, jy


def test_inlet_first_moment_is_eq37_every_step():
    w = open_channel_small(xc=20.0).replace(nx=60, ny=24, r_core=3.0, r_shell=6.0, yc=11.5)
    sim = OracleSim(w)
    sim.init_droplet()
    uin = inlet_profile(w)
    for _ in range(6):
        sim.step(3)
        jx, jy = first_moments(sim.f, 0)
        assert np.abs(jx - uin).max() < 1e-15
        assert np.abs(jy).max() < 1e-15
        # the entering order-parameter populations are zero (ambient inflow)
        for g in (sim.g1, sim.g2):
            assert np.abs(g[[1, 5, 8], :, 0]).max() == 0.0


def test_fluid_at_rest_without_inflow_stays_at_rest():
    w = open_channel_small(u_inlet=0.0).replace(nx=40, ny=16, H0=0.0)
    sim = empty_channel(w)
    f0 = sim.f.copy()
    sim.step(30)
    assert np.abs(sim.f - f0).max() < 1e-16


def test_centre_line_droplet_keeps_the_mirror_symmetry():
    ny = 30
    w = open_channel_small(xc=9.0, u_inlet=0.05).replace(nx=70, ny=ny, yc=(ny - 1) / 2.0, r_core=3.0,
                                                           r_shell=7.0)
    sim = OracleSim(w)
    sim.init_droplet()
    sim.step(60)
    m = sim.moments()
    for key in ("phi1", "phi2", "ux", "pstar", "Hx"):
        a = m[key]
        assert np.abs(a - a[::-1, :]).max() < 1e-12 * max(1.0, np.abs(a).max()), key
    for key in ("uy", "Hy"):
        a = m[key]
        assert np.abs(a + a[::-1, :]).max() < 1e-12 * max(1.0, np.abs(a).max()), key
    # the droplet's rear interface reaches the inlet's stencil: the test covers it
    assert m["phi2"][:, 0].max() > 1e-3


def test_phase_mass_is_conserved_away_from_the_ends():
    """Over a short run; later the ambient fluid takes up a trace of each droplet phase
    (order 1e-6 after 2000 steps of this channel) which the outlet then carries away."""
    w = open_channel_small(xc=60.0).replace(nx=120, ny=30, yc=14.5, r_core=4.0, r_shell=8.0)
    sim = OracleSim(w)
    p1, p2 = sim.init_droplet()
    m1, m2 = p1.sum(), p2.sum()
    sim.step(80)
    m = sim.moments()
    assert abs(m["phi1"].sum() - m1) < 1e-11 * m1
    assert abs(m["phi2"].sum() - m2) < 1e-11 * m2


def test_droplet_leaves_through_the_outlet():
    w = open_channel_small(xc=48.0, u_inlet=0.08).replace(nx=64, ny=24, yc=11.5, r_core=3.0, r_shell=6.0)
    sim = OracleSim(w)
    p1, p2 = sim.init_droplet()
    mass0 = p1.sum() + p2.sum()
    sim.step(900)
    m = sim.moments()
    mass = m["phi1"].sum() + m["phi2"].sum()
    assert mass < 0.1 * mass0, mass / mass0
    for key in ("phi1", "phi2"):
        assert np.isfinite(m[key]).all()
        assert m[key].min() > -0.05 and m[key].max() < 1.05
    assert np.isfinite(m["ux"]).all() and np.abs(m["ux"]).max() < 0.2


def test_quasi_steady_flow_satisfies_continuity_column_by_column():
    """Empty channel from the Eq. 37 profile.  The convective outlet makes the unknown
    populations' streamwise gradient vanish while the pressure-driven flow has one, so the
    pressure level rises at a uniform rate; mass conservation then ties the drop of the
    section flux between columns to that rate: Q(i) - Q(i+1) = ny dp*/dt."""
    w = open_channel_small(u_inlet=0.05).replace(nx=80, ny=20, H0=0.0)
    sim = empty_channel(w)
    sim.step(1500)
    p_a = sim.moments()["pstar"].copy()
    sim.step(100)
    m = sim.moments()
    rate = (m["pstar"] - p_a) / 100.0
    assert rate.std() < 0.02 * rate.mean()  # uniform rise
    Q = m["ux"].sum(axis=0)
    dQ = Q[:-1] - Q[1:]
    expected = w.ny * rate.mean()
    assert np.abs(dQ[5:-5] - expected).max() < 0.03 * expected
    assert abs(Q[0] - inlet_profile(w).sum()) < 1e-12
