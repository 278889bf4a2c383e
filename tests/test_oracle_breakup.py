"""Breakup probe in the oracle (Sec. 2.5: the inner droplet touching the shell's
interface): a core well inside its shell has no contact node, a core poking through the
shell's side touches the carrier there (symmetric about the axis of the offset), the
periodic seam moves nothing but x, and the outer droplet's circular-mean x is its centre."""
import numpy as np

from fcd_inputs import Workload
from oracle import OracleSim


def compound(nx, ny, xs, ys, rs, xc, yc, rc, xi=4.0):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)

    def disc(x0, y0, r):
        dx = (x - x0 + nx / 2) % nx - nx / 2
        return 0.5 * (1.0 + np.tanh(2.0 * (r - np.hypot(dx, y - y0)) / xi))

    core = disc(xc, yc, rc)
    outer = np.maximum(disc(xs, ys, rs), core)
    return core, outer - core


def probe(phi1, phi2):
    ny, nx = phi1.shape
    s = OracleSim(Workload(name="brk", nx=nx, ny=ny, xi=4.0))
    z = np.zeros_like(phi1)
    s.init_fields(phi1, phi2, z, z, solve=False)
    return s.breakup_probe()


def test_intact_and_touching_cores():
    nx, ny = 120, 61
    p1, p2 = compound(nx, ny, 60.0, 30.0, 20.0, 60.0, 30.0, 9.0)
    out = probe(p1, p2)
    assert out[0] == 0 and out[1] == -1.0 and out[2] == -1.0, out
    assert abs(out[3] - 60.0) < 1e-6, out
    # the core shifted right until it crosses the shell's interface
    p1, p2 = compound(nx, ny, 60.0, 30.0, 20.0, 74.0, 30.0, 10.0)
    out = probe(p1, p2)
    assert out[0] > 0, out
    assert abs(out[1] - 30.0) < 1e-9, out  # symmetric about the row of the offset
    assert 78.0 < out[2] < 86.0, out      # on the shell's right side (its edge at x = 80)


def test_periodic_seam_shifts_only_x():
    nx, ny = 120, 61
    p1, p2 = compound(nx, ny, 60.0, 30.0, 20.0, 74.0, 30.0, 10.0)
    a = probe(p1, p2)
    b = probe(np.roll(p1, 50, axis=1), np.roll(p2, 50, axis=1))
    assert a[0] == b[0] and abs(a[1] - b[1]) < 1e-12, (a, b)
    assert abs(((b[2] - a[2] - 50.0) + 60.0) % 120.0 - 60.0) < 1e-9, (a, b)
    assert abs(((b[3] - a[3] - 50.0) + 60.0) % 120.0 - 60.0) < 1e-9, (a, b)
