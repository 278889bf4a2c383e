"""Quasi-static coupling in the oracle (the potential solved every K steps and held in
between; K = 1 is the paper's every-step coupling): K = 1 is the plain step bit for bit, a
K beyond the run holds psi' at the initial solve exactly, and the deviation from the
every-step run grows like K - 1, the average number of steps psi' lags behind phi."""
import numpy as np

from fcd_inputs import channel_drive, single_channel_small
from oracle import OracleSim
from oracle.oracle import OracleSolver


def channel():
    w = single_channel_small(bond=4.0).replace(nx=80, ny=24, xc=30.0, yc=11.5, r_core=3.0, r_shell=7.0)
    return w.replace(drive_G=channel_drive(0.01, 1.0, 0.8, 24))


def run(w, every, nsteps, chunks=1):
    s = OracleSim(w, OracleSolver.direct(every=every))
    s.init_droplet()
    for _ in range(chunks):  # several calls: the solve phase carries over between them
        s.step(nsteps // chunks)
    return s


def test_every_one_is_the_plain_step_and_a_long_hold_keeps_the_initial_potential():
    w = channel()
    a = run(w, 1, 12)
    b = run(w, 0, 12, chunks=3)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g1, b.g1) and np.array_equal(a.psi, b.psi)
    s = OracleSim(w, OracleSolver.direct(every=1000))
    s.init_droplet()
    psi0 = s.psi.copy()
    s.step(5)
    s.step(7)
    assert np.array_equal(s.psi, psi0)
    # the hold changes the run: phi differs from the every-step run
    assert np.abs(s.g1.sum(0) - a.g1.sum(0)).max() > 1e-9


def test_chunked_steps_keep_the_solve_phase():
    w = channel()
    a = run(w, 4, 24)
    b = run(w, 4, 24, chunks=4)  # 6 steps per call: solves at 0, 4, 8, ... regardless
    assert np.array_equal(a.g1, b.g1) and np.array_equal(a.psi, b.psi)


def test_deviation_from_every_step_coupling_grows_like_the_lag():
    w = channel()
    ref = run(w, 1, 48)
    dev = {}
    for k in (2, 4, 8):
        s = run(w, k, 48)
        dev[k] = np.abs(s.g1.sum(0) - ref.g1.sum(0)).max()
    # psi' lags phi by (K - 1) / 2 steps on average: deviations in the ratio of K - 1
    assert 0.75 * 3.0 < dev[4] / dev[2] < 1.25 * 3.0, dev
    assert 0.75 * 7.0 / 3.0 < dev[8] / dev[4] < 1.25 * 7.0 / 3.0, dev
