"""Batched adjoint: every channel's gradient from one batched reverse sweep against the
single-channel adjoint of the same channel (FP64, short and longer horizons), and FP32
batches of the 256 x 64 adjoint channels against single-channel FP64 gradients
(dD_o/d(H0, alpha), 1e-3, over a short horizon: over thousands of steps FP32 rounding moves
the gradients of strongly field-driven channels far more, see the design notes)."""
import math
import sys

import numpy as np
import pytest

from fcd_inputs import Workload, adjoint_batch, channel_drive, h0_from_bond

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_2410_11129_amd import fcd  # noqa: E402
from paper_2410_11129_amd.adjoint import AdjointRun, BatchAdjointRun, theta_of  # noqa: E402
from paper_2410_11129_amd.sim import Batch, Channel  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def field_channels():
    """Three channels of different size, surface tensions and field angle."""
    out = []
    for k, (nx, ny, rc, rs, alpha, s12, s13, s23) in enumerate((
            (96, 32, 5.0, 9.0, 30.0, 0.008, 0.012, 0.01),
            (64, 24, 4.0, 7.0, 75.0, 0.01, 0.01, 0.01),
            (128, 20, 3.0, 6.0, 10.0, 0.012, 0.009, 0.011))):
        u = 0.01
        out.append(Workload(name=f"badj_{k}", nx=nx, ny=ny, tau=(0.8, 0.8, 0.8), chi=(0.0, 1.0, 0.0),
                            sigma12=s12, sigma13=s13, sigma23=s23, xi=4.0,
                            H0=h0_from_bond(1.0, "shell", 1.0, rc, rs, s12, s23), alpha=math.radians(alpha),
                            drive_G=channel_drive(u, 1.0, 0.8, ny), xc=nx / 3.0, yc=ny / 2.0 - 0.7,
                            r_core=rc, r_shell=rs, u_ref=u))
    return out


def single_grad(w, nsteps, dJ, every=8, tol=1e-12):
    ch = Channel(w, tol=tol)
    run = AdjointRun(ch, nsteps, every)
    D = run.forward(theta_of(w))
    g = np.array(run.backward(dJ))
    ch.close()
    return D, g


@pytest.mark.parametrize("solver", ["sor", "mg"])
def test_batch_adjoint_equals_single_channel_adjoints_fp64(solver):
    """The batch's potentials by SOR or by the batched multigrid (forward and adjoint solves):
    every channel's gradient as its single-channel adjoint's."""
    ws = field_channels()
    nsteps = 20
    say(f"case batch adjoint fp64 {[(w.nx, w.ny) for w in ws]} {nsteps} steps, solver {solver}")
    kw = dict(solver=fcd.FCD_SOLVER_MG, smooth=2) if solver == "mg" else {}
    bt = Batch(ws, precision=fcd.FCD_FP64, tol=1e-12, **kw)
    bt.init_droplets()
    run = BatchAdjointRun(bt, nsteps, 6)
    D = run.forward()
    dJ = [(1.0, 0.5)] * len(ws)
    g = run.backward(dJ)
    for k, w in enumerate(ws):
        Ds, gs = single_grad(w, nsteps, dJ[k])
        th = np.array(theta_of(w))
        sc = np.where(np.arange(6) == 1, 1.0, np.abs(th))
        err = np.abs((np.array(g[k]) - gs) * sc)
        say(f"  {w.name}: D {D[k]} vs {Ds}; max scaled gradient error {err.max():.2e} of {np.abs(gs * sc).max():.2e}")
        assert abs(D[k][0] - Ds[0]) < 1e-11 and abs(D[k][1] - Ds[1]) < 1e-11
        assert np.all(err <= 1e-7 * np.abs(gs * sc) + 1e-10 * np.abs(gs * sc).max()), (w.name, g[k], gs)
    bt.close()


def test_batch_adjoint_fp32_tracks_fp64_single():
    ws = [w.replace(steps=60) for w in adjoint_batch()[:6]]
    nsteps, every = 60, 15
    say(f"case batch adjoint fp32, 6 channels 256x64, {nsteps} steps")
    bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5)
    bt.init_droplets()
    run = BatchAdjointRun(bt, nsteps, every)
    run.forward()
    g = run.backward([(1.0, 0.0)] * len(ws))
    for k, w in enumerate(ws):
        _, gs = single_grad(w, nsteps, (1.0, 0.0), tol=1e-10)
        for q, name in ((0, "H0"), (1, "alpha")):
            rel = abs(g[k][q] - gs[q]) / max(abs(gs[q]), 1e-300)
            say(f"  {w.name} Bo {w.bond:.2f} dDo/d{name}: fp32 batch {g[k][q]:.6e} fp64 {gs[q]:.6e} rel {rel:.1e}")
            # an exactly vanishing derivative (no field) is compared absolutely
            assert rel < 1e-3 or (gs[q] == 0.0 and g[k][q] == 0.0), (w.name, name)
    bt.close()


def test_batch_adjoint_fp64_long_horizon_matches_single():
    """The FP64 batch over a longer horizon, with the SOR factors tuned per channel and the
    default schedule (four-sweep tail launches included), against single-channel FP64
    gradients of the same 256 x 64 channels (including the most field-driven one)."""
    nsteps, every = 600, 60
    ws = adjoint_batch(steps=nsteps)[:3]
    say(f"case batch adjoint fp64, 3 channels 256x64, {nsteps} steps, checkpoint {every}")
    bt = Batch(ws, precision=fcd.FCD_FP64, tol=1e-10)
    bt.init_droplets()
    bt.step(4)
    bt.tune_omega(2)
    bt.init_droplets()
    run = BatchAdjointRun(bt, nsteps, every)
    D = run.forward()
    g = run.backward([(1.0, 0.0)] * len(ws))
    bt.close()
    for k, w in enumerate(ws):
        Ds, gs = single_grad(w, nsteps, (1.0, 0.0), every=every, tol=1e-10)
        assert abs(D[k][0] - Ds[0]) <= 1e-9 * abs(Ds[0]) + 1e-13, (w.name, D[k][0], Ds[0])
        for q, name in ((0, "H0"), (1, "alpha")):
            rel = abs(g[k][q] - gs[q]) / abs(gs[q])
            say(f"  {w.name} Bo {w.bond:.2f} dDo/d{name}: fp64 batch {g[k][q]:.9e} single {gs[q]:.9e} rel {rel:.1e}")
            assert rel < 1e-5, (w.name, name)


def test_batch_adjoint_leaves_final_state():
    ws = field_channels()[:2]
    say("case batch adjoint final state")
    bt = Batch(ws, precision=fcd.FCD_FP64, tol=1e-12)
    bt.init_droplets()
    run = BatchAdjointRun(bt, 9, 4)
    run.forward()
    s_fwd = [bt.state(k) for k in range(len(ws))]
    run.backward([(1.0, 0.0)] * len(ws))
    for k in range(len(ws)):
        assert np.array_equal(bt.state(k), s_fwd[k])
    bt.close()


def test_fp64_gradient_is_ill_conditioned_at_the_batched_adjoint_horizon():
    """Why the FP32 batched adjoint cannot meet 1e-3 at the stated 3000 steps: the FP64
    single-channel gradient of the most field-driven 256 x 64 channel (Bo_m = 5.4) itself
    moves by tens of percent when the initial state is perturbed by a random relative 6e-8
    (the size of FP32 rounding), while over 300 steps it moves by ~1e-6: the trajectory
    amplifies perturbations over the horizon, so no computation rounded at FP32's level can
    reproduce the FP64 gradient there."""
    w = adjoint_batch(steps=3000)[1]
    say(f"case FP64 gradient conditioning, {w.name} Bo {w.bond:.2f}")

    def grad(horizon, pert):
        ch = Channel(w, tol=1e-10)
        run = AdjointRun(ch, horizon, horizon // 20)
        ch.init_droplet()
        s = ch.state()
        rng = np.random.default_rng(5)
        ch.write_state(s * (1.0 + pert * rng.uniform(-1.0, 1.0, s.shape)))
        fcd.fcd_adjoint_forward(ch.h, horizon, horizon // 20, run.work.data_ptr())
        g = np.array(fcd.fcd_adjoint_backward(ch.h, [1.0, 0.0]))
        ch.close()
        return g

    rel = {}
    for horizon in (300, 3000):
        g0, g1 = grad(horizon, 0.0), grad(horizon, 6e-8)
        rel[horizon] = np.abs(g1[:2] - g0[:2]) / np.abs(g0[:2])
        say(f"  {horizon} steps: dD_o/d(H0, alpha) {g0[:2]} relative change {rel[horizon]}")
    assert rel[300].max() < 1e-4
    assert rel[3000].max() > 3e-2
