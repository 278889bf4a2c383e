"""Batched channels (one launch per kernel for all channels) vs each channel run alone."""
import sys

import numpy as np
import pytest

from fcd_inputs import Workload, channel_drive, random_phase_fields, regime_sweep_batch, single_channel_small
from oracle import OracleSim

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_2410_11129_amd import fcd  # noqa: E402
from paper_2410_11129_amd.sim import Batch, Channel  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def uneven_channels():
    """Three channels of different size, parameters and field (one without field)."""
    a = single_channel_small().replace(name="a", nx=100, ny=22, xc=30.0, yc=10.5, r_core=3.0, r_shell=7.0,
                                       drive_G=channel_drive(0.01, 1.0, 0.8, 22))
    b = Workload(name="b", nx=64, ny=16, rho=(2.0, 1.0, 1.0), tau=(1.0, 0.25, 0.25), chi=(2.0, 0.0, 0.0),
                 sigma12=0.008, sigma13=0.01, sigma23=0.012, xi=4.0, H0=0.0, alpha=0.0,
                 drive_G=channel_drive(0.01, 1.0, 0.25, 16), xc=20.0, yc=7.5, r_core=3.0, r_shell=6.0)
    c = single_channel_small().replace(name="c", nx=130, ny=41, xc=60.0, yc=20.0, r_core=5.0, r_shell=11.0,
                                       alpha=1.1, drive_G=channel_drive(0.01, 1.0, 0.8, 41))
    # narrower than a fused-sweep tile with its halo: the halo wraps onto the tile itself
    d = single_channel_small().replace(name="d", nx=48, ny=19, xc=20.0, yc=9.0, r_core=2.5, r_shell=5.5,
                                       alpha=0.4, drive_G=channel_drive(0.01, 1.0, 0.8, 19))
    return [a, b, c, d]


def test_batch_channels_match_oracle_fp64():
    ws = uneven_channels()
    say("case batch fp64 3 uneven channels vs oracle")
    bt = Batch(ws, precision=fcd.FCD_FP64, tol=1e-12)
    bt.init_droplets()
    bt.step(30)
    dg = bt.deformation()
    for k, w in enumerate(ws):
        s = OracleSim(w)
        s.init_droplet(solve=False)
        assert s.step(30) == 0
        ref = np.concatenate([s.f, s.g1, s.g2])
        assert np.abs(bt.state(k) - ref).max() < 1e-11, w.name
        m, om = bt.moments(k), s.moments()
        for key in om:
            assert np.abs(m[key] - om[key]).max() < 1e-11, (w.name, key)
        od = s.diagnostics()
        assert abs(dg[k][0] - od[0]) < 1e-11 and abs(dg[k][1] - od[1]) < 1e-11


def test_batch_fp32_regime_channels_track_fp64():
    """Six channels of the regime sweep in FP32 against the single-channel FP64 path.

    On these channels (sigma up to 0.033, tau = 0.2, strong fields) the method itself is
    sensitive at isolated nodes where phi overshoots: the FP64 oracle, perturbed by random
    relative errors of 6e-8 (FP32 rounding) every step, moves phi by 1.3e-3 at single
    nodes within 100 steps while D moves by < 1e-5.  So the max-norm bar of 1e-4 on phi
    is applied over the first 20 steps, before that amplification; after 200 steps D is
    held to 1e-3 and phi to 1e-4 in the mean.
    """
    ws = [w.replace(steps=200) for w in regime_sweep_batch()[::11]]
    say(f"case batch fp32 regime subset sizes {[(w.nx, w.ny) for w in ws]}")
    bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5)
    bt.init_droplets()
    gs = []
    for w in ws:
        g = Channel(w, tol=1e-10)
        g.init_droplet()
        gs.append(g)
    for n_steps, final in ((20, False), (180, True)):
        bt.step(n_steps)
        dg = bt.deformation()
        for k, (w, g) in enumerate(zip(ws, gs)):
            g.step(n_steps)
            m32, m64 = bt.moments(k), g.moments()
            d64 = g.deformation()
            e_mean = max(np.abs(m32[key] - m64[key]).mean() for key in ("phi1", "phi2", "phi3"))
            e_max = max(np.abs(m32[key] - m64[key]).max() for key in ("phi1", "phi2", "phi3"))
            say(f"  {w.name} Bo {w.bond:.2f} after {'200' if final else '20'} steps: mean|dphi| {e_mean:.2e} "
                f"max|dphi| {e_max:.2e} dD {abs(dg[k][0] - d64[0]):.2e} {abs(dg[k][1] - d64[1]):.2e}")
            if not final:
                assert e_max < 1e-4, w.name
            else:
                assert e_mean < 1e-4, w.name
                assert abs(dg[k][0] - d64[0]) < 1e-3 and abs(dg[k][1] - d64[1]) < 1e-3
                assert abs(dg[k][2] - d64[2]) < 1e-4 * d64[2]
    for g in gs:
        g.close()


def test_batch_deterministic_and_single_channel_batch():
    ws = uneven_channels()
    say("case batch determinism")
    out = []
    for _ in range(2):
        bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5)
        bt.init_droplets()
        bt.step(20)
        out.append([bt.state(k) for k in range(len(ws))])
        bt.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)
    # a channel's sweeps are decided on the device from its own residual alone, so a
    # batch of one gives that channel's state bit for bit
    one = Batch([ws[2]], precision=fcd.FCD_FP32, tol=1e-5)
    one.init_droplets()
    one.step(20)
    assert np.array_equal(one.state(0), out[0][2])


@pytest.mark.parametrize("precision", [fcd.FCD_FP64, fcd.FCD_FP32])
def test_batch_schedules_and_autotuner_do_not_change_results(precision):
    """Tile shapes, graph block sizes, fused sweeps and tail fusion change launch geometry
    only: every schedule, and the autotuner's trial steps, give the same states bit for
    bit."""
    ws = uneven_channels()
    say(f"case batch schedules precision {precision}")
    tol = 1e-12 if precision == fcd.FCD_FP64 else 1e-5
    ref = Batch(ws, precision=precision, tol=tol)
    ref.init_droplets()
    ref.step(6)
    want = [ref.state(k) for k in range(len(ws))]
    for rows, block, fused, tail in ((1, 4, 0, 0), (8, 128, 1, 4), (2, 32, 2, 0), (4, 8, 0, 4), (8, 8, 4, 0),
                                     (2, 32, 4, 2), (4, 8, 2, 4)):
        bt = Batch(ws, precision=precision, tol=tol)
        bt.set_schedule(rows, block, fused)
        bt.set_tail_fusion(tail, 8)  # blocks from the ninth sweep of a solve on
        bt.init_droplets()
        for _ in range(3):  # several graph replays with eager work between them
            bt.step(2)
        for k in range(len(ws)):
            assert np.array_equal(bt.state(k), want[k]), (rows, block, fused, tail, k)
        bt.close()
    tuned = Batch(ws, precision=precision, tol=tol)
    tuned.init_droplets()
    # advances 12 * 4 * (1 + 1) = 96 steps, then 4 * (1 + 1) for the tail fusion
    rows, block, fused, tail, after = tuned.autotune(1)
    assert rows in (1, 2, 4, 8) and block % 4 == 0 and fused in (0, 1, 2, 4)
    assert (tail, after) in ((0, 0), (4, 32), (4, 64), (4, 128))
    ref.step(98)
    for k in range(len(ws)):
        assert np.array_equal(tuned.state(k), ref.state(k)), k
    tuned.close()
    ref.close()


def test_sor_factor_tuner_is_reproducible():
    """The per-channel SOR factor tuner picks from the candidates by sweep counts alone:
    two identical batches pick the same factors, a channel without field (no sweeps)
    keeps the first candidate, and the batch then runs and converges with them."""
    import math
    ws = uneven_channels()
    scales = (1.25, 1.0, 0.775)
    say("case batch SOR factor tuner")
    picks = []
    for _ in range(2):
        bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5)
        bt.init_droplets()
        bt.step(3)
        picks.append(bt.tune_omega(2, scales))
        bt.init_droplets()
        bt.step(4)
        assert np.isfinite(np.asarray(bt.deformation())).all()
        bt.close()
    assert picks[0] == picks[1]
    for w, om in zip(ws, picks[0]):
        cands = [2.0 / (1.0 + s * math.sin(math.pi / (w.ny + 1))) for s in scales]
        assert min(abs(om - c) for c in cands) < 1e-15, (w.name, om, cands)
        if w.H0 == 0.0:
            assert om == cands[0]


def test_many_channels_and_a_longer_test_interval():
    """More channels than the decision kernel's block (its channel scan and tile list run in
    chunks), and a test interval of 8 (two- and four-sweep launches per interval): each
    channel ends bit for bit as it does in a batch of its own."""
    base = single_channel_small().replace(nx=48, ny=14, xc=16.0, yc=6.5, r_core=2.0, r_shell=4.5,
                                          drive_G=channel_drive(0.01, 1.0, 0.8, 14))
    ws = [base.replace(name=f"m{k}", H0=base.H0 * (0.5 + (k % 7) / 7.0), alpha=0.1 * (k % 5),
                       ny=14 + (k % 3), drive_G=channel_drive(0.01, 1.0, 0.8, 14 + (k % 3)))
          for k in range(300)]
    say(f"case batch of {len(ws)} channels, test interval 8")
    for fused, tail in ((2, 4), (1, 0), (4, 0)):
        bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5, check_every=8)
        bt.set_schedule(4, 16, fused)
        bt.set_tail_fusion(tail, 8)
        bt.init_droplets()
        bt.step(3)
        got = {k: bt.state(k) for k in (0, 1, 137, 299)}
        bt.close()
        for k, st in got.items():
            one = Batch([ws[k]], precision=fcd.FCD_FP32, tol=1e-5, check_every=8)
            one.set_schedule(4, 16, 0)
            one.init_droplets()
            one.step(3)
            assert np.array_equal(one.state(0), st), (fused, tail, k)
            one.close()


MG = dict(solver=fcd.FCD_SOLVER_MG, smooth=2)


def test_batch_multigrid_matches_oracle_fp64():
    """The batched multigrid (one launch per level for every channel; each channel's
    convergence decided on the device after its cycle's first sweep) on the uneven channels
    (one without field, odd ny, one narrower than a tile) against the oracle, to the SOR
    batch's bar."""
    ws = uneven_channels()
    say("case batch multigrid fp64 uneven channels vs oracle")
    bt = Batch(ws, precision=fcd.FCD_FP64, tol=1e-12, **MG)
    bt.init_droplets()
    bt.step(30)
    cycles = bt.stats()[1]
    say(f"  {cycles:.0f} V-cycles launched over 30 steps")
    # V-cycles, not SOR sweeps (an SOR batch needs hundreds of sweeps a step here)
    assert cycles <= 30 * 40
    dg = bt.deformation()
    for k, w in enumerate(ws):
        s = OracleSim(w)
        s.init_droplet(solve=False)
        assert s.step(30) == 0
        ref = np.concatenate([s.f, s.g1, s.g2])
        assert np.abs(bt.state(k) - ref).max() < 1e-11, w.name
        m, om = bt.moments(k), s.moments()
        for key in om:
            assert np.abs(m[key] - om[key]).max() < 1e-11, (w.name, key)
        od = s.diagnostics()
        assert abs(dg[k][0] - od[0]) < 1e-11 and abs(dg[k][1] - od[1]) < 1e-11
    bt.close()


@pytest.mark.parametrize("precision", [fcd.FCD_FP64, fcd.FCD_FP32])
def test_batch_multigrid_channel_equals_its_batch_of_one(precision):
    """A channel's cycles are decided on the device from its own residual alone: in a batch
    of 300 channels (more than the decision kernel's block) of differing size, field and
    hierarchy depth, each sampled channel ends bit for bit as in a batch of its own."""
    base = single_channel_small().replace(nx=48, ny=14, xc=16.0, yc=6.5, r_core=2.0, r_shell=4.5,
                                          drive_G=channel_drive(0.01, 1.0, 0.8, 14))
    ws = [base.replace(name=f"m{k}", H0=base.H0 * (0.5 + (k % 7) / 7.0), alpha=0.1 * (k % 5),
                       ny=14 + (k % 5), nx=48 + 16 * (k % 3), drive_G=channel_drive(0.01, 1.0, 0.8, 14 + (k % 5)))
          for k in range(300)] + uneven_channels()
    tol = 1e-10 if precision == fcd.FCD_FP64 else 1e-5
    say(f"case batch multigrid of {len(ws)} channels, precision {precision}")
    bt = Batch(ws, precision=precision, tol=tol, **MG)
    bt.init_droplets()
    bt.step(6)
    got = {k: bt.state(k) for k in (0, 1, 137, 299, 300, 302, 303)}
    bt.close()
    for k, st in got.items():
        one = Batch([ws[k]], precision=precision, tol=tol, **MG)
        one.init_droplets()
        one.step(6)
        assert np.array_equal(one.state(0), st), k
        one.close()


def test_batch_multigrid_fp32_regime_channels_track_fp64():
    """The FP32 multigrid batch on the regime-sweep channels (odd ny among them) against
    single-channel FP64 runs, to the bars of the FP32 SOR batch: max |d phi| <= 1e-4 after
    20 steps; after 200, mean |d phi| <= 1e-4 and |dD| <= 1e-3."""
    ws = [w.replace(steps=200) for w in regime_sweep_batch()[::11]]
    say(f"case batch multigrid fp32 regime subset sizes {[(w.nx, w.ny) for w in ws]}")
    bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5, **MG)
    bt.init_droplets()
    gs = []
    for w in ws:
        g = Channel(w, tol=1e-10)
        g.init_droplet()
        gs.append(g)
    for n_steps, final in ((20, False), (180, True)):
        bt.step(n_steps)
        dg = bt.deformation()
        for k, (w, g) in enumerate(zip(ws, gs)):
            g.step(n_steps)
            m32, m64 = bt.moments(k), g.moments()
            d64 = g.deformation()
            e_mean = max(np.abs(m32[key] - m64[key]).mean() for key in ("phi1", "phi2", "phi3"))
            e_max = max(np.abs(m32[key] - m64[key]).max() for key in ("phi1", "phi2", "phi3"))
            say(f"  {w.name} Bo {w.bond:.2f} after {'200' if final else '20'} steps: mean|dphi| {e_mean:.2e} "
                f"max|dphi| {e_max:.2e} dD {abs(dg[k][0] - d64[0]):.2e} {abs(dg[k][1] - d64[1]):.2e}")
            if not final:
                assert e_max < 1e-4, w.name
            else:
                assert e_mean < 1e-4, w.name
                assert abs(dg[k][0] - d64[0]) < 1e-3 and abs(dg[k][1] - d64[1]) < 1e-3
    for g in gs:
        g.close()
    bt.close()
