#!/usr/bin/env python3
"""Benchmark of the coupled ferrofluid compound-droplet step on one MI355X.

Workload: the 2048 x 512 channel (shell r = 80, core r = 40, Ca = 0.1, densities 2:1:1,
viscosities 5:1:1, ferrofluid core mu_r = 3, field at 90 degrees, Bo_m = 2), FP64.
A step is one full coupled update: phase moments, potential solve to
max |L(psi0 + psi')| <= 1e-10 H0 (multigrid V-cycles warm-started from the extrapolated
previous solutions, or four-colour SOR), fused collide-and-stream.
Inputs are resident in HBM before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "MLUPS + HBM GB/s of coupled step; batched instances/hr; adjoint/forward ratio"



# HBM bytes per launch of the collide-and-stream kernel on the 2048 x 512 FP64 channel from
# two rocprofv3 counter passes (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, the factors that a
# 2 GiB device copy reads on the same counters), with the first 16 hex digits of the sha256
# of the sources the kernel was built from; reported only while the sources are unchanged.
TRAFFIC_BYTES = {"collide_stream": (2 * 129801 + 230388) * 1024}
TRAFFIC_SOURCES = {"paper_2410_11129_amd/csrc/fcd_step.hpp": "0955c195fe226b4b",
                   "paper_2410_11129_amd/csrc/fcd_device.hpp": "2dc4056d7fa7d715",
                   "paper_2410_11129_amd/csrc/fcd_kernels.hip": "08640913d66b3237"}


def sources_match(table: dict) -> bool:
    import hashlib
    for rel, digest in table.items():
        with open(os.path.join(ROOT, rel), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest()[:16] != digest:
                return False
    return True


def values_per_site(solver: str) -> dict:
    """Algorithmic device traffic per lattice site of one launch of each single-kernel
    timing class, in values of the working precision.  collide_stream reads 27
    distributions + phi1, phi2, psi' and writes 27; phase reads 18 distributions and writes
    phi1, phi2, mu_r; the finest-level tile smoother reads psi' and mu_r and writes psi'
    (its right-hand side is formed from H0 and mu_r in registers); the fused prolongation +
    post-smoothing also reads the coarse correction (a quarter plane).  An SOR sweep reads
    mu_r and psi' and writes psi'.  Composite classes (a V-cycle, a convergence test) have
    no single-kernel figure."""
    v = {"collide_stream": 57.0, "phase": 21.0, "mg_smooth0": 3.0, "mg_post0": 3.25}
    if solver == "sor":
        v["potential_iter"] = 3.0
        v["residual"] = 2.0
    return v


def step_bytes_per_site(esz: int, cycles: float, solver: str, extrapolate: int, smooth: int = 1) -> float:
    """Algorithmic HBM bytes per lattice site of one whole coupled step (every launch, each
    plane counted once per pass, tile halos and re-reads not counted).  Values are esz bytes;
    the multigrid's coarse levels are FP32 and level l holds 4^-l of the sites.
    collide-and-stream 57 values; phase moments 18 read + 3 written; warm start (psi' and the
    three history planes written, psi' and two of them read, the third too for the cubic
    start) 7, or 8 when cubic; mu_r read once for the coarse mu of all
    levels (FP32 writes: sum 4 * 4^-l = 4/3 B).  A V-cycle on the finest level: `smooth`
    pre-smoothing launches of 3 (psi', mu_r read, result written), restriction fused with the
    level-1 smoothing 2 read + 2 B of FP32 writes (f and u of level 1), `smooth`
    post-smoothing launches of 3, the first also reading the level-1 correction (1 B); every
    coarse level (one launch down, one up) repeats the single-launch pattern in FP32 on 4^-l
    of the sites: sum_l 8 * 4 * 4^-l = 32/3 B.  An SOR sweep: mu_r and psi' read, psi' written; a
    residual test every sweep adds two reads."""
    b = (57 + 21) * esz + ((8 if extrapolate == 3 else 7) * esz if extrapolate else 0)
    if solver == "mg":
        b += esz + 4.0 / 3.0 + cycles * ((6 * smooth + 2) * esz + 3 + 32.0 / 3.0)
    else:
        b += cycles * 3 * esz
    return b


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(steps: int, bond: float, tol: float) -> dict:
    """The oracle beside the headline: the same 2048 x 512 channel and Bo_m, FP64, its
    potential by four-colour SOR warm-started from the previous step's psi' to the same
    max |L(psi0 + psi')| <= tol H0, built on this machine with -O3 -march=native and its row
    loops shared out by OpenMP over every core it is given.  Set-up (not timed): initial
    state, the initial potential solve from zero and one step; then `steps` timed steps."""
    import math

    import oracle.oracle as oo
    oo.use_fast_build()
    from fcd_inputs import single_channel_large
    from oracle import OracleSim, OracleSolver
    w = single_channel_large(bond=bond)
    omega = 2.0 / (1.0 + math.sin(math.pi / (w.ny + 1)))
    s = OracleSim(w, OracleSolver.sor(omega, tol, 1 << 30, 20))
    t0 = time.perf_counter()
    s.init_droplet(solve=False)
    assert s.solve_potential() == 0
    assert s.step(1) == 0
    t_setup = time.perf_counter() - t0
    sweeps = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        assert s.step(1) == 0
        sweeps += s.sweeps
    dt = time.perf_counter() - t0
    threads = oo.lib().orc_threads()
    log(f"bench: cpu baseline {steps} steps in {dt:.1f} s after {t_setup:.1f} s of set-up, {threads} threads")
    return {"value": round(w.sites * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{steps} coupled steps of {w.name} at Bo_m={bond:g}, FP64, potential by four-colour "
                      f"SOR to {tol:g} H0 warm-started from the previous step ({sweeps / steps:.0f} sweeps per "
                      f"step), after set-up; oracle built -O3 -march=native with OpenMP rows on {threads} threads; "
                      f"{dt:.1f} s timed"}


def batched_sweep(torch, steps: int, seq_steps: int) -> dict:
    """The 64-channel regime sweep (ny ~ U{64..256}, nx = 4 ny) as one FP32 batch and, for
    the gain at equal precision, as one FP64 batch at the single channels' tolerance, both
    with the batched multigrid (one finest sweep each way; quadratic warm start in FP32, cubic
    in FP64), against the same channels run
    one after another as single FP64 channels on this GPU (multigrid, two finest sweeps, cubic
    warm start).
    The FP32 batch with its tuned four-colour SOR is timed too (the batch's other solver).
    The rates are extrapolated to the sweep's 10k steps per channel from timed windows.
    Tuners run before the timed windows and are not part of them."""
    from fcd_inputs import regime_sweep_batch
    from paper_2410_11129_amd import fcd
    from paper_2410_11129_amd.sim import Batch, Channel
    ws = regime_sweep_batch()
    nsteps_target = ws[0].steps
    sites = sum(w.sites for w in ws)

    def timed(bt, n):
        bt.init_droplets()
        bt.step(8)  # past the start-up transient
        torch.cuda.synchronize()
        it0 = bt.stats()[1]
        t0 = time.perf_counter()
        bt.step(n)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        return dt, (bt.stats()[1] - it0) / n

    mg = dict(solver=fcd.FCD_SOLVER_MG, smooth=1)
    bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5, **mg)
    dt_batch, cyc32 = timed(bt, steps)
    bt.close()
    # FP64 with the cubic warm start, as the sequential channels (in FP32 its coefficients
    # amplify the solve's rounding and the quadratic start is faster)
    bt = Batch(ws, precision=fcd.FCD_FP64, tol=1e-10, extrapolate=3, **mg)
    dt_batch64, cyc64 = timed(bt, max(1, steps // 4))
    bt.close()
    # the FP32 batch with its SOR solver, factors and launch schedule tuned first
    bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5)
    bt.init_droplets()
    bt.step(8)
    bt.tune_omega(4)
    bt.init_droplets()
    rows, block, fused, tail_fused, tail_after = bt.autotune(3)
    bt.step(4)
    torch.cuda.synchronize()
    it0 = bt.stats()[1]
    t0 = time.perf_counter()
    bt.step(steps)
    torch.cuda.synchronize()
    dt_sor = (time.perf_counter() - t0) / steps
    sweeps = (bt.stats()[1] - it0) / steps
    bt.close()
    del bt
    seq = 0.0
    for w in (ws if seq_steps > 0 else []):
        ch = Channel(w, tol=1e-10, smooth=2, extrapolate=3)
        ch.init_droplet()
        ch.step(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(seq_steps)
        torch.cuda.synchronize()
        seq += (time.perf_counter() - t0) / seq_steps
        ch.close()
    iph = lambda dt: len(ws) / (nsteps_target * dt) * 3600.0  # noqa: E731
    seq_iph = len(ws) / (nsteps_target * seq) * 3600.0 if seq_steps > 0 else None
    return {"channels": len(ws), "sites": sites, "steps_per_channel": nsteps_target,
            "solver": "batched multigrid",
            "batch_fp32_ms_per_step": round(dt_batch * 1e3, 4), "batch_MLUPS": round(sites / dt_batch / 1e6, 1),
            "batch_fp32_vcycles_per_step": round(cyc32, 2),
            "instances_per_hour_batch_fp32": round(iph(dt_batch), 1),
            "batch_fp64_ms_per_step": round(dt_batch64 * 1e3, 4),
            "batch_fp64_vcycles_per_step": round(cyc64, 2),
            "instances_per_hour_batch_fp64": round(iph(dt_batch64), 1),
            "instances_per_hour_sequential_fp64": round(seq_iph, 1) if seq_iph else None,
            "speedup": round(iph(dt_batch) / seq_iph, 2) if seq_iph else None,
            "speedup_fp64_batch": round(iph(dt_batch64) / seq_iph, 2) if seq_iph else None,
            "sor_fp32": {"ms_per_step": round(dt_sor * 1e3, 4), "sweeps_per_step": round(sweeps, 2),
                         "instances_per_hour": round(iph(dt_sor), 1),
                         "schedule": {"tile_rows": rows, "block_sweeps": block, "fused_sweeps": fused,
                                      "tail_fused_sweeps": tail_fused, "tail_after_sweeps": tail_after}},
            "sample": f"batch: {steps} timed steps (FP64 {max(1, steps // 4)}); sequential: {seq_steps} timed "
                      f"steps per channel"}


def regime_accuracy(torch, stride: int, steps: int) -> dict:
    """Accuracy of the FP32 regime batch at the sweep's full horizon: every `stride`-th of the
    64 regime channels run as one FP32 batch (tol 1e-5) and, one after another, as single
    FP64 channels (tol 1e-10), `steps` steps each; D_o, D_i and max / mean |d phi| at the end
    (the stated bars: 1e-3 on D, 1e-4 on phi).  Not part of the default run (minutes)."""
    import numpy as np

    from fcd_inputs import regime_sweep_batch
    from paper_2410_11129_amd import fcd
    from paper_2410_11129_amd.sim import Batch, Channel
    ws = regime_sweep_batch(steps=steps)[::stride]
    bt = Batch(ws, precision=fcd.FCD_FP32, tol=1e-5)
    bt.init_droplets()
    bt.step(steps)
    d32 = bt.deformation()
    rows = []
    for k, w in enumerate(ws):
        m32 = bt.moments(k, fcd.FCD_M_PHI1 | fcd.FCD_M_PHI2)
        ch = Channel(w, tol=1e-10)
        ch.init_droplet()
        ch.step(steps)
        d64 = ch.deformation()
        m64 = ch.moments(fcd.FCD_M_PHI1 | fcd.FCD_M_PHI2)
        ch.close()
        dphi = [np.abs(m32[q] - m64[q]) for q in ("phi1", "phi2")]
        rows.append({"channel": w.name, "nx": w.nx, "ny": w.ny, "bond": round(w.bond, 3),
                     "capillary": round(w.capillary, 4), "dD_o": float(f"{abs(d32[k][0] - d64[0]):.3e}"),
                     "dD_i": float(f"{abs(d32[k][1] - d64[1]):.3e}"),
                     "max_dphi": float(f"{max(d.max() for d in dphi):.3e}"),
                     "mean_dphi": float(f"{max(d.mean() for d in dphi):.3e}")})
        log(f"bench: regime accuracy {rows[-1]}")
    bt.close()
    return {"steps": steps, "channels": rows,
            "max_dD": max(max(r["dD_o"], r["dD_i"]) for r in rows),
            "max_dphi": max(r["max_dphi"] for r in rows), "max_mean_dphi": max(r["mean_dphi"] for r in rows)}


def adjoint_ratio(torch, steps: int, every: int) -> dict:
    """Cost of the checkpointed gradient on the 512 x 128 channel (shell mu_r = 2, field at
    30 degrees, Bo_m = 1), FP64: plain forward of `steps` steps, then the checkpointing
    forward and the reverse sweep (which recomputes every segment) of the same run."""
    from fcd_inputs import adjoint_channel
    from paper_2410_11129_amd import fcd
    from paper_2410_11129_amd.adjoint import AdjointRun, theta_of
    from paper_2410_11129_amd.sim import Channel
    w = adjoint_channel(steps=steps)
    ch = Channel(w, tol=1e-10)
    ch.init_droplet()
    ch.step(20)  # warm-up
    ch.init_droplet()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    run = AdjointRun(ch, steps, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D = run.forward(theta_of(w))
    torch.cuda.synchronize()
    t_cfwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = run.backward([1.0, 0.0])
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    nbytes = run.work.numel()
    ch.close()
    return {"workload": f"{w.name}_fp64", "steps": steps, "ckpt_every": every,
            "forward_s": round(t_fwd, 4), "checkpointed_forward_s": round(t_cfwd, 4), "backward_s": round(t_bwd, 4),
            "adjoint_forward_ratio": round((t_cfwd + t_bwd) / t_fwd, 3),
            "backward_forward_ratio": round(t_bwd / t_fwd, 3), "work_MB": round(nbytes / 1e6, 1),
            "D_o": D[0], "dDo_dtheta": dict(zip(("H0", "alpha", "u_ref", "sigma12", "sigma13", "sigma23"), g))}


def batched_adjoint(torch, steps: int, every: int) -> dict:
    """The 32 adjoint channels (256 x 64, Bo_m ~ U(0, 6), Ca ~ U(0.05, 0.2), random field
    angle) as one batch: checkpointed forward + batched reverse sweep of `steps` steps, in
    FP32 and in FP64, the forward and adjoint potentials by the batched multigrid, against the
    single-channel FP64 adjoint of the first two channels run one after another
    (per-instance rates)."""
    from fcd_inputs import adjoint_batch
    from paper_2410_11129_amd import fcd
    from paper_2410_11129_amd.adjoint import AdjointRun, BatchAdjointRun, theta_of
    from paper_2410_11129_amd.sim import Batch, Channel
    ws = adjoint_batch(steps=steps)
    seq = 0.0
    gs = []
    for w in ws[:2]:
        ch = Channel(w, tol=1e-10)
        r1 = AdjointRun(ch, steps, every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r1.forward(theta_of(w))
        gs.append(r1.backward((1.0, 0.0)))
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
        ch.close()
    per_seq = seq / 2
    # conditioning of the horizon: channel 1's FP64 gradient again, its initial state
    # perturbed by a random relative 6e-8 (the size of FP32 rounding)
    import numpy as np
    ch = Channel(ws[1], tol=1e-10)
    r1 = AdjointRun(ch, steps, every)
    ch.init_droplet()
    st = ch.state()
    ch.write_state(st * (1.0 + 6e-8 * np.random.default_rng(5).uniform(-1.0, 1.0, st.shape)))
    fcd.fcd_adjoint_forward(ch.h, steps, every, r1.work.data_ptr())
    gp = fcd.fcd_adjoint_backward(ch.h, [1.0, 0.0])
    ch.close()
    del r1
    sens = max(abs(gp[q] - gs[1][q]) / abs(gs[1][q]) for q in (0, 1))
    out = {"channels": len(ws), "steps": steps, "ckpt_every": every,
           "s_per_gradient_sequential_fp64": round(per_seq, 4),
           "fp64_gradient_change_under_6e-8_perturbation": float(f"{sens:.3e}")}
    for name, prec, tol, sm in (("fp32", fcd.FCD_FP32, 1e-5, 1), ("fp64", fcd.FCD_FP64, 1e-10, 2)):
        bt = Batch(ws, precision=prec, tol=tol, solver=fcd.FCD_SOLVER_MG, smooth=sm)
        bt.init_droplets()
        run = BatchAdjointRun(bt, steps, every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.forward()
        g = run.backward([(1.0, 0.0)] * len(ws))
        torch.cuda.synchronize()
        dt_batch = time.perf_counter() - t0
        bt.close()
        del run
        per_batch = dt_batch / len(ws)
        rel = [abs(g[k][q] - gs[k][q]) / abs(gs[k][q]) for k in range(2) for q in (0, 1)]
        # the same error relative to the instance's (H0, alpha) gradient norm, H0-scaled
        rel_norm = []
        for k in range(2):
            sc = (ws[k].H0, 1.0)
            norm = max(abs(gs[k][q] * sc[q]) for q in (0, 1))
            rel_norm += [abs(g[k][q] - gs[k][q]) * sc[q] / norm for q in (0, 1)]
        out[name] = {"batch_s": round(dt_batch, 3), "s_per_gradient": round(per_batch, 4),
                     "speedup_vs_sequential_fp64": round(per_seq / per_batch, 2),
                     "max_rel_diff_dDo_dH0_dalpha_vs_fp64": float(f"{max(rel):.3e}"),
                     "max_diff_rel_to_gradient_norm": float(f"{max(rel_norm):.3e}")}
        torch.cuda.empty_cache()
    return out


def quasi_static(torch, steps: int) -> dict:
    """The 2048 x 512 FP64 channel (Bo_m = 2, multigrid to 1e-10 with the headline's solver
    settings) with the potential solved every K steps and held in between (an option, not
    the paper's every-step coupling):
    throughput for K = 4 and 8, and how far phi1 and D_o drift from the every-step run over
    the same `steps` steps from the same state."""
    from fcd_inputs import single_channel_large
    from paper_2410_11129_amd import fcd
    from paper_2410_11129_amd.sim import Channel
    w = single_channel_large(bond=2.0)
    ref = None
    out = {"workload": "channel_2048x512_fp64_bo2", "steps": steps}
    for K in (1, 4, 8):
        ch = Channel(w, tol=1e-10, every=K, extrapolate=3, smooth=2)
        ch.init_droplet()
        ch.solve_potential(1e-10)
        ch.step(8)  # every K divides 8: the timed window starts on a solve step
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        phi1 = ch.moments(fcd.FCD_M_PHI1)["phi1"]
        D = ch.deformation()[0]
        ch.close()
        if ref is None:
            ref = (phi1, D)
            out["every_1_MLUPS"] = round(w.sites / dt / 1e6, 1)
            continue
        out[f"every_{K}"] = {"MLUPS": round(w.sites / dt / 1e6, 1),
                             "max_abs_dphi1_vs_every_step": float(f"{abs(phi1 - ref[0]).max():.3e}"),
                             "dD_o_vs_every_step": float(f"{D - ref[1]:.3e}")}
    return out


def open_channel(torch, steps: int) -> dict:
    """The paper's open-channel set-up (900 x 150, Eq. 37 inlet, convective outlet; Bo_m = 2,
    ferrofluid shell, multigrid to 1e-10), FP64: throughput with the end-column boundary
    launches against the same lattice and droplet run as a periodic channel under the
    equivalent body force.  The hierarchy of 900 x 150 runs through odd levels (450 x 75,
    225 x 37, 113 x 19, then a tail of 57 x 9, 29 x 4, 15 x 2); two finest-level sweeps each
    way were the fastest of 1-6 measured on this lattice."""
    from fcd_inputs import channel_drive, open_channel_paper
    from paper_2410_11129_amd.sim import Channel
    w = open_channel_paper(bond=2.0)
    periodic = w.replace(u_inlet=None, drive_G=channel_drive(w.u_inlet, w.rho[2], w.tau[2], w.ny))
    out = {"workload": "open_channel_900x150_fp64_bo2", "steps": steps}
    for name, ww in (("open", w), ("periodic", periodic)):
        ch = Channel(ww, tol=1e-10, smooth=2, extrapolate=3)
        ch.init_droplet()
        ch.solve_potential(1e-10)
        ch.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"{name}_MLUPS"] = round(ww.sites / dt / 1e6, 1)
        out[f"{name}_ms_per_step"] = round(dt * 1e3, 4)
        out[f"{name}_vcycles_per_step"] = round(ch.stats()[1] / (steps + 20), 2)
        ch.close()
    return out


def copy_bandwidth_gbs(torch) -> float:
    n = 1 << 28  # 2 GiB of float64 each way
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    return 2 * n * 8 / dt / 1e9


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    # steps run after the initial state and before the warm-up, so that the timed window
    # lies in the developed run rather than its start-up transient (the initial state has
    # p* = 0 and no Laplace pressure, and its acoustic transient makes the first ~60 steps'
    # potential solves need up to 11 V-cycles against 4-5 later); the start-up window
    # (right after the initial state) is measured too and reported beside it
    ap.add_argument("--preroll", type=int, default=500)
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64")
    ap.add_argument("--bond", type=float, default=2.0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--solver", choices=("mg", "sor"), default="mg")
    # finest-level smoothing sweeps (one launch each) before and after each coarse
    # correction: 3 needs 2.15 V-cycles per step against 4.0 with 1 (measured, 2048 x 512
    # FP64 Bo_m = 2, steps 501-540: 0.531 against 0.632 ms/step; 4, 5, 6: 0.556, 0.601, 0.649)
    ap.add_argument("--smooth", type=int, default=2)
    ap.add_argument("--coarse-sweeps", type=int, default=2)
    ap.add_argument("--check-every", type=int, default=1)
    ap.add_argument("--no-extrapolate", action="store_true")  # the same as --extrapolate 0
    ap.add_argument("--extrapolate", type=int, choices=(0, 1, 2, 3), default=3)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--sequential-steps", type=int, default=20)  # 0: no sequential comparator
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--regime-accuracy", type=int, default=0,
                    help="also compare every N-th regime channel, FP32 batch against FP64 single, at 10k steps")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-ckpt", type=int, default=100)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--quasi-static-steps", type=int, default=400)
    ap.add_argument("--no-quasi-static", action="store_true")
    ap.add_argument("--open-channel-steps", type=int, default=1000)
    ap.add_argument("--no-open-channel", action="store_true")
    ap.add_argument("--batch-adjoint-steps", type=int, default=3000)
    ap.add_argument("--batch-adjoint-ckpt", type=int, default=150)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not built.", file=sys.stderr)
        return 2

    import torch
    from fcd_inputs import single_channel_large
    from paper_2410_11129_amd import fcd
    from paper_2410_11129_amd.sim import Channel

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = fcd.FCD_FP64 if args.precision == "fp64" else fcd.FCD_FP32
    esz = 8 if prec == fcd.FCD_FP64 else 4
    tol = args.tol if prec == fcd.FCD_FP64 else max(args.tol, 1e-5)
    w = single_channel_large(bond=args.bond)
    log(f"bench: {w.name} {w.nx}x{w.ny} {args.precision} Bo_m={args.bond} H0={w.H0:.5g} tol={tol:g}")
    solver = fcd.FCD_SOLVER_MG if args.solver == "mg" else fcd.FCD_SOLVER_SOR
    extrap = 0 if args.no_extrapolate else args.extrapolate
    ch = Channel(w, precision=prec, solver=solver, tol=tol, check_every=args.check_every if args.solver == "mg" else 8,
                 max_iters=1 << 30, smooth=args.smooth, coarse_sweeps=args.coarse_sweeps,
                 extrapolate=extrap)
    ch.init_droplet()
    t0 = time.perf_counter()
    st, sw0, res0 = ch.solve_potential(tol, 1 << 30)
    log(f"bench: initial potential solve {sw0} iterations, residual {res0:.3e}, {time.perf_counter() - t0:.2f} s")

    def timed_window(live=False):
        """(seconds, potential iterations) of args.steps steps after args.warmup; live: the
        collide-and-stream launches of the timed steps record their own start and end
        (HIP events on the handle's stream), returned as a third item (ms, launches)."""
        ch.step(args.warmup)
        torch.cuda.synchronize()
        s0 = ch.stats()[1]
        if live:
            fcd.fcd_timing(ch.h, 2)
        t1 = time.perf_counter()
        ch.step(args.steps)
        torch.cuda.synchronize()
        out = (time.perf_counter() - t1, ch.stats()[1] - s0)
        if live:
            out += (fcd.fcd_timing_read(ch.h)["collide_stream"],)
            fcd.fcd_timing(ch.h, 0)
        return out

    done = 0
    startup = None
    if args.preroll > 0:
        dt0, sw_0 = timed_window()
        done = args.warmup + args.steps
        startup = {"steps_after_init": [args.warmup + 1, done], "ms_per_step": round(dt0 / args.steps * 1e3, 4),
                   "MLUPS": round(w.sites * args.steps / dt0 / 1e6, 3),
                   "potential_iters_per_step": round(sw_0 / args.steps, 2)}
        log(f"bench: start-up window {startup}")
        if args.preroll > done:
            ch.step(args.preroll - done)
            done = args.preroll
    dt, sweeps, live = timed_window(live=True)
    first = done + args.warmup + 1
    # per-kernel breakdown in a separate window: HIP events around every launch add host
    # work between launches and select the host-decided solve, so they stay out of the
    # timed steps above (which time only the collide-and-stream, by its own launches' events)
    prof_steps = max(1, min(args.steps, 20))
    fcd.fcd_timing(ch.h, True)
    ch.step(prof_steps)
    timing = fcd.fcd_timing_read(ch.h)
    fcd.fcd_timing(ch.h, False)
    d = ch.deformation()
    log(f"bench: {args.steps} steps in {dt:.3f} s, {sweeps / max(args.steps, 1):.2f} potential iterations/step, "
        f"D_o={d[0]:.5f} D_i={d[1]:.5f}; timing {timing}")

    sites = w.sites
    VALUES_PER_SITE = values_per_site(args.solver)
    mlups = sites * args.steps / dt / 1e6
    per_kind = {}
    for k, (ms, n) in timing.items():
        if n == 0:
            continue
        avg_s = ms / n / 1e3
        per_kind[k] = {"launches": n, "avg_us": round(avg_s * 1e6, 3), "ms_per_step": round(ms / prof_steps, 4)}
        if k in VALUES_PER_SITE:
            per_kind[k]["GBps"] = round(VALUES_PER_SITE[k] * esz * sites / avg_s / 1e9, 1)
    # Roofline of the dominant HBM-bound kernel, the fused collide-and-stream (rocprof: ~84 us of
    # the step's ~0.34 ms; the finest smoothing kernels follow at ~12 us per launch), timed by
    # HIP events that its own launches record during the timed steps.  The rest of the
    # potential solve is a chain of small coarse-level kernels bound by launch and dependency
    # latency, not by bandwidth, so no HBM roofline applies to them.
    dom = "collide_stream"
    traffic = None
    if prec == fcd.FCD_FP64 and (w.nx, w.ny) == (2048, 512) and sources_match(TRAFFIC_SOURCES):
        traffic = TRAFFIC_BYTES[dom]
    live_ms, live_n = live
    live_gbps = round(VALUES_PER_SITE[dom] * esz * sites / (live_ms / live_n / 1e3) / 1e9, 1)
    roof = {"bound": "hbm", "kernel": dom, "achieved": live_gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(live_gbps / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": VALUES_PER_SITE[dom] * esz * sites, "launches": live_n,
            "avg_us": round(live_ms / live_n * 1e3, 3)}
    cycles = sweeps / max(args.steps, 1)
    step_b = step_bytes_per_site(esz, cycles, args.solver, extrap, args.smooth)
    step_gbps = step_b * sites / (dt / args.steps) / 1e9
    kernel_ms = sum(per_kind[k]["ms_per_step"] for k in ("collide_stream", "phase") if k in per_kind)
    ms_step = dt / args.steps * 1e3
    out = {
        "metric": METRIC, "value": round(mlups, 3), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == fcd.FCD_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}_{args.precision}_bo{args.bond:g}", "nx": w.nx, "ny": w.ny,
                   "bond": args.bond, "potential_solver": args.solver, "potential_tol": tol,
                   "potential_iters_per_step": round(sweeps / args.steps, 2),
                   "timed_steps_after_init": [first, first + args.steps - 1]},
        "roofline": roof,
        # the whole step against HBM: algorithmic bytes of every launch (step_bytes_per_site)
        # over the timed step; the potential's share is everything but the collide-and-stream
        # and phase kernels (their per-kernel times from the event-timed window)
        "step_bytes_per_site": round(step_b, 1),
        "step_GBps": round(step_gbps, 1),
        "step_frac": round(step_gbps / HBM_PEAK_GBS, 4),
        "potential_share": round(max(0.0, ms_step - kernel_ms) / ms_step, 4),
        "kernels": per_kind,
    }
    if startup is not None:
        out["startup_window"] = startup
    try:
        out["copy_GBps_torch"] = round(copy_bandwidth_gbs(torch), 1)
    except Exception as e:  # noqa: BLE001
        log(f"bench: copy bandwidth probe failed: {e}")
    del ch
    if not args.no_batched:
        out["batched"] = batched_sweep(torch, args.batched_steps, args.sequential_steps)
        log(f"bench: batched {out['batched']}")
    if args.regime_accuracy > 0:
        out["regime_accuracy"] = regime_accuracy(torch, args.regime_accuracy, 10000)
    if not args.no_quasi_static:
        out["quasi_static"] = quasi_static(torch, args.quasi_static_steps)
        log(f"bench: quasi-static coupling {out['quasi_static']}")
    if not args.no_open_channel:
        out["open_channel"] = open_channel(torch, args.open_channel_steps)
        log(f"bench: open channel {out['open_channel']}")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio(torch, args.adjoint_steps, args.adjoint_ckpt)
        log(f"bench: adjoint {out['adjoint']}")
        out["batched_adjoint"] = batched_adjoint(torch, args.batch_adjoint_steps, args.batch_adjoint_ckpt)
        log(f"bench: batched adjoint {out['batched_adjoint']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, args.bond, args.tol)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
