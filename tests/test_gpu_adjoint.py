"""Hand-written adjoint of the coupled step (checkpointed) against reference gradients.

The gradient of J = a D_o + b D_i (the second-moment deformations that stand in for the
index of Eq. 42, after n steps from the compound droplet) with respect to
(H0, alpha, u_ref, sigma12, sigma13, sigma23) is compared with the FP64 oracle's
complex-step gradient (exact banded-Cholesky potential solve; exact to rounding, so the bar
is tight), and with Richardson-extrapolated central differences of (1) the GPU FP64 forward
and (2) the FP64 CPU oracle, to 1e-4 relative.
"""
import math
import sys

import numpy as np
import pytest

from fcd_inputs import Workload, channel_drive, h0_from_bond
from oracle import OracleSim
from oracle.oracle import complex_step_gradient

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_2410_11129_amd import fcd  # noqa: E402
from paper_2410_11129_amd.adjoint import AdjointRun, deformation, theta_of  # noqa: E402
from paper_2410_11129_amd.sim import Channel  # noqa: E402

A_O, A_I = 1.0, 0.5  # J = A_O D_o + A_I D_i
NSTEPS = 30
REL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_channel(H0=None, alpha=math.radians(30.0)):
    """96 x 32 channel, ferrofluid shell, three different surface tensions, field at 30 deg."""
    ny, tau3, u = 32, 0.8, 0.01
    s12, s13, s23 = 0.008, 0.012, 0.01
    rc, rs = 5.0, 9.0
    h0 = h0_from_bond(1.0, "shell", 1.0, rc, rs, s12, s23) if H0 is None else H0
    return Workload(name="adj_96x32", nx=96, ny=ny, tau=(tau3, tau3, tau3), chi=(0.0, 1.0, 0.0),
                    sigma12=s12, sigma13=s13, sigma23=s23, xi=4.0, H0=h0, alpha=alpha,
                    drive_G=channel_drive(u, 1.0, tau3, ny), xc=30.0, yc=15.3, r_core=rc, r_shell=rs,
                    u_ref=u)


def at(w, theta):
    H0, alpha, u, s12, s13, s23 = theta
    return w.replace(H0=H0, alpha=alpha, u_ref=u, sigma12=s12, sigma13=s13, sigma23=s23,
                     drive_G=channel_drive(u, w.rho[2], w.tau[2], w.ny))


def richardson(J, theta, k, rel):
    """Central difference of J along theta[k], extrapolated from steps h and h/2."""
    h = rel * (abs(theta[k]) if theta[k] != 0 else 1.0)

    def cd(hh):
        tp, tm = list(theta), list(theta)
        tp[k] += hh
        tm[k] -= hh
        return (J(tp) - J(tm)) / (2 * hh)

    d1, d2 = cd(h), cd(h / 2)
    return (4 * d2 - d1) / 3


def gpu_J(w, tol=1e-13):
    ch = Channel(w, tol=tol, extrapolate=0)

    def J(theta):
        ch.set_workload(at(w, theta))
        ch.init_droplet()
        ch.step(NSTEPS)
        d = ch.deformation()
        return A_O * d[0] + A_I * d[1]

    return J, ch


def oracle_J(w):
    def J(theta):
        s = OracleSim(at(w, theta))
        s.init_droplet(solve=False)
        assert s.step(NSTEPS) == 0
        d = s.diagnostics()
        return A_O * d[0] + A_I * d[1]

    return J


def adjoint_grad(w, every=8, tol=1e-13, precision=fcd.FCD_FP64):
    ch = Channel(w, precision=precision, tol=tol)
    run = AdjointRun(ch, NSTEPS, every)
    D = run.forward(theta_of(w))
    g = run.backward([A_O, A_I])
    return D, np.array(g), ch


def check(g_adj, g_ref, theta, J0, what):
    # compare the dimensionless sensitivities theta_k dJ/dtheta_k; alpha is taken in
    # units of one radian
    for k in range(6):
        sc = abs(theta[k]) if k != 1 else 1.0
        a, r = g_adj[k] * sc, g_ref[k] * sc
        tol = REL * abs(r) + 1e-9 * abs(J0)
        say(f"  {what} k={k}: adjoint {g_adj[k]:.10e} reference {g_ref[k]:.10e} rel {abs(a - r) / max(abs(r), 1e-300):.2e}")
        assert abs(a - r) <= tol, (what, k, g_adj[k], g_ref[k])


def test_adjoint_matches_gpu_central_differences():
    w = small_channel()
    say(f"case adjoint vs GPU FD, {w.nx}x{w.ny}, {NSTEPS} steps, ckpt 8")
    theta = theta_of(w)
    D, g, ch = adjoint_grad(w)
    J, ch2 = gpu_J(w)
    J0 = J(theta)
    assert abs(J0 - (A_O * D[0] + A_I * D[1])) < 1e-12
    fd = np.array([richardson(J, theta, k, 1e-3) for k in range(6)])
    check(g, fd, theta, J0, "gpu-fd")
    ch.close()
    ch2.close()


def test_adjoint_matches_oracle_central_differences():
    w = small_channel()
    say(f"case adjoint vs oracle FD, {w.nx}x{w.ny}, {NSTEPS} steps")
    theta = theta_of(w)
    D, g, ch = adjoint_grad(w)
    J = oracle_J(w)
    J0 = J(theta)
    assert abs(J0 - (A_O * D[0] + A_I * D[1])) < 1e-11
    fd = np.array([richardson(J, theta, k, 1e-3) for k in range(6)])
    check(g, fd, theta, J0, "oracle-fd")
    ch.close()


def cs_check(w, nsteps, every, rel, extrapolate=2):
    theta = theta_of(w)
    ch = Channel(w, tol=1e-13, extrapolate=extrapolate)
    run = AdjointRun(ch, nsteps, every)
    D = run.forward(theta)
    g = np.array(run.backward([A_O, A_I]))
    ch.close()
    J0, g_cs = complex_step_gradient(w, nsteps, (A_O, A_I))
    assert abs(J0 - (A_O * D[0] + A_I * D[1])) <= 1e-11 * max(1.0, abs(J0)), (J0, D)
    sc = np.array([abs(theta[k]) if k != 1 else 1.0 for k in range(6)])
    worst = 0.0
    for k in range(6):
        a, r = g[k] * sc[k], g_cs[k] * sc[k]
        e = abs(a - r) / abs(r)
        worst = max(worst, e)
        say(f"  k={k}: adjoint {g[k]:.14e} complex step {g_cs[k]:.14e} rel {e:.2e}")
        assert abs(a - r) <= rel * abs(r), (k, g[k], g_cs[k])
    return worst


def test_adjoint_matches_oracle_complex_step_gradient():
    """Every component within 1e-10 relative of the oracle's complex-step derivative: both
    sides are FP64 and the GPU's potential is solved to 1e-13 H0, so what separates them is
    rounding carried through 30 steps and the solve's tolerance (measured on the box: 8e-12
    at worst, on dJ/du_ref)."""
    w = small_channel()
    say(f"case adjoint vs oracle complex step, {w.nx}x{w.ny}, {NSTEPS} steps, ckpt 8")
    cs_check(w, NSTEPS, 8, 1e-10)


def test_adjoint_matches_oracle_complex_step_gradient_over_300_steps():
    """The same over 300 steps with a checkpoint every 25 (the trajectory has moved the
    droplet by a few nodes; rounding is carried ten times longer; measured 4.5e-13)."""
    w = small_channel()
    say(f"case adjoint vs oracle complex step, {w.nx}x{w.ny}, 300 steps, ckpt 25")
    cs_check(w, 300, 25, 1e-10)


def test_adjoint_with_cubic_warm_start_matches_oracle_complex_step_gradient():
    """The forward's solves started from the cubic extrapolation in time (the checkpoints
    record the third history plane, so recomputed segments repeat the forward exactly; the
    adjoint solves start at most quadratically)."""
    w = small_channel()
    say(f"case adjoint cubic start vs oracle complex step, {w.nx}x{w.ny}, {NSTEPS} steps, ckpt 8")
    cs_check(w, NSTEPS, 8, 1e-10, extrapolate=3)


def test_checkpoint_interval_does_not_change_gradient():
    w = small_channel()
    say("case adjoint checkpoint intervals 1, 7, 30")
    gs = [adjoint_grad(w, every=e)[1] for e in (1, 7, NSTEPS)]
    for g in gs[1:]:
        assert np.abs(g - gs[0]).max() <= 1e-12 * np.abs(gs[0]).max()


def test_backward_leaves_final_state_and_autograd_function():
    w = small_channel()
    say("case adjoint through torch.autograd")
    ch = Channel(w, tol=1e-13)
    run = AdjointRun(ch, NSTEPS, 8)
    theta = torch.tensor(theta_of(w), dtype=torch.float64, requires_grad=True)
    D = deformation(theta, run)
    s_fwd = ch.state()
    J = A_O * D[0] + A_I * D[1]
    J.backward()
    assert np.array_equal(ch.state(), s_fwd)
    _, g, ch2 = adjoint_grad(w)
    assert np.abs(theta.grad.numpy() - g).max() <= 1e-13 * np.abs(g).max()
    ch.close()
    ch2.close()


def test_zero_field_gradients():
    """At H0 = 0 the Kelvin force is quadratic in H0: dJ/dH0 = dJ/dalpha = 0."""
    w = small_channel(H0=0.0)
    say("case adjoint at H0 = 0")
    theta = theta_of(w)
    D, g, ch = adjoint_grad(w)
    assert g[0] == 0.0 and g[1] == 0.0
    J, ch2 = gpu_J(w)
    J0 = J(theta)
    fd = np.array([0.0, 0.0] + [richardson(J, theta, k, 1e-3) for k in range(2, 6)])
    check(g, fd, theta, J0, "gpu-fd H0=0")
    ch.close()
    ch2.close()


def test_fp32_adjoint_tracks_fp64():
    w = small_channel()
    say("case adjoint fp32 vs fp64")
    _, g64, c1 = adjoint_grad(w)
    _, g32, c2 = adjoint_grad(w, tol=1e-5, precision=fcd.FCD_FP32)
    theta = theta_of(w)
    sc = np.array([abs(theta[k]) if k != 1 else 1.0 for k in range(6)])
    err = np.abs((g32 - g64) * sc).max() / np.abs(g64 * sc).max()
    say(f"  fp32 relative gradient error {err:.2e}")
    assert err < 1e-3
    c1.close()
    c2.close()


def test_adjoint_at_the_512x128_workload_matches_central_differences():
    """The adjoint workload itself: 512 x 128 channel (shell r = 30, core r = 15, shell
    mu_r = 2, Bo_m = 1, field at 30 degrees), 2000 steps, a checkpoint every 100 steps, the
    gradient of the terminal shell deformation D_o against central differences of the GPU
    FP64 forward with h = 1e-6 relative, Richardson-extrapolated from h and h/2, the
    potential solved to 1e-13 H0 from the previous step's psi' (no extrapolation, so the
    forward is a smooth function of the parameters).  Each component within 1e-4 relative
    of its own value, with an absolute floor of 1e-4 of the largest sensitivity for the
    nearly vanishing dD_o/dsigma13 (core and ambient meet only through the tanh tails)."""
    from fcd_inputs import adjoint_channel
    w = adjoint_channel(steps=2000)
    n, every = 2000, 100
    say(f"case adjoint vs GPU FD, {w.nx}x{w.ny}, {n} steps, ckpt {every}")
    theta = theta_of(w)
    ch = Channel(w, tol=1e-13, extrapolate=0)
    run = AdjointRun(ch, n, every)
    D = run.forward(theta)
    g = np.array(run.backward([1.0, 0.0]))
    ch.close()
    ch2 = Channel(w, tol=1e-13, extrapolate=0)

    def J(th):
        ch2.set_workload(at(w, th))
        ch2.init_droplet()
        ch2.step(n)
        return ch2.deformation()[0]

    J0 = J(theta)
    assert abs(J0 - D[0]) < 1e-12 * max(1.0, abs(D[0])), (J0, D[0])
    fd = np.array([richardson(J, theta, k, 1e-6) for k in range(6)])
    ch2.close()
    sc = np.array([abs(theta[k]) if k != 1 else 1.0 for k in range(6)])
    floor = 1e-4 * np.abs(fd * sc).max()
    for k in range(6):
        a, r = g[k] * sc[k], fd[k] * sc[k]
        say(f"  k={k}: adjoint {g[k]:.10e} fd {fd[k]:.10e} rel {abs(a - r) / max(abs(r), 1e-300):.2e}")
        assert abs(a - r) <= 1e-4 * abs(r) + floor, (k, g[k], fd[k])
