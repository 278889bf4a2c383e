"""Workload recipes: channel sizes, droplet geometry and lattice parameters.

The paper (arXiv:2410.11129, Sec. 2.5, Table 1) states its set-up in dimensionless
groups: radius ratio, density and kinematic-viscosity ratios (Eq. 39), the capillary
number (Eq. 40) and the magnetic Bond number (Eq. 41).  The helpers here turn those
groups into lattice parameters; they are the recipe of the synthetic inputs, not a part
of the time step.  Choices the paper leaves open are stated where they are made:

* the periodic channel is driven by a uniform body force sized so that the Poiseuille
  profile between halfway-bounce-back walls peaks at ``u_ref`` (the paper drives an
  open channel by an inlet profile whose peak, Eq. 37 as printed, is ``u_avg``);
* ``u_ref`` (the velocity scale of Eq. 40) is that peak;
* mu0 = 1 in lattice units (only mu0 * H0^2 enters the force, Eq. 7);
* where a workload names no ambient relaxation time, tau_3 = 0.2 and u_ref = 0.01;
  where it names no susceptibility, the ferrofluid has chi = 1 (Sec. 2.5, after Eq. 41);
* the interface normal n = grad phi / |grad phi| is undefined where grad phi = 0; it is
  regularised as grad phi / sqrt(|grad phi|^2 + eps_n^2) with eps_n = 1e-4.  A smaller
  eps_n lets rounding noise in grad phi at extremum points of phi (droplet centres) set
  the direction of the counter-diffusion flux: in FP64 two correct implementations drift
  apart (1.9e-5 in phi over 1000 steps of the 200 x 50 channel after a one-ulp
  perturbation at eps_n = 1e-12, 1e-14 at 1e-4), and in FP32, where that noise is ~1e-7,
  phi moves by up to 3e-6 / 2.8e-5 / 1.2e-4 within 20 steps of the regime channels at
  eps_n = 1e-4 / 3e-5 / 1e-5, and the FP32 batched adjoint over 60 steps leaves its 1e-3
  bar at 3e-5 (3e-3 on one channel).  The price is a bias in the far tails of the
  profiles, where |grad phi| ~ phi ~ eps_n, and with them the second moments: against the
  eps_n -> 0 limit, D moves by 1.0e-3 / 3.6e-4 / 1.3e-4 over those 1000 steps at the same
  three values.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

CS2 = 1.0 / 3.0


@dataclasses.dataclass
class Workload:
    """One channel: lattice, materials, field, drive and the initial droplet."""

    name: str
    nx: int
    ny: int
    rho: Tuple[float, float, float] = (1.0, 1.0, 1.0)  # core, shell, ambient
    tau: Tuple[float, float, float] = (0.8, 0.8, 0.8)
    chi: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    sigma12: float = 0.01
    sigma13: float = 0.01
    sigma23: float = 0.01
    eta: float = 0.0
    xi: float = 5.0
    mobility: float = 0.3
    H0: float = 0.0
    alpha: float = 0.0  # radians
    mu0: float = 1.0
    drive_G: float = 0.0
    grav: Tuple[float, float] = (0.0, 0.0)
    eps_n: float = 1e-4  # normal regularisation, see the module docstring
    xc: float = 0.0
    yc: float = 0.0
    r_core: float = 0.0
    r_shell: float = 0.0
    steps: int = 0
    u_ref: float = 0.01
    ferro: str = "shell"
    bond: float = 0.0
    capillary: Optional[float] = None
    u_inlet: Optional[float] = None  # open channel: u_avg of Eq. 37; None: periodic channel

    @property
    def sites(self) -> int:
        return self.nx * self.ny

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def channel_drive(u_peak: float, rho3: float, tau3: float, ny: int) -> float:
    """Body force density G whose Poiseuille profile between walls at y = -1/2 and
    y = ny - 1/2 peaks at u_peak: u(y) = G/(2 rho nu) (y+1/2)(ny-1/2-y), nu = c_s^2 tau."""
    nu3 = CS2 * tau3
    return 8.0 * rho3 * nu3 * u_peak / float(ny * ny)


def sigma_from_capillary(ca: float, rho3: float, tau3: float, u_ref: float) -> float:
    """sigma_23 from Ca = rho_3 nu_3 u / sigma_23 (Eq. 40)."""
    return rho3 * CS2 * tau3 * u_ref / ca


def h0_from_bond(bond: float, ferro: str, chi_ferro: float, r_core: float, r_shell: float,
                 sigma12: float, sigma23: float, mu0: float = 1.0) -> float:
    """H0 from the magnetic Bond number, Eq. 41 solved for H0."""
    if bond <= 0.0:
        return 0.0
    if ferro == "core":
        return math.sqrt(2.0 * bond * sigma12 / (mu0 * chi_ferro * r_core))
    if ferro == "shell":
        return math.sqrt(2.0 * bond * (sigma12 * r_core + sigma23 * r_shell)
                         / (mu0 * chi_ferro * (r_shell ** 2 - r_core ** 2)))
    raise ValueError(f"ferro must be 'core' or 'shell', got {ferro!r}")


def _chi(ferro: str, chi_value: float) -> Tuple[float, float, float]:
    return (chi_value, 0.0, 0.0) if ferro == "core" else (0.0, chi_value, 0.0)


def single_channel_small(bond: float = 1.0, steps: int = 1000) -> Workload:
    """200 x 50 periodic channel, shell r = 12, core r = 6 centred at (50, 25),
    interface width 4, equal densities, tau = 0.8 in every phase, equal surface
    tensions 0.01, ferrofluid shell mu_r = 2, field along x, drive peaking at 0.01."""
    nx, ny, rs, rc = 200, 50, 12.0, 6.0
    sig = 0.01
    return Workload(
        name="channel_200x50_fp64", nx=nx, ny=ny, tau=(0.8, 0.8, 0.8), chi=_chi("shell", 1.0),
        sigma12=sig, sigma13=sig, sigma23=sig, xi=4.0,
        H0=h0_from_bond(bond, "shell", 1.0, rc, rs, sig, sig), alpha=0.0,
        drive_G=channel_drive(0.01, 1.0, 0.8, ny), xc=50.0, yc=25.0, r_core=rc, r_shell=rs,
        steps=steps, u_ref=0.01, ferro="shell", bond=bond)


def single_channel_large(bond: float = 2.0, steps: int = 20000) -> Workload:
    """2048 x 512 channel, shell r = 80, core r = 40, Ca = 0.1, densities 2:1:1 and
    kinematic viscosities 5:1:1 (core:shell:ambient), ferrofluid core mu_r = 3,
    field at 90 degrees; droplet centred four shell radii from x = 0 on the mid-plane."""
    nx, ny, rs, rc = 2048, 512, 80.0, 40.0
    tau3, u_ref, ca = 0.2, 0.01, 0.1
    sig = sigma_from_capillary(ca, 1.0, tau3, u_ref)
    return Workload(
        name="channel_2048x512", nx=nx, ny=ny, rho=(2.0, 1.0, 1.0), tau=(5 * tau3, tau3, tau3),
        chi=_chi("core", 2.0), sigma12=sig, sigma13=sig, sigma23=sig, xi=5.0,
        H0=h0_from_bond(bond, "core", 2.0, rc, rs, sig, sig), alpha=math.pi / 2,
        drive_G=channel_drive(u_ref, 1.0, tau3, ny), xc=4 * rs, yc=(ny - 1) / 2.0,
        r_core=rc, r_shell=rs, steps=steps, u_ref=u_ref, ferro="core", bond=bond, capillary=ca)


def open_channel_small(xc: float = 170.0, bond: float = 1.0, u_inlet: float = 0.05,
                       steps: int = 400) -> Workload:
    """200 x 50 open channel (Eq. 37 inlet at x = 0, convective outlet at x = 199, no body
    force), the 200 x 50 droplet and materials otherwise.  With the default centre
    x = 170 and centreline inflow 0.05 the shell reaches the outlet within about 250
    steps; a centre near x = 15 puts its rear interface against the inlet instead."""
    return single_channel_small(bond=bond, steps=steps).replace(
        name="open_channel_200x50", drive_G=0.0, u_inlet=u_inlet, xc=xc, u_ref=u_inlet)


def open_channel_paper(bond: float = 2.0, steps: int = 20000) -> Workload:
    """The paper's open-channel set-up (Sec. 2.5, Sec. 3.1): L x H = 900 x 150, core r = 20,
    shell r = 35, the droplet centred 4 r_core from the inlet on the centre line (as
    printed), ferrofluid shell, field along x, Ca = 0.15, equal densities, viscosities and
    surface tensions; Eq. 37 inflow with centreline value u_ref = 0.01."""
    nx, ny, rs, rc = 900, 150, 35.0, 20.0
    tau3, u_ref, ca = 0.2, 0.01, 0.15
    sig = sigma_from_capillary(ca, 1.0, tau3, u_ref)
    return Workload(
        name="open_channel_900x150", nx=nx, ny=ny, tau=(tau3, tau3, tau3), chi=_chi("shell", 1.0),
        sigma12=sig, sigma13=sig, sigma23=sig, xi=5.0,
        H0=h0_from_bond(bond, "shell", 1.0, rc, rs, sig, sig), alpha=0.0, drive_G=0.0,
        xc=4 * rc, yc=(ny - 1) / 2.0, r_core=rc, r_shell=rs, steps=steps, u_ref=u_ref,
        ferro="shell", bond=bond, capillary=ca, u_inlet=u_ref)


def adjoint_channel(steps: int = 2000) -> Workload:
    """512 x 128 channel, shell r = 30, core r = 15, ferrofluid shell mu_r = 2,
    Bo_m = 1, field at 30 degrees (off the mirror-symmetric angles), Ca = 0.15."""
    nx, ny, rs, rc = 512, 128, 30.0, 15.0
    tau3, u_ref, ca = 0.2, 0.01, 0.15
    sig = sigma_from_capillary(ca, 1.0, tau3, u_ref)
    return Workload(
        name="channel_512x128", nx=nx, ny=ny, tau=(tau3, tau3, tau3), chi=_chi("shell", 1.0),
        sigma12=sig, sigma13=sig, sigma23=sig, xi=5.0,
        H0=h0_from_bond(1.0, "shell", 1.0, rc, rs, sig, sig), alpha=math.radians(30.0),
        drive_G=channel_drive(u_ref, 1.0, tau3, ny), xc=4 * rs, yc=(ny - 1) / 2.0,
        r_core=rc, r_shell=rs, steps=steps, u_ref=u_ref, ferro="shell", bond=1.0, capillary=ca)


def regime_sweep_batch(seed: int = 20241011, steps: int = 10000) -> List[Workload]:
    """64 channels of uneven size for a (Bo_m, Ca) regime map: ny ~ U{64..256},
    nx = 4 ny, shell r = 0.3 ny, core/shell radius ratio ~ U(0.3, 0.7); Bo_m on
    linspace(0, 8, 8) x Ca on linspace(0.02, 0.3, 8); ferrofluid core or shell and
    field angle 0 or 90 degrees by fair coin flips; chi = 1."""
    rng = np.random.default_rng(seed)
    bonds = np.linspace(0.0, 8.0, 8)
    cas = np.linspace(0.02, 0.3, 8)
    out = []
    tau3, u_ref = 0.2, 0.01
    for k in range(64):
        ny = int(rng.integers(64, 257))
        nx = 4 * ny
        rs = 0.3 * ny
        rc = rs * float(rng.uniform(0.3, 0.7))
        ferro = "core" if rng.random() < 0.5 else "shell"
        alpha = 0.0 if rng.random() < 0.5 else math.pi / 2
        bo, ca = float(bonds[k // 8]), float(cas[k % 8])
        sig = sigma_from_capillary(ca, 1.0, tau3, u_ref)
        out.append(Workload(
            name=f"sweep_{k:02d}", nx=nx, ny=ny, tau=(tau3, tau3, tau3), chi=_chi(ferro, 1.0),
            sigma12=sig, sigma13=sig, sigma23=sig, xi=5.0,
            H0=h0_from_bond(bo, ferro, 1.0, rc, rs, sig, sig), alpha=alpha,
            drive_G=channel_drive(u_ref, 1.0, tau3, ny), xc=nx / 4.0, yc=(ny - 1) / 2.0,
            r_core=rc, r_shell=rs, steps=steps, u_ref=u_ref, ferro=ferro, bond=bo, capillary=ca))
    return out


def adjoint_batch(seed: int = 20241012, steps: int = 3000) -> List[Workload]:
    """32 channels 256 x 64 (shell r = 18, core r = 9), ferrofluid shell,
    Bo_m ~ U(0, 6), Ca ~ U(0.05, 0.2), field angle ~ U(0, 90) degrees."""
    rng = np.random.default_rng(seed)
    tau3, u_ref = 0.2, 0.01
    out = []
    for k in range(32):
        bo = float(rng.uniform(0.0, 6.0))
        ca = float(rng.uniform(0.05, 0.2))
        alpha = math.radians(float(rng.uniform(0.0, 90.0)))
        sig = sigma_from_capillary(ca, 1.0, tau3, u_ref)
        out.append(Workload(
            name=f"adj_{k:02d}", nx=256, ny=64, tau=(tau3, tau3, tau3), chi=_chi("shell", 1.0),
            sigma12=sig, sigma13=sig, sigma23=sig, xi=5.0,
            H0=h0_from_bond(bo, "shell", 1.0, 9.0, 18.0, sig, sig), alpha=alpha,
            drive_G=channel_drive(u_ref, 1.0, tau3, 64), xc=64.0, yc=31.5,
            r_core=9.0, r_shell=18.0, steps=steps, u_ref=u_ref, ferro="shell", bond=bo,
            capillary=ca))
    return out


def _smooth_periodic_x(a: np.ndarray, passes: int) -> np.ndarray:
    for _ in range(passes):
        a = (np.roll(a, 1, axis=1) + a + np.roll(a, -1, axis=1)) / 3.0
        up = np.concatenate([a[:1], a[:-1]], axis=0)
        dn = np.concatenate([a[1:], a[-1:]], axis=0)
        a = (up + a + dn) / 3.0
    return a


def random_phase_fields(nx: int, ny: int, seed: int, smooth: int = 6,
                        u_amp: float = 0.01, p_amp: float = 0.01):
    """Smooth random order parameters (phi1, phi2 >= 0, phi1 + phi2 <= 1), velocity and
    normalised pressure, as [ny][nx] float64 arrays: (phi1, phi2, ux, uy, pstar)."""
    rng = np.random.default_rng(seed)
    z = [_smooth_periodic_x(rng.standard_normal((ny, nx)), smooth) for _ in range(5)]
    z = [v / (np.abs(v).max() + 1e-300) for v in z]
    a = 1.0 / (1.0 + np.exp(-4.0 * z[0]))
    b = 1.0 / (1.0 + np.exp(-4.0 * z[1]))
    phi1 = a * b
    phi2 = (1.0 - a) * b
    return (np.ascontiguousarray(phi1), np.ascontiguousarray(phi2),
            np.ascontiguousarray(u_amp * z[2]), np.ascontiguousarray(u_amp * z[3]),
            np.ascontiguousarray(p_amp * z[4]))
