"""Pins of the ternary free energy (Eq. 26-28) and chemical potentials (Eq. 25)."""
import numpy as np
import pytest

from fcd_inputs import Workload
from oracle.oracle import lib, params_from_workload, ptr


def params(s12, s13, s23, eta=0.0, xi=5.0):
    w = Workload(name="fe", nx=4, ny=4, sigma12=s12, sigma13=s13, sigma23=s23, eta=eta, xi=xi)
    return params_from_workload(w)


def H(p, ph):
    return lib().orc_free_energy(p, ptr(np.array(ph, float)))


def dH(p, ph):
    out = np.zeros(3)
    lib().orc_free_energy_grad(p, ptr(np.array(ph, float)), ptr(out))
    return out


def mu(p, ph, lap):
    out = np.zeros(3)
    lib().orc_chem_potential(p, ptr(np.array(ph, float)), ptr(np.array(lap, float)), ptr(out))
    return out


SIGMAS = [(0.01, 0.01, 0.01), (0.01, 0.017, 0.01), (0.012, 0.004, 0.009), (0.01, 0.01, 0.01, 0.05)]


@pytest.mark.parametrize("sig", SIGMAS)
def test_gradient_matches_finite_differences(sig):
    p = params(*sig)
    rng = np.random.default_rng(3)
    for _ in range(20):
        ph = rng.uniform(-0.1, 1.1, 3)
        g = dH(p, ph)
        h = 1e-5
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            num = (H(p, ph + e) - H(p, ph - e)) / (2 * h)
            assert g[k] == pytest.approx(num, rel=1e-8, abs=1e-14)


@pytest.mark.parametrize("sig", SIGMAS[:3])
def test_absent_phase_stays_absent(sig):
    """Algebraic consistency: where phase 2 is absent, its chemical potential vanishes
    for any surface tensions (partial spreading, eta = 0)."""
    p = params(*sig)
    for phi1 in np.linspace(0.0, 1.0, 11):
        m = mu(p, (phi1, 0.0, 1.0 - phi1), (0.3, 0.0, -0.3))
        assert abs(m[1]) < 1e-17


@pytest.mark.parametrize("s13", [0.004, 0.01, 0.017])
@pytest.mark.parametrize("xi", [4.0, 5.0])
def test_binary_reduction(s13, xi):
    """With phase 2 absent the ternary force (mu1 - mu3) grad phi1 must be the binary
    phase-field force of surface tension sigma13: mu_b = 4 beta phi (phi-1)(phi-1/2) -
    kappa lap phi with beta = 12 sigma/xi, kappa = 3 sigma xi / 2."""
    p = params(0.01, s13, 0.01, xi=xi)
    beta = 12.0 * s13 / xi
    kappa = 1.5 * s13 * xi
    for phi in np.linspace(0.0, 1.0, 9):
        for lap in (-0.2, 0.0, 0.05):
            m = mu(p, (phi, 0.0, 1.0 - phi), (lap, 0.0, -lap))
            mb = 4 * beta * phi * (phi - 1) * (phi - 0.5) - kappa * lap
            assert m[0] - m[2] == pytest.approx(mb, abs=1e-16)


def test_relabelling_symmetry():
    """Swapping phases 1 and 2 together with sigma13 <-> sigma23 swaps mu1 and mu2."""
    rng = np.random.default_rng(11)
    pa = params(0.01, 0.013, 0.006)
    pb = params(0.01, 0.006, 0.013)
    for _ in range(10):
        ph = rng.uniform(0, 1, 3)
        lap = rng.standard_normal(3) * 0.1
        ma = mu(pa, ph, lap)
        mb = mu(pb, (ph[1], ph[0], ph[2]), (lap[1], lap[0], lap[2]))
        assert ma[0] == pytest.approx(mb[1], rel=1e-12, abs=1e-18)
        assert ma[1] == pytest.approx(mb[0], rel=1e-12, abs=1e-18)
        assert ma[2] == pytest.approx(mb[2], rel=1e-12, abs=1e-18)
