"""ctypes marshalling for the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fcd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)


class OracleParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("open_x", C.c_int32), ("pad1", C.c_int32),
        ("rho", C.c_double * 3), ("tau", C.c_double * 3), ("chi", C.c_double * 3),
        ("sigma12", C.c_double), ("sigma13", C.c_double), ("sigma23", C.c_double),
        ("eta", C.c_double), ("xi", C.c_double), ("mobility", C.c_double),
        ("H0", C.c_double), ("alpha", C.c_double), ("mu0", C.c_double),
        ("drive_G", C.c_double), ("grav_x", C.c_double), ("grav_y", C.c_double),
        ("eps_n", C.c_double), ("u_inlet", C.c_double),
    ]


class OracleSolver(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("max_sweeps", C.c_int32), ("check_every", C.c_int32),
        ("every", C.c_int32), ("omega", C.c_double), ("tol", C.c_double),
    ]

    @classmethod
    def direct(cls, every: int = 1) -> "OracleSolver":
        return cls(0, 0, 1, every, 1.0, 0.0)

    @classmethod
    def sor(cls, omega: float, tol: float, max_sweeps: int = 100000, check_every: int = 1, every: int = 1):
        return cls(1, max_sweeps, check_every, every, omega, tol)


_LIB_FAST = os.path.join(_HERE, "liboracle_fast.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no architecture-specific flags, one
    thread): the checker the tests load."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_fast() -> str:
    """The same source built for the CPU baseline of the benchmark on the machine that
    runs it: -O3 -march=native with its row loops shared out by OpenMP (the per-node
    arithmetic, and so every result, is that of the plain build)."""
    tmp = _LIB_FAST + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-std=c11", "-Wall", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_FAST)
    return _LIB_FAST


_lib = None
_lib_fast = None


def _load(path: str):
    L = C.CDLL(path)
    P = C.POINTER(OracleParams)
    S = C.POINTER(OracleSolver)
    L.orc_gamma.argtypes = [_dp, _dp]
    L.orc_feq.argtypes = [C.c_double, _dp, _dp]
    L.orc_forcing.argtypes = [_dp, C.c_double, _dp]
    L.orc_collide_f.argtypes = [_dp, C.c_double, _dp, _dp, C.c_double, C.c_double, _dp]
    L.orc_mrt_matrices.argtypes = [_dp, _dp]
    L.orc_lattice.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), _dp]
    L.orc_free_energy.argtypes = [P, _dp]
    L.orc_free_energy.restype = C.c_double
    L.orc_free_energy_grad.argtypes = [P, _dp, _dp]
    L.orc_chem_potential.argtypes = [P, _dp, _dp, _dp]
    L.orc_solve_potential_phi.argtypes = [P, _dp, _dp, S, _dp, _dp, _dp,
                                          C.POINTER(C.c_int32), _dp]
    L.orc_potential_residual_phi.argtypes = [P, _dp, _dp, _dp, _dp]
    L.orc_potential_residual_phi.restype = C.c_double
    L.orc_apply_L.argtypes = [P, _dp, _dp, _dp]
    L.orc_init_fields.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_init_droplet.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double,
                                   _dp, _dp, _dp, _dp, _dp]
    L.orc_step.argtypes = [P, S, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, C.POINTER(C.c_int32), _dp]
    L.orc_moments.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
    L.orc_forces.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
    L.orc_deformation_w.argtypes = [C.c_int32, C.c_int32, _dp]
    L.orc_deformation_w.restype = C.c_double
    L.orc_diagnostics.argtypes = [P, _dp, _dp, _dp]
    L.orc_extent_deformation.argtypes = [P, _dp, _dp, _dp]
    L.orc_breakup_probe.argtypes = [P, _dp, _dp, _dp]
    L.orc_stencils.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp, _dp]
    L.orc_mu_r.argtypes = [P, _dp, _dp, _dp]
    L.orc_phase_source.argtypes = [P, _dp, _dp, _dp]
    L.orc_threads.argtypes = []
    L.orc_threads.restype = C.c_int
    for name in ("orc_init_fields", "orc_init_droplet", "orc_step", "orc_moments",
                 "orc_forces", "orc_diagnostics", "orc_extent_deformation", "orc_breakup_probe",
                 "orc_solve_potential_phi"):
        getattr(L, name).restype = C.c_int
    return L


def use_fast_build():
    """Make lib() load the -O3 -march=native OpenMP build (call before the first lib())."""
    global _LIB
    if _lib is not None and _LIB != _LIB_FAST:
        raise RuntimeError("the oracle library is already loaded")
    _LIB = build_fast()


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _load(_LIB)
    return _lib


def lib_fast():
    """The -O3 -march=native OpenMP build (built on first use on this machine), loaded beside
    lib(): the same source and per-node arithmetic, for the large CPU runs."""
    global _lib_fast
    if _lib_fast is None:
        _lib_fast = _load(build_fast())
    return _lib_fast


def ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "float64 C-contiguous arrays only"
    return a.ctypes.data_as(_dp)


def params_from_workload(w) -> OracleParams:
    p = OracleParams()
    p.nx, p.ny = w.nx, w.ny
    for k in range(3):
        p.rho[k], p.tau[k], p.chi[k] = w.rho[k], w.tau[k], w.chi[k]
    p.sigma12, p.sigma13, p.sigma23, p.eta = w.sigma12, w.sigma13, w.sigma23, w.eta
    p.xi, p.mobility = w.xi, w.mobility
    p.H0, p.alpha, p.mu0 = w.H0, w.alpha, w.mu0
    p.drive_G, p.grav_x, p.grav_y = w.drive_G, w.grav[0], w.grav[1]
    p.eps_n = w.eps_n
    p.open_x = 0 if w.u_inlet is None else 1
    p.u_inlet = 0.0 if w.u_inlet is None else w.u_inlet
    return p


class OracleSim:
    """State (f, g1, g2 as [9][ny][nx]; psi' as [ny][nx]) plus calls into the oracle."""

    MOMENT_NAMES = ("pstar", "ux", "uy", "phi1", "phi2", "phi3", "rho", "psi", "Hx", "Hy")
    FORCE_NAMES = ("Fs_x", "Fs_y", "Fm_x", "Fm_y", "Fmu_x", "Fmu_y", "Ft_x", "Ft_y")

    def __init__(self, workload, solver: OracleSolver | None = None, fast: bool = False):
        self.w = workload
        self.L = lib_fast() if fast else lib()  # fast: the -O3 -march=native OpenMP build
        self.p = params_from_workload(workload)
        self.solver = solver if solver is not None else OracleSolver.direct()
        ny, nx = workload.ny, workload.nx
        self.f = np.zeros((9, ny, nx))
        self.g1 = np.zeros((9, ny, nx))
        self.g2 = np.zeros((9, ny, nx))
        self.psi = np.zeros((ny, nx))
        self.sweeps = 0
        self.resid = 0.0
        self.nstep = 0  # steps since the initial state (quasi-static coupling phase)

    # --- initial state ---------------------------------------------------------
    def init_droplet(self, solve: bool = True):
        w = self.w
        phi1 = np.zeros((w.ny, w.nx))
        phi2 = np.zeros((w.ny, w.nx))
        rc = self.L.orc_init_droplet(C.byref(self.p), w.xc, w.yc, w.r_core, w.r_shell,
                                    ptr(self.f), ptr(self.g1), ptr(self.g2), ptr(phi1), ptr(phi2))
        assert rc == 0, rc
        self.nstep = 0
        if solve:
            self.solve_potential()
        return phi1, phi2

    def init_fields(self, phi1, phi2, ux, uy, pstar=None, solve: bool = True):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (phi1, phi2, ux, uy)]
        ps = None if pstar is None else np.ascontiguousarray(pstar, dtype=np.float64)
        rc = self.L.orc_init_fields(C.byref(self.p), *[ptr(a) for a in arrs], ptr(ps),
                                   ptr(self.f), ptr(self.g1), ptr(self.g2))
        assert rc == 0, rc
        self.nstep = 0
        if solve:
            self.solve_potential()

    # --- potential ---------------------------------------------------------------
    def phases(self):
        return self.g1.sum(axis=0), self.g2.sum(axis=0)

    def solve_potential(self, solver: OracleSolver | None = None):
        phi1, phi2 = self.phases()
        phi1 = np.ascontiguousarray(phi1)
        phi2 = np.ascontiguousarray(phi2)
        sw = C.c_int32(0)
        res = C.c_double(0.0)
        s = solver if solver is not None else self.solver
        rc = self.L.orc_solve_potential_phi(C.byref(self.p), ptr(phi1), ptr(phi2), C.byref(s),
                                           ptr(self.psi), None, None, C.byref(sw), C.byref(res))
        self.sweeps, self.resid = sw.value, res.value
        return rc

    # --- stepping --------------------------------------------------------------
    def step(self, n: int) -> int:
        sw = C.c_int32(0)
        res = C.c_double(0.0)
        rc = self.L.orc_step(C.byref(self.p), C.byref(self.solver), int(n), int(self.nstep), ptr(self.f),
                            ptr(self.g1), ptr(self.g2), ptr(self.psi), C.byref(sw), C.byref(res))
        self.sweeps, self.resid = sw.value, res.value
        self.nstep += int(n)
        return rc

    # --- outputs -----------------------------------------------------------------
    def moments(self) -> dict:
        out = np.zeros((10, self.w.ny, self.w.nx))
        rc = self.L.orc_moments(C.byref(self.p), ptr(self.f), ptr(self.g1), ptr(self.g2),
                               ptr(self.psi), ptr(out))
        assert rc == 0, rc
        return {k: out[i] for i, k in enumerate(self.MOMENT_NAMES)}

    def forces(self) -> dict:
        out = np.zeros((8, self.w.ny, self.w.nx))
        rc = self.L.orc_forces(C.byref(self.p), ptr(self.f), ptr(self.g1), ptr(self.g2),
                              ptr(self.psi), ptr(out))
        assert rc == 0, rc
        return {k: out[i] for i, k in enumerate(self.FORCE_NAMES)}

    def diagnostics(self):
        out = np.zeros(4)
        rc = self.L.orc_diagnostics(C.byref(self.p), ptr(self.g1), ptr(self.g2), ptr(out))
        assert rc == 0, rc
        return out

    def breakup_probe(self):
        """{contact nodes, their mean y, their circular-mean x, outer droplet's circular-mean x}."""
        out = np.zeros(4)
        rc = self.L.orc_breakup_probe(C.byref(self.p), ptr(self.g1), ptr(self.g2), ptr(out))
        assert rc == 0, rc
        return out

    def extent_deformation(self):
        """{T_o, T_i, l_y outer, l_x outer, l_y inner, l_x inner} (Eq. 42 extents)."""
        out = np.zeros(6)
        rc = self.L.orc_extent_deformation(C.byref(self.p), ptr(self.g1), ptr(self.g2), ptr(out))
        assert rc == 0, rc
        return out


# --- complex-step build ---------------------------------------------------------------
# The same source compiled with real = double _Complex (ORC_COMPLEX_STEP): a parameter
# given an imaginary part i h carries h times its first derivative through every step, so
# dJ/dtheta = Im J(theta + i h) / h to rounding, with no difference of nearby values.

_LIB_CS = os.path.join(_HERE, "liboracle_cs.so")
_lib_cs = None
_vp = C.c_void_p


def build_cstep(force: bool = True) -> str:
    """Compile the complex-step build (plain -O2; complex division by Smith's method,
    without the library's rescaling for infinities, which these values never reach)."""
    if force or not os.path.exists(_LIB_CS):
        tmp = _LIB_CS + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-DORC_COMPLEX_STEP",
                               "-fcx-fortran-rules", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_CS)
    return _LIB_CS


_R2 = C.c_double * 2  # one double _Complex


class OracleParamsCS(C.Structure):
    """orc_params of the complex-step build: every floating field is a double _Complex."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("open_x", C.c_int32), ("pad1", C.c_int32),
        ("rho", _R2 * 3), ("tau", _R2 * 3), ("chi", _R2 * 3),
        ("sigma12", _R2), ("sigma13", _R2), ("sigma23", _R2),
        ("eta", _R2), ("xi", _R2), ("mobility", _R2),
        ("H0", _R2), ("alpha", _R2), ("mu0", _R2),
        ("drive_G", _R2), ("grav_x", _R2), ("grav_y", _R2),
        ("eps_n", _R2), ("u_inlet", _R2),
    ]


def _c(v) -> "_R2":
    z = complex(v)
    return _R2(z.real, z.imag)


def params_cs_from_workload(w, drive_G=None) -> OracleParamsCS:
    """Complex parameters from a workload whose fields may hold complex numbers."""
    p = OracleParamsCS()
    p.nx, p.ny = w.nx, w.ny
    for k in range(3):
        p.rho[k], p.tau[k], p.chi[k] = _c(w.rho[k]), _c(w.tau[k]), _c(w.chi[k])
    p.sigma12, p.sigma13, p.sigma23, p.eta = _c(w.sigma12), _c(w.sigma13), _c(w.sigma23), _c(w.eta)
    p.xi, p.mobility = _c(w.xi), _c(w.mobility)
    p.H0, p.alpha, p.mu0 = _c(w.H0), _c(w.alpha), _c(w.mu0)
    p.drive_G = _c(w.drive_G if drive_G is None else drive_G)
    p.grav_x, p.grav_y = _c(w.grav[0]), _c(w.grav[1])
    p.eps_n = _c(w.eps_n)
    p.open_x = 0 if w.u_inlet is None else 1
    p.u_inlet = _c(0.0 if w.u_inlet is None else w.u_inlet)
    return p


def lib_cstep():
    global _lib_cs
    if _lib_cs is None:
        L = C.CDLL(build_cstep(force=not os.path.exists(_LIB_CS)))
        P = C.POINTER(OracleParamsCS)
        S = C.POINTER(OracleSolver)
        L.orc_init_droplet.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double, _vp, _vp, _vp, _vp, _vp]
        L.orc_step.argtypes = [P, S, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]
        L.orc_diagnostics.argtypes = [P, _vp, _vp, _vp]
        for name in ("orc_init_droplet", "orc_step", "orc_diagnostics"):
            getattr(L, name).restype = C.c_int
        _lib_cs = L
    return _lib_cs


def _zp(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags["C_CONTIGUOUS"], "complex128 C-contiguous arrays only"
    return a.ctypes.data_as(_vp)


# the parameters of the gradient, in the order the adjoint reports them
THETA_NAMES = ("H0", "alpha", "u_ref", "sigma12", "sigma13", "sigma23")


def complex_step_run(w, nsteps: int, k: int | None, h: float = 1e-20, solver: OracleSolver | None = None):
    """Droplet initial state of workload w, then nsteps oracle steps with parameter k of
    THETA_NAMES given the imaginary part h (none when k is None); returns the complex
    diagnostics {D_o, D_i, sum phi1, sum phi2}.  u_ref enters through the channel drive
    G = 8 rho_3 nu_3 u_ref / ny^2 (the Poiseuille peak u_ref), which is linear in it."""
    from fcd_inputs import channel_drive
    L = lib_cstep()
    theta = {n: complex(getattr(w, n)) for n in THETA_NAMES}
    if k is not None:
        theta[THETA_NAMES[k]] += 1j * h
    wc = w.replace(H0=theta["H0"], alpha=theta["alpha"], sigma12=theta["sigma12"], sigma13=theta["sigma13"],
                   sigma23=theta["sigma23"])
    p = params_cs_from_workload(wc, drive_G=channel_drive(theta["u_ref"], w.rho[2], w.tau[2], w.ny))
    s = solver if solver is not None else OracleSolver.direct()
    ny, nx = w.ny, w.nx
    f = np.zeros((9, ny, nx), np.complex128)
    g1 = np.zeros_like(f)
    g2 = np.zeros_like(f)
    phi1 = np.zeros((ny, nx), np.complex128)
    phi2 = np.zeros_like(phi1)
    psi = np.zeros_like(phi1)
    assert L.orc_init_droplet(C.byref(p), w.xc, w.yc, w.r_core, w.r_shell, _zp(f), _zp(g1), _zp(g2), _zp(phi1),
                              _zp(phi2)) == 0
    sw, res = C.c_int32(0), C.c_double(0.0)
    rc = L.orc_step(C.byref(p), C.byref(s), int(nsteps), 0, _zp(f), _zp(g1), _zp(g2), _zp(psi), C.byref(sw),
                    C.byref(res))
    assert rc == 0, rc
    out = np.zeros(4, np.complex128)
    assert L.orc_diagnostics(C.byref(p), _zp(g1), _zp(g2), _zp(out)) == 0
    return out


def complex_step_gradient(w, nsteps: int, weights=(1.0, 0.0), h: float = 1e-20):
    """J = a D_o + b D_i after nsteps from the droplet state, and dJ/dtheta for the six
    parameters of THETA_NAMES, each from one complex-step run: Im J(theta_k + i h) / h."""
    a, b = weights
    grad = np.zeros(6)
    J = None
    for k in range(6):
        d = complex_step_run(w, nsteps, k, h)
        Jc = a * d[0] + b * d[1]
        grad[k] = Jc.imag / h
        J = Jc.real if J is None else J
    return J, grad
