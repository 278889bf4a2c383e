"""Thin ctypes binding of the C ABI in include/fcd.h (argument marshalling only).

Every function here forwards to the function of the same name in libfcd.so; all work
runs in the library's HIP kernels.  Loading fails loudly when libfcd.so is missing:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcd.so")

FCD_OK, FCD_ERR_ARG, FCD_ERR_HIP, FCD_ERR_OOM = 0, -1, -2, -3
FCD_ERR_DIVERGED, FCD_ERR_NOT_CONVERGED, FCD_ERR_UNSUPPORTED = -4, -5, -6
FCD_FP64, FCD_FP32 = 0, 1
FCD_SOLVER_SOR, FCD_SOLVER_MG = 0, 1

FCD_M_PSTAR, FCD_M_UX, FCD_M_UY = 1 << 0, 1 << 1, 1 << 2
FCD_M_PHI1, FCD_M_PHI2, FCD_M_PHI3 = 1 << 3, 1 << 4, 1 << 5
FCD_M_RHO, FCD_M_PSI, FCD_M_HX, FCD_M_HY = 1 << 6, 1 << 7, 1 << 8, 1 << 9
FCD_M_ALL = (1 << 10) - 1
MOMENT_NAMES = ("pstar", "ux", "uy", "phi1", "phi2", "phi3", "rho", "psi", "Hx", "Hy")
FCD_NOALLOC_MAX_NY = 8192  # rows fcd_deformation_noalloc's device array holds

# Every symbol include/fcd.h declares.
EXPORTS = (
    "fcd_scratch_bytes", "fcd_create", "fcd_set_params", "fcd_set_open_channel", "fcd_init_compound_droplet",
    "fcd_init_fields", "fcd_solve_potential", "fcd_step", "fcd_read_moments", "fcd_read_state",
    "fcd_write_state", "fcd_read_psi", "fcd_write_psi", "fcd_deformation", "fcd_extent_deformation", "fcd_breakup_probe",
    "fcd_breakup_track", "fcd_deformation_noalloc", "fcd_stats", "fcd_timing",
    "fcd_timing_read", "fcd_use_graphs", "fcd_sync", "fcd_destroy", "fcd_last_error", "fcd_adjoint_bytes", "fcd_adjoint_forward",
    "fcd_adjoint_backward", "fcd_batch_sizes", "fcd_batch_create",
    "fcd_batch_init_compound_droplet", "fcd_batch_step", "fcd_batch_deformation", "fcd_batch_read_state",
    "fcd_batch_read_moments", "fcd_batch_set_schedule", "fcd_batch_set_tail_fusion", "fcd_batch_autotune", "fcd_batch_tune_omega", "fcd_batch_adjoint_bytes",
    "fcd_batch_adjoint_forward", "fcd_batch_adjoint_backward", "fcd_batch_stats",
    "fcd_batch_destroy",
)
TIMING_KINDS = ("collide_stream", "potential_iter", "residual", "phase", "mg_smooth0", "mg_post0")


class fcd_lattice(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32), ("pitch", C.c_int32)]


class fcd_params(C.Structure):
    _fields_ = [
        ("rho", C.c_double * 3), ("tau", C.c_double * 3), ("chi", C.c_double * 3),
        ("sigma12", C.c_double), ("sigma13", C.c_double), ("sigma23", C.c_double),
        ("eta", C.c_double), ("xi", C.c_double), ("mobility", C.c_double),
        ("H0", C.c_double), ("alpha", C.c_double), ("mu0", C.c_double),
        ("drive_G", C.c_double), ("grav_x", C.c_double), ("grav_y", C.c_double),
        ("eps_n", C.c_double), ("pot_tol", C.c_double), ("pot_omega", C.c_double), ("u_limit", C.c_double),
        ("pot_solver", C.c_int32), ("pot_check_every", C.c_int32), ("pot_max_iters", C.c_int32),
        ("pot_smooth", C.c_int32), ("pot_coarse_sweeps", C.c_int32), ("pot_extrapolate", C.c_int32),
        ("pot_every", C.c_int32), ("div_check_every", C.c_int32),
    ]


class fcd_buffers(C.Structure):
    _fields_ = [("dist", C.c_void_p * 2), ("phi", C.c_void_p), ("psi", C.c_void_p),
                ("scratch", C.c_void_p)]


class FcdError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded libfcd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2410_11129_amd/build.py "
                              "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.fcd_scratch_bytes.argtypes = [C.POINTER(fcd_lattice)]
        L.fcd_scratch_bytes.restype = C.c_size_t
        L.fcd_create.argtypes = [C.POINTER(fcd_lattice), C.POINTER(fcd_params), C.POINTER(fcd_buffers),
                                 C.c_void_p, C.POINTER(C.c_void_p)]
        L.fcd_set_params.argtypes = [H, C.POINTER(fcd_params)]
        L.fcd_init_compound_droplet.argtypes = [H, C.c_double, C.c_double, C.c_double, C.c_double]
        L.fcd_set_open_channel.argtypes = [H, C.c_double]
        L.fcd_init_fields.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.fcd_solve_potential.argtypes = [H, C.c_double, C.c_int32, C.POINTER(C.c_int32), dp]
        L.fcd_step.argtypes = [H, C.c_int32]
        L.fcd_read_moments.argtypes = [H, C.c_uint32, C.c_void_p]
        L.fcd_read_state.argtypes = [H, C.c_void_p]
        L.fcd_write_state.argtypes = [H, C.c_void_p]
        L.fcd_read_psi.argtypes = [H, C.c_void_p]
        L.fcd_write_psi.argtypes = [H, C.c_void_p]
        L.fcd_deformation.argtypes = [H, dp]
        L.fcd_extent_deformation.argtypes = [H, dp]
        L.fcd_breakup_probe.argtypes = [H, dp]
        L.fcd_breakup_track.argtypes = [H, dp]
        L.fcd_deformation_noalloc.argtypes = [C.POINTER(fcd_lattice), C.c_void_p, C.c_void_p, C.c_void_p]
        L.fcd_stats.argtypes = [H, dp]
        L.fcd_timing.argtypes = [H, C.c_int32]
        L.fcd_timing_read.argtypes = [H, dp]
        L.fcd_use_graphs.argtypes = [H, C.c_int32]
        L.fcd_sync.argtypes = [H]
        L.fcd_destroy.argtypes = [H]
        L.fcd_adjoint_bytes.argtypes = [C.POINTER(fcd_lattice), C.c_int32, C.c_int32]
        L.fcd_adjoint_bytes.restype = C.c_size_t
        L.fcd_adjoint_forward.argtypes = [H, C.c_int32, C.c_int32, C.c_void_p, dp]
        L.fcd_adjoint_backward.argtypes = [H, dp, dp]
        L.fcd_batch_sizes.argtypes = [C.c_int32, C.POINTER(fcd_lattice), C.POINTER(C.c_size_t)]
        L.fcd_batch_create.argtypes = [C.c_int32, C.POINTER(fcd_lattice), C.POINTER(fcd_params), C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
        L.fcd_batch_init_compound_droplet.argtypes = [H, dp]
        L.fcd_batch_step.argtypes = [H, C.c_int32]
        L.fcd_batch_set_schedule.argtypes = [H, C.c_int32, C.c_int32, C.c_int32]
        L.fcd_batch_set_tail_fusion.argtypes = [H, C.c_int32, C.c_int32]
        L.fcd_batch_adjoint_bytes.argtypes = [H, C.c_int32, C.c_int32]
        L.fcd_batch_adjoint_bytes.restype = C.c_size_t
        L.fcd_batch_adjoint_forward.argtypes = [H, C.c_int32, C.c_int32, C.c_void_p, dp]
        L.fcd_batch_adjoint_backward.argtypes = [H, dp, dp]
        L.fcd_batch_autotune.argtypes = [H, C.c_int32, C.POINTER(C.c_int32)]
        L.fcd_batch_tune_omega.argtypes = [H, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.fcd_batch_deformation.argtypes = [H, dp]
        L.fcd_batch_read_state.argtypes = [H, C.c_int32, C.c_void_p]
        L.fcd_batch_read_moments.argtypes = [H, C.c_int32, C.c_uint32, C.c_void_p]
        L.fcd_batch_stats.argtypes = [H, dp]
        L.fcd_batch_destroy.argtypes = [H]
        L.fcd_last_error.argtypes = []
        L.fcd_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("fcd_scratch_bytes", "fcd_last_error", "fcd_adjoint_bytes", "fcd_batch_adjoint_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def fcd_last_error() -> str:
    return lib().fcd_last_error().decode()


def _check(st: int, where: str, allow=()) -> int:
    if st != FCD_OK and st not in allow:
        raise FcdError(st, where, fcd_last_error())
    return st


def fcd_scratch_bytes(lat: fcd_lattice) -> int:
    return lib().fcd_scratch_bytes(C.byref(lat))


def fcd_create(lat: fcd_lattice, prm: fcd_params, buf: fcd_buffers, stream: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().fcd_create(C.byref(lat), C.byref(prm), C.byref(buf), C.c_void_p(stream), C.byref(h)),
           "fcd_create")
    return h


def fcd_set_params(h, prm: fcd_params):
    _check(lib().fcd_set_params(h, C.byref(prm)), "fcd_set_params")


def fcd_set_open_channel(h, u_avg: float):
    _check(lib().fcd_set_open_channel(h, u_avg), "fcd_set_open_channel")


def fcd_init_compound_droplet(h, xc: float, yc: float, r_core: float, r_shell: float):
    _check(lib().fcd_init_compound_droplet(h, xc, yc, r_core, r_shell), "fcd_init_compound_droplet")


def fcd_init_fields(h, phi1: int, phi2: int, ux: int, uy: int, pstar: int | None):
    _check(lib().fcd_init_fields(h, phi1, phi2, ux, uy, pstar), "fcd_init_fields")


def fcd_solve_potential(h, tol: float, max_iters: int, allow_not_converged: bool = False):
    sw = C.c_int32(0)
    res = C.c_double(0.0)
    st = lib().fcd_solve_potential(h, tol, max_iters, C.byref(sw), C.byref(res))
    _check(st, "fcd_solve_potential", (FCD_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return st, sw.value, res.value


def fcd_step(h, nsteps: int):
    _check(lib().fcd_step(h, int(nsteps)), "fcd_step")


def fcd_read_moments(h, mask: int, out: int):
    _check(lib().fcd_read_moments(h, mask, out), "fcd_read_moments")


def fcd_read_state(h, out: int):
    _check(lib().fcd_read_state(h, out), "fcd_read_state")


def fcd_write_state(h, src: int):
    _check(lib().fcd_write_state(h, src), "fcd_write_state")


def fcd_read_psi(h, out: int):
    _check(lib().fcd_read_psi(h, out), "fcd_read_psi")


def fcd_write_psi(h, src: int):
    _check(lib().fcd_write_psi(h, src), "fcd_write_psi")


def fcd_deformation(h):
    out = (C.c_double * 4)()
    _check(lib().fcd_deformation(h, out), "fcd_deformation")
    return list(out)


def fcd_breakup_probe(h):
    out = (C.c_double * 4)()
    _check(lib().fcd_breakup_probe(h, out), "fcd_breakup_probe")
    return list(out)


def fcd_deformation_noalloc(lat: fcd_lattice, phi: int, stream: int, out: int):
    """Async; out is a device pointer to four doubles."""
    _check(lib().fcd_deformation_noalloc(C.byref(lat), C.c_void_p(phi), C.c_void_p(stream), C.c_void_p(out)),
           "fcd_deformation_noalloc")


def fcd_breakup_track(h):
    out = (C.c_double * 6)()
    _check(lib().fcd_breakup_track(h, out), "fcd_breakup_track")
    return list(out)


def fcd_extent_deformation(h):
    out = (C.c_double * 6)()
    _check(lib().fcd_extent_deformation(h, out), "fcd_extent_deformation")
    return list(out)


def fcd_stats(h):
    out = (C.c_double * 3)()
    _check(lib().fcd_stats(h, out), "fcd_stats")
    return list(out)


def fcd_timing(h, enable):
    """enable: False / 0 off, True / 1 every launch of the step, 2 the collide-and-stream only."""
    _check(lib().fcd_timing(h, int(enable)), "fcd_timing")


def fcd_use_graphs(h, enable: bool):
    _check(lib().fcd_use_graphs(h, 1 if enable else 0), "fcd_use_graphs")


def fcd_timing_read(h) -> dict:
    """{kind: (total_ms, launches)} for the kernel classes in TIMING_KINDS."""
    out = (C.c_double * (2 * len(TIMING_KINDS)))()
    _check(lib().fcd_timing_read(h, out), "fcd_timing_read")
    return {k: (out[2 * i], int(out[2 * i + 1])) for i, k in enumerate(TIMING_KINDS)}


def fcd_sync(h):
    _check(lib().fcd_sync(h), "fcd_sync")


def fcd_destroy(h):
    _check(lib().fcd_destroy(h), "fcd_destroy")


def fcd_batch_sizes(lats) -> tuple:
    arr = (fcd_lattice * len(lats))(*lats)
    out = (C.c_size_t * 3)()
    _check(lib().fcd_batch_sizes(len(lats), arr, out), "fcd_batch_sizes")
    return tuple(out)


def fcd_batch_create(lats, prms, state: int, aux: int, scratch: int, stream: int) -> C.c_void_p:
    la = (fcd_lattice * len(lats))(*lats)
    pa = (fcd_params * len(prms))(*prms)
    b = C.c_void_p()
    _check(lib().fcd_batch_create(len(lats), la, pa, C.c_void_p(state), C.c_void_p(aux), C.c_void_p(scratch),
                                  C.c_void_p(stream), C.byref(b)), "fcd_batch_create")
    return b


def fcd_batch_init_compound_droplet(b, geom):
    g = (C.c_double * len(geom))(*geom)
    _check(lib().fcd_batch_init_compound_droplet(b, g), "fcd_batch_init_compound_droplet")


def fcd_batch_step(b, nsteps: int):
    _check(lib().fcd_batch_step(b, int(nsteps)), "fcd_batch_step")


def fcd_batch_deformation(b, n: int):
    out = (C.c_double * (4 * n))()
    _check(lib().fcd_batch_deformation(b, out), "fcd_batch_deformation")
    return [list(out[4 * k:4 * k + 4]) for k in range(n)]


def fcd_batch_read_state(b, k: int, out: int):
    _check(lib().fcd_batch_read_state(b, k, out), "fcd_batch_read_state")


def fcd_batch_read_moments(b, k: int, mask: int, out: int):
    _check(lib().fcd_batch_read_moments(b, k, mask, out), "fcd_batch_read_moments")


def fcd_batch_stats(b):
    out = (C.c_double * 3)()
    _check(lib().fcd_batch_stats(b, out), "fcd_batch_stats")
    return list(out)


def fcd_batch_destroy(b):
    _check(lib().fcd_batch_destroy(b), "fcd_batch_destroy")


def fcd_adjoint_bytes(lat: fcd_lattice, nsteps: int, ckpt_every: int) -> int:
    return lib().fcd_adjoint_bytes(C.byref(lat), nsteps, ckpt_every)


def fcd_adjoint_forward(h, nsteps: int, ckpt_every: int, work: int):
    out = (C.c_double * 2)()
    _check(lib().fcd_adjoint_forward(h, nsteps, ckpt_every, C.c_void_p(work), out), "fcd_adjoint_forward")
    return list(out)


def fcd_adjoint_backward(h, dJ_dD):
    d = (C.c_double * 2)(*dJ_dD)
    out = (C.c_double * 6)()
    _check(lib().fcd_adjoint_backward(h, d, out), "fcd_adjoint_backward")
    return list(out)


def fcd_batch_set_schedule(b, tile_rows: int, block_sweeps: int, fused_sweeps: int):
    _check(lib().fcd_batch_set_schedule(b, tile_rows, block_sweeps, fused_sweeps), "fcd_batch_set_schedule")


def fcd_batch_set_tail_fusion(b, fused_sweeps: int, after_sweeps: int):
    _check(lib().fcd_batch_set_tail_fusion(b, fused_sweeps, after_sweeps), "fcd_batch_set_tail_fusion")


def fcd_batch_autotune(b, steps_per_candidate: int):
    out = (C.c_int32 * 5)()
    _check(lib().fcd_batch_autotune(b, steps_per_candidate, out), "fcd_batch_autotune")
    return tuple(int(v) for v in out)


def fcd_batch_tune_omega(b, n: int, steps: int, scales):
    sc = (C.c_double * len(scales))(*scales)
    out = (C.c_double * n)()
    _check(lib().fcd_batch_tune_omega(b, steps, len(scales), sc, out), "fcd_batch_tune_omega")
    return list(out)


def fcd_batch_adjoint_bytes(b, nsteps: int, ckpt_every: int) -> int:
    return lib().fcd_batch_adjoint_bytes(b, nsteps, ckpt_every)


def fcd_batch_adjoint_forward(b, n: int, nsteps: int, ckpt_every: int, work: int):
    out = (C.c_double * (2 * n))()
    _check(lib().fcd_batch_adjoint_forward(b, nsteps, ckpt_every, C.c_void_p(work), out), "fcd_batch_adjoint_forward")
    return [(out[2 * k], out[2 * k + 1]) for k in range(n)]


def fcd_batch_adjoint_backward(b, dJ_dD):
    n = len(dJ_dD)
    d = (C.c_double * (2 * n))(*[v for pair in dJ_dD for v in pair])
    out = (C.c_double * (6 * n))()
    _check(lib().fcd_batch_adjoint_backward(b, d, out), "fcd_batch_adjoint_backward")
    return [list(out[6 * k:6 * k + 6]) for k in range(n)]
