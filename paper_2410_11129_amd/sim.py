"""Torch-allocated buffers around one library handle (memory and streams only)."""
from __future__ import annotations

import ctypes as C

import torch

from . import fcd


def make_params(w, solver: int = fcd.FCD_SOLVER_MG, tol: float = 1e-10, omega: float = 0.0,
                check_every: int = 1, max_iters: int = 100000, smooth: int = 1, coarse_sweeps: int = 2,
                extrapolate: int = 2, every: int = 1, u_limit: float = 0.0,
                div_check_every: int = 0) -> fcd.fcd_params:
    """fcd_params from a workload description (any object with the workload fields)."""
    p = fcd.fcd_params()
    for k in range(3):
        p.rho[k], p.tau[k], p.chi[k] = w.rho[k], w.tau[k], w.chi[k]
    p.sigma12, p.sigma13, p.sigma23, p.eta = w.sigma12, w.sigma13, w.sigma23, w.eta
    p.xi, p.mobility, p.H0, p.alpha, p.mu0 = w.xi, w.mobility, w.H0, w.alpha, w.mu0
    p.drive_G, p.grav_x, p.grav_y, p.eps_n = w.drive_G, w.grav[0], w.grav[1], w.eps_n
    p.pot_tol, p.pot_omega, p.pot_solver = tol, omega, solver
    p.pot_check_every, p.pot_max_iters = check_every, max_iters
    p.pot_smooth, p.pot_coarse_sweeps, p.pot_extrapolate = smooth, coarse_sweeps, extrapolate
    p.pot_every = every
    p.u_limit, p.div_check_every = u_limit, div_check_every  # divergence guard (0: defaults)
    return p


def padded_pitch(nx: int, elem_bytes: int) -> int:
    """Row pitch rounded up to a multiple of 256 bytes."""
    per = 256 // elem_bytes
    return ((nx + per - 1) // per) * per


class Channel:
    """One channel on one GPU: device planes owned here (torch), handle owned by the library."""

    def __init__(self, w, precision: int = fcd.FCD_FP64, device: str = "cuda:0", pitch: int | None = None,
                 stream: torch.cuda.Stream | None = None, **solver):
        self.w = w
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == fcd.FCD_FP64 else torch.float32
        esz = 8 if precision == fcd.FCD_FP64 else 4
        self.pitch = pitch if pitch is not None else padded_pitch(w.nx, esz)
        self.lat = fcd.fcd_lattice(w.nx, w.ny, precision, self.pitch)
        self.solver = dict(solver)
        self.prm = make_params(w, **solver)
        ny, P = w.ny, self.pitch
        self.dist = [torch.zeros((27, ny, P), dtype=self.dtype, device=self.device) for _ in range(2)]
        self.phi = torch.zeros((3, ny, P), dtype=self.dtype, device=self.device)
        self.psi = torch.zeros((ny, P), dtype=self.dtype, device=self.device)
        nscr = (fcd.fcd_scratch_bytes(self.lat) + 7) // 8
        self.scratch = torch.zeros(nscr, dtype=torch.float64, device=self.device)
        self.buf = fcd.fcd_buffers()
        self.buf.dist[0] = self.dist[0].data_ptr()
        self.buf.dist[1] = self.dist[1].data_ptr()
        self.buf.phi = self.phi.data_ptr()
        self.buf.psi = self.psi.data_ptr()
        self.buf.scratch = self.scratch.data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = fcd.fcd_create(self.lat, self.prm, self.buf, self.stream.cuda_stream)
        if w.u_inlet is not None:  # open channel (Eq. 37 inlet, convective outlet)
            fcd.fcd_set_open_channel(self.h, w.u_inlet)

    def close(self):
        if self.h is not None:
            fcd.fcd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- set-up ----------------------------------------------------------------
    def init_droplet(self):
        w = self.w
        fcd.fcd_init_compound_droplet(self.h, w.xc, w.yc, w.r_core, w.r_shell)

    def init_fields(self, phi1, phi2, ux, uy, pstar=None):
        t = [torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
             for a in (phi1, phi2, ux, uy)]
        ps = None if pstar is None else torch.as_tensor(pstar, dtype=torch.float64).to(self.device).contiguous()
        fcd.fcd_init_fields(self.h, *[a.data_ptr() for a in t], None if ps is None else ps.data_ptr())
        self.stream.synchronize()

    def set_params(self, **solver):
        if solver:
            self.solver = dict(solver)
        self.prm = make_params(self.w, **self.solver)
        fcd.fcd_set_params(self.h, self.prm)

    def set_workload(self, w):
        """Change materials, field and drive (same lattice); keeps the solver settings."""
        if (w.nx, w.ny) != (self.w.nx, self.w.ny):
            raise ValueError("set_workload cannot change the lattice size")
        self.w = w
        self.set_params()

    # --- work ------------------------------------------------------------------
    def solve_potential(self, tol: float, max_iters: int = 200000):
        return fcd.fcd_solve_potential(self.h, tol, max_iters)

    def step(self, n: int):
        fcd.fcd_step(self.h, n)

    # --- outputs ---------------------------------------------------------------
    def moments(self, mask: int = fcd.FCD_M_ALL) -> dict:
        names = [n for k, n in enumerate(fcd.MOMENT_NAMES) if mask & (1 << k)]
        out = torch.empty((len(names), self.w.ny, self.w.nx), dtype=torch.float64, device=self.device)
        fcd.fcd_read_moments(self.h, mask, out.data_ptr())
        self.stream.synchronize()
        host = out.cpu().numpy()
        return {n: host[i] for i, n in enumerate(names)}

    def state(self):
        out = torch.empty((27, self.w.ny, self.w.nx), dtype=torch.float64, device=self.device)
        fcd.fcd_read_state(self.h, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy()

    def write_state(self, arr):
        t = torch.as_tensor(arr, dtype=torch.float64).to(self.device).contiguous()
        fcd.fcd_write_state(self.h, t.data_ptr())
        self.stream.synchronize()

    def psi_dense(self):
        out = torch.empty((self.w.ny, self.w.nx), dtype=torch.float64, device=self.device)
        fcd.fcd_read_psi(self.h, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy()

    def deformation(self):
        return fcd.fcd_deformation(self.h)

    def extent_deformation(self):
        """[T_o, T_i, l_y outer, l_x outer, l_y inner, l_x inner] (Eq. 42)."""
        return fcd.fcd_extent_deformation(self.h)

    def breakup_probe(self):
        """[contact nodes, their mean y, their circular-mean x, outer droplet's circular-mean x]."""
        return fcd.fcd_breakup_probe(self.h)

    def stats(self):
        return fcd.fcd_stats(self.h)

    def sync(self):
        fcd.fcd_sync(self.h)


class Batch:
    """Many channels stepped together; device buffers owned here (torch)."""

    def __init__(self, workloads, precision: int = fcd.FCD_FP32, device: str = "cuda:0",
                 stream: torch.cuda.Stream | None = None, **solver):
        self.ws = list(workloads)
        self.n = len(self.ws)
        self.device = torch.device(device)
        self.lats = [fcd.fcd_lattice(w.nx, w.ny, precision, w.nx) for w in self.ws]
        solver.setdefault("solver", fcd.FCD_SOLVER_SOR)
        solver.setdefault("check_every", 4)
        self.prms = [make_params(w, **solver) for w in self.ws]
        sizes = fcd.fcd_batch_sizes(self.lats)
        self.bufs = [torch.zeros((max(int(b), 8) + 255) // 256 * 256 // 8, dtype=torch.float64, device=self.device)
                     for b in sizes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = fcd.fcd_batch_create(self.lats, self.prms, *[b.data_ptr() for b in self.bufs],
                                      self.stream.cuda_stream)

    def close(self):
        if self.h is not None:
            fcd.fcd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_droplets(self):
        geom = []
        for w in self.ws:
            geom += [w.xc, w.yc, w.r_core, w.r_shell]
        fcd.fcd_batch_init_compound_droplet(self.h, geom)

    def step(self, n: int):
        fcd.fcd_batch_step(self.h, n)

    def set_schedule(self, tile_rows: int, block_sweeps: int, fused_sweeps: int):
        fcd.fcd_batch_set_schedule(self.h, tile_rows, block_sweeps, fused_sweeps)

    def set_tail_fusion(self, fused_sweeps: int, after_sweeps: int):
        fcd.fcd_batch_set_tail_fusion(self.h, fused_sweeps, after_sweeps)

    def autotune(self, steps_per_candidate: int = 2):
        """Pick the launch schedule by timing real steps; returns (tile_rows,
        block_sweeps, fused_sweeps, tail fused_sweeps, tail after_sweeps)."""
        return fcd.fcd_batch_autotune(self.h, steps_per_candidate)

    def tune_omega(self, steps: int = 4, scales=(1.25, 1.0, 0.9, 0.775)):
        """Per-channel SOR factors 2 / (1 + s sin(pi / (ny + 1))), s from `scales`, chosen by
        the fewest sweeps over `steps` steps per candidate (advances the batch); returns
        the factors."""
        return fcd.fcd_batch_tune_omega(self.h, self.n, steps, list(scales))

    def deformation(self):
        return fcd.fcd_batch_deformation(self.h, self.n)

    def state(self, k: int):
        w = self.ws[k]
        out = torch.empty((27, w.ny, w.nx), dtype=torch.float64, device=self.device)
        fcd.fcd_batch_read_state(self.h, k, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy()

    def moments(self, k: int, mask: int = fcd.FCD_M_ALL) -> dict:
        w = self.ws[k]
        names = [nm for q, nm in enumerate(fcd.MOMENT_NAMES) if mask & (1 << q)]
        out = torch.empty((len(names), w.ny, w.nx), dtype=torch.float64, device=self.device)
        fcd.fcd_batch_read_moments(self.h, k, mask, out.data_ptr())
        self.stream.synchronize()
        host = out.cpu().numpy()
        return {nm: host[i] for i, nm in enumerate(names)}

    def stats(self):
        return fcd.fcd_batch_stats(self.h)


def run_to_breakup(ch: Channel, max_steps: int, every: int = 10) -> dict | None:
    """Step a channel from its initial state, tracking the breakup probe every `every`
    steps (fcd_breakup_track, which follows the droplet across the periodic boundary and
    forms the breakup numbers of Sec. 2.5 / Fig. 3), until the inner droplet touches the
    shell's interface; None if it has not within max_steps."""
    fcd.fcd_breakup_track(ch.h)  # the reference position
    t = 0
    while t < max_steps:
        n = min(every, max_steps - t)
        ch.step(n)
        t += n
        cnt, t_b_star, L_b_star, y_b_star, x_b, y_b = fcd.fcd_breakup_track(ch.h)
        if cnt > 0:
            return {"steps": t, "contact_nodes": int(cnt), "x_b": x_b, "y_b": y_b,
                    "t_b_star": t_b_star, "L_b_star": L_b_star, "y_b_star": y_b_star}
    return None
