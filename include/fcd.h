/*
 * fcd.h -- C ABI of the MI355X (gfx950) library for the coupled time step of the
 * hybrid finite-difference / phase-field MRT lattice Boltzmann method for a ferrofluid
 * compound droplet in a channel (Poureslami, Majidi, Ranjbar Kermani, Bijarchi,
 * arXiv:2410.11129, Sec. 2.1-2.5).
 *
 * Lattice and layout.  Node (i, j) sits at x = i, y = j with 0 <= i < nx along the
 * channel (periodic) and 0 <= j < ny across it; no-slip walls lie half a cell beyond
 * the first and last rows.  Every device plane is row-major with a row pitch of
 * `pitch` elements ([ny][pitch], x fastest).  A state buffer holds 27 planes: the
 * hydrodynamic distribution f_0..f_8 (Eq. 12) and the two phase-field distributions
 * g^1_0..8, g^2_0..8 (Eq. 29), directions in the order of Eq. 20 (rest, E, N, W, S,
 * NE, NW, SW, SE).  The stored state is the post-streaming one.
 *
 * Ownership.  Every large buffer is allocated by the caller (e.g. as a torch tensor)
 * and must stay valid until fcd_destroy; the library never frees it.  The handle
 * owns only host-side bookkeeping and a pinned host word for convergence tests.
 *
 * Streams.  Work is enqueued on the HIP stream given at creation.  Calls marked
 * "sync" wait for that stream before returning.
 *
 * Errors.  Every call returns an fcd_status; nothing throws or aborts across the
 * ABI.  fcd_last_error() returns a message for the calling thread's last failure.
 * Argument errors (null pointers, sizes, pitch, precision) give FCD_ERR_ARG and
 * enqueue no work.
 */
#ifndef FCD_H
#define FCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcd_handle fcd_handle;

typedef enum {
    FCD_OK = 0,
    FCD_ERR_ARG = -1,
    FCD_ERR_HIP = -2,
    FCD_ERR_OOM = -3,
    FCD_ERR_DIVERGED = -4,
    FCD_ERR_NOT_CONVERGED = -5,
    FCD_ERR_UNSUPPORTED = -6
} fcd_status;

enum { FCD_FP64 = 0, FCD_FP32 = 1 };
enum { FCD_SOLVER_SOR = 0, FCD_SOLVER_MG = 1 };

typedef struct {
    int32_t nx;        /* nodes along the channel; even and >= 4 (four-colour ordering) */
    int32_t ny;        /* nodes across the channel; >= 2 */
    int32_t precision; /* FCD_FP64 or FCD_FP32: element type of every device plane */
    int32_t pitch;     /* elements per row of every plane; >= nx */
} fcd_lattice;

/* Physical and solver parameters, lattice units (delta x = delta t = 1).
 * Phase index 0 = core, 1 = shell, 2 = ambient. */
typedef struct {
    double rho[3];  /* densities, mixed linearly (Eq. 33) */
    double tau[3];  /* relaxation times tau = nu / c_s^2 (Eq. 14), mixed linearly */
    double chi[3];  /* susceptibilities, harmonic mixing of 1 + chi (Eq. 8) */
    double sigma12, sigma13, sigma23; /* surface tensions (Eq. 27-28) */
    double eta;      /* total-spreading coefficient of Eq. 28 (0: partial spreading) */
    double xi;       /* interface width (Eq. 23) */
    double mobility; /* M of Eq. 30; tau_phi = M / c_s^2 */
    double H0;       /* applied field strength */
    double alpha;    /* applied field angle to the channel axis, radians */
    double mu0;      /* permeability of vacuum in lattice units (Eq. 7) */
    double drive_G;  /* uniform body-force density along x driving the channel flow */
    double grav_x, grav_y; /* gravity: F_b = rho g */
    double eps_n;    /* n = grad phi / sqrt(|grad phi|^2 + eps_n^2) */
    double pot_tol;  /* potential solve stops when max |L(psi0 + psi')| <= pot_tol * H0, or
                        at the working precision's rounding floor 16 eps max |C psi'| (C: sum
                        of the operator's coefficients at a node) if that is larger */
    double pot_omega; /* SOR over-relaxation in (0, 2); 0 selects 2 / (1 + sin(pi / (ny + 1))).
                         Multigrid: used when the hierarchy has one level (ny odd), else
                         the default serves its coarsest level. */
    double u_limit;   /* divergence guard: a node with max(|u_x|, |u_y|) above u_limit, or a
                         non-finite p*, phi1 or phi2, marks the state as diverged (the lattice
                         sound speed is c_s = 1/sqrt(3); 0 selects 0.5) */
    int32_t pot_solver;      /* FCD_SOLVER_SOR or FCD_SOLVER_MG */
    int32_t pot_check_every; /* SOR sweeps / multigrid V-cycles between residual tests */
    int32_t pot_max_iters;   /* SOR sweeps / V-cycles allowed per solve */
    int32_t pot_smooth;      /* multigrid: four-colour Gauss-Seidel sweeps of the finest level before and
                                after each coarse correction (one launch each); coarse levels always
                                take one launch of two tile sweeps each way */
    int32_t pot_coarse_sweeps; /* multigrid: SOR sweeps on the coarsest level, times max(1, ny_c / 2);
                                  a negative value -N: exactly N sweeps; 0 is rejected */
    int32_t pot_extrapolate; /* warm start of each step's solve: 0 the previous psi', 1 the linear
                                extrapolation 2 psi'(t-1) - psi'(t-2), 2 the quadratic one
                                3 psi'(t-1) - 3 psi'(t-2) + psi'(t-3), 3 the cubic one
                                4 psi'(t-1) - 6 psi'(t-2) + 4 psi'(t-3) - psi'(t-4) (each order once
                                that many solutions exist); SOR batches: linear at most; the
                                adjoint solves: quadratic at most */
    int32_t pot_every;       /* quasi-static coupling: the potential is solved on steps 0, K, 2K, ...
                                after the last state change and held in between (K = pot_every;
                                0 or 1: every step, the paper's coupling; the adjoints need <= 1;
                                batches use channel 0's value) */
    int32_t div_check_every; /* steps between host reads of the device divergence flag inside
                                fcd_step / fcd_batch_step (0 selects 64); every residual test of
                                the potential solve reads it as well */
} fcd_params;

/* Caller-owned device buffers (element type = lattice precision). */
typedef struct {
    void* dist[2]; /* two state buffers, each [27][ny][pitch]; they swap roles every step and
                      the handle tracks which holds the current state (initially dist[0]) */
    void* phi;     /* [3][ny][pitch]: phi1, phi2, mu_r of the current state */
    void* psi;     /* [ny][pitch]: the potential perturbation psi' (psi = psi0 + psi') */
    void* scratch; /* fcd_scratch_bytes() bytes, any alignment >= 256 */
} fcd_buffers;

/* Moments selectable in fcd_read_moments (bit k selects field k; fields are written
 * in increasing k as consecutive dense [ny][nx] FP64 planes). */
enum {
    FCD_M_PSTAR = 1u << 0, /* p* = p/(rho c_s^2) = sum f (Eq. 21) */
    FCD_M_UX = 1u << 1,    /* u = sum f e + F_t/(2 rho) (Eq. 22) */
    FCD_M_UY = 1u << 2,
    FCD_M_PHI1 = 1u << 3,  /* phi_i = sum g^i (Eq. 32) */
    FCD_M_PHI2 = 1u << 4,
    FCD_M_PHI3 = 1u << 5,  /* 1 - phi1 - phi2 (Eq. 24) */
    FCD_M_RHO = 1u << 6,   /* Eq. 33 */
    FCD_M_PSI = 1u << 7,   /* psi' */
    FCD_M_HX = 1u << 8,    /* H = H0 (cos a, sin a) - grad psi' (Eq. 5) */
    FCD_M_HY = 1u << 9,
    FCD_M_ALL = (1u << 10) - 1
};

/* Bytes of device scratch the handle needs for this lattice: reductions, the multigrid
 * hierarchy (coarse mu, correction and right-hand side per level) and one plane of psi'
 * history for the extrapolated warm start. */
size_t fcd_scratch_bytes(const fcd_lattice* lat);

/* Validate the lattice and buffers and build a handle bound to `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Enqueues no work. */
fcd_status fcd_create(const fcd_lattice* lat, const fcd_params* prm, const fcd_buffers* buf,
                      void* hip_stream, fcd_handle** out);

/* Replace the parameters (takes effect for work enqueued afterwards). */
fcd_status fcd_set_params(fcd_handle* h, const fcd_params* prm);

/* Open channel of Sec. 2.5: from now on x = 0 is the velocity inlet of Eq. 37,
 * u = 4 u_avg (y/H)(1 - y/H), v = 0, with y = j + 1/2 and H = ny (Zou-He closure of f;
 * the inflow carries only the ambient phase), and x = nx - 1 is the convective outlet
 * f(t+1, N) = [f(t, N) + U f(t+1, N-1)] / (1 + U) for f, g1 and g2, U the section mean
 * of the inlet profile.  The phi stencils at the two end columns take zero normal
 * gradient; psi' keeps its periodic closure in x.  The channel is usually driven by the
 * inflow alone (drive_G = 0).  Call before fcd_init_compound_droplet, which then uses the
 * Eq. 37 profile and no periodic image.  Waits for the handle's stream.  FCD_ERR_ARG
 * unless 0 <= u_avg < 1.  The adjoint rejects an open-channel handle; batches are
 * periodic. */
fcd_status fcd_set_open_channel(fcd_handle* h, double u_avg);

/* Initial state of Sec. 2.5: concentric core (radius r_core) and shell (r_shell)
 * centred at (xc, yc), tanh profiles of width xi (minimum image in x); ambient
 * Poiseuille velocity under drive_G; p* = 0; f = f^eq (Eq. 16), g^i = phi_i Gamma
 * (Eq. 18); psi' = 0.  Async. */
fcd_status fcd_init_compound_droplet(fcd_handle* h, double xc, double yc, double r_core,
                                     double r_shell);

/* Initial state from fields: dense [ny][nx] FP64 device arrays phi1, phi2, ux, uy and
 * pstar (nullable = 0).  f = f^eq(p*, u), g^i = phi_i Gamma(u); psi' = 0.  Async. */
fcd_status fcd_init_fields(fcd_handle* h, const double* phi1, const double* phi2,
                           const double* ux, const double* uy, const double* pstar);

/* Solve the potential for the current state (Eq. 6), warm-started from the stored psi',
 * with the configured solver (four-colour SOR or multigrid V-cycles), until
 * max |L(psi0 + psi')| <= tol * H0 or max_iters sweeps / cycles (multigrid with the LDS
 * tail: tests decided on the GPU, as in fcd_step).  Sync.  iters_out /
 * resid_out (nullable) receive the iteration count and the final residual.  Returns
 * FCD_ERR_NOT_CONVERGED if the tolerance was not met. */
fcd_status fcd_solve_potential(fcd_handle* h, double tol, int32_t max_iters,
                               int32_t* iters_out, double* resid_out);

/* Advance nsteps coupled time steps: phases and mu_r, potential solve (pot_tol,
 * pot_max_iters), then the fused collide-and-stream of f, g1, g2 with all forces.
 * A multigrid solve whose hierarchy ends in the LDS tail is decided on the GPU: a
 * residual test before every V-cycle, decided by the test kernel itself, with the next
 * V-cycle and the collide-and-stream launched ahead of the decision and gated on it;
 * the collision publishes the outcome to pinned host memory, which the host reads
 * while that collision runs, and the host adds V-cycles only when the solve needs more
 * than one.  Other solves (SOR, a hierarchy without the tail, per-kernel timing on)
 * synchronise the stream at each residual test.  Both take the same decisions: the
 * results are bitwise the same.
 * Divergence guard: the collide-and-stream kernel raises a device flag when a node's
 * velocity exceeds u_limit or its p*, phi1 or phi2 is not finite; the flag stays set
 * until the state is replaced (fcd_init_*, fcd_write_state).  It is read at every
 * residual test, every div_check_every steps and by every sync call of the handle, and
 * a set flag makes the call return FCD_ERR_DIVERGED (the message gives the largest
 * |u| seen, or names a non-finite state).  Detection lags the kernel that raised it by
 * at most one step when the potential is solved, by div_check_every steps when not. */
fcd_status fcd_step(fcd_handle* h, int32_t nsteps);

/* Write the fields selected by `mask` (FCD_M_*) for the current state into `out`,
 * a device FP64 buffer of popcount(mask) dense [ny][nx] planes.  The force terms of
 * u use the stored psi'.  Async. */
fcd_status fcd_read_moments(fcd_handle* h, uint32_t mask, double* out);

/* Copy the state to / from a dense [27][ny][nx] FP64 device array.  Async. */
fcd_status fcd_read_state(fcd_handle* h, double* out);
fcd_status fcd_write_state(fcd_handle* h, const double* in);

/* Copy psi' to / from a dense [ny][nx] FP64 device array.  Async. */
fcd_status fcd_read_psi(fcd_handle* h, double* out);
fcd_status fcd_write_psi(fcd_handle* h, const double* in);

/* Second-moment deformation of the shell (weight 1 - phi3) and the core (weight
 * phi1) about a circular-mean centroid in periodic x, D = (sqrt Iyy - sqrt Ixx) /
 * (sqrt Iyy + sqrt Ixx) (equal to the index of Eq. 42 for an ellipse), plus the total
 * masses of phases 1 and 2.  out = {D_o, D_i, mass1, mass2}.  Sync. */
fcd_status fcd_deformation(fcd_handle* h, double out[4]);

/* Extent-based deformation index of Eq. 42, T = (l_y - l_x) / (l_y + l_x), of the outer
 * droplet (w = phi1 + phi2) and the inner one (w = phi1), the interface at w = 1/2: l_y is
 * the largest vertical extent over the columns (the longest run of rows with w >= 1/2
 * between its linearly interpolated crossings; a run reaching a wall row ends at the wall),
 * l_x the length of the longest run with w >= 1/2 along the centreline (the middle row, or
 * the mean of the two middle rows when ny is even; periodic, nx when it closes on itself).
 * Not smooth in the state (hence not the adjoint's objective).  out = {T_o, T_i, l_y outer,
 * l_x outer, l_y inner, l_x inner}; T = 0 when both extents vanish.  Sync. */
fcd_status fcd_extent_deformation(fcd_handle* h, double out[6]);

/* Breakup probe (Sec. 2.5: breakup is the inner droplet touching the shell's interface).
 * A contact node is a core node (phi1 >= 1/2) with a nine-point neighbour in the carrier
 * (phi3 >= 1/2; columns periodic, no neighbours beyond the walls).  out = {number of
 * contact nodes (0: no breakup), their mean y, their circular-mean x in [0, nx), the
 * circular-mean x of the outer droplet weighted by phi1 + phi2 (for tracking its travel
 * across the periodic boundary)}; the means are -1 where their weights vanish.  Sync. */
fcd_status fcd_breakup_probe(fcd_handle* h, double out[4]);

/* Breakup tracking and the breakup numbers of Sec. 2.5 / Fig. 3.  Call once after the
 * initial state is set (that call fixes the reference), then every few steps, at most
 * half a channel period of droplet travel apart.  Each call runs fcd_breakup_probe and
 * follows the outer droplet's circular-mean x across the periodic boundary.  out =
 * {contact nodes (0: no breakup yet), t_b* = t_b u / (2 r_shell) (Eq. 38; t_b the steps
 * since the initial state, u the centreline inflow of Eq. 37 in the open channel or the
 * Poiseuille peak the drive sustains in the periodic one; -1 unless the state came from
 * fcd_init_compound_droplet), L_b* = x_b / ny with x_b the contact point's distance along
 * the channel from x = 0 (the inlet of the open channel; in the periodic channel followed
 * across the boundary), y_b* = |y_b - (ny - 1)/2| / ny, x_b, y_b}; entries 1..5 are -1
 * while there is no contact.  Replacing the state (fcd_init_*, fcd_write_state) resets the
 * tracking.  Sync. */
fcd_status fcd_breakup_track(fcd_handle* h, double out[6]);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the deformation and masses of
 * fcd_deformation for phase planes the caller holds, with no handle and no scratch
 * buffer.  phi: device [3][ny][pitch] planes of the lattice's precision (phi1, phi2, mu_r
 * as a handle's phase buffer holds them; phi1 and phi2 are read); out: device buffer of
 * four doubles {D_o, D_i, mass1, mass2}, written by the last kernel.  Uses a library-owned
 * device array of FCD_NOALLOC_MAX_NY x 8 + 32 doubles (about 512 KiB) per GPU, held until
 * the process ends; FCD_ERR_ARG for ny > FCD_NOALLOC_MAX_NY.  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (other streams or threads) race.
 * Allocates nothing; async on hip_stream (a hipStream_t; NULL = the null stream).  The
 * result equals fcd_deformation's bit for bit on the same planes. */
#define FCD_NOALLOC_MAX_NY 8192
fcd_status fcd_deformation_noalloc(const fcd_lattice* lat, const void* phi, void* hip_stream, double* out);

/* Counters since creation: out = {steps, potential iterations (SOR sweeps or V-cycles),
 * last residual}.  Host only. */
fcd_status fcd_stats(fcd_handle* h, double out[3]);

/* Per-kernel timing with HIP events recorded on the handle's stream around every
 * launch of the step's kernels.  fcd_timing(h, 1) clears the totals and starts
 * recording; fcd_timing(h, 0) stops; fcd_timing(h, 2) records only the launches of the
 * collide-and-stream that ran (class 0; the kernel launch records its own start and end,
 * and the steps keep their device-decided path).  Sync.  fcd_timing_read (sync) fills out[2*k] with the
 * total milliseconds and out[2*k+1] with the launch count of class k:
 * 0 fused collide-stream kernel; 1 one potential iteration (a four-colour SOR sweep,
 * or the part of a multigrid V-cycle that follows the convergence test);
 * 2 convergence test (SOR: residual kernel; multigrid: the V-cycle's first smoothing
 * kernel, which reduces the residual of its input); 3 phase moments; 4 multigrid finest-level pre-smoothing kernel; 5 multigrid finest-level
 * prolongation + post-smoothing kernel.  Classes 4 and 5 are single kernels, also
 * counted inside classes 1 and 2.  out must hold 12 doubles.  While timing is on, time
 * steps decide their multigrid tests on the host (one stream synchronisation per test, no
 * launches ahead of a decision), with the same decisions and results as the
 * device-decided steps. */
fcd_status fcd_timing(fcd_handle* h, int32_t enable);
fcd_status fcd_timing_read(fcd_handle* h, double out[12]);

/* Repeated launch sequences of a host-decided potential solve (a multigrid V-cycle and
 * the part of it after the convergence test) run as HIP graphs captured on first use and
 * replayed on the handle's stream (default: enabled); a time step's solve decided on
 * the GPU (fcd_step) launches eagerly either way.  enable = 0 launches every kernel
 * eagerly; the results are bitwise the same.  Graphs are also bypassed while
 * fcd_timing is on.  Sync. */
fcd_status fcd_use_graphs(fcd_handle* h, int32_t enable);

/* Wait for the stream and report any asynchronous HIP error, then FCD_ERR_DIVERGED if
 * the divergence flag is set.  Sync. */
fcd_status fcd_sync(fcd_handle* h);

/* Free the handle (not the caller's buffers).  Waits for the stream. */
fcd_status fcd_destroy(fcd_handle* h);

/* Message of the calling thread's last error ("" if none). */
const char* fcd_last_error(void);

/* ---------------------------------------------------------------------------------
 * Adjoint (reverse-mode gradient) of J = dJ_dD[0] D_o + dJ_dD[1] D_i after nsteps steps,
 * where D_o, D_i are the deformations of fcd_deformation, with respect to
 * p = (H0, alpha, u_ref, sigma12, sigma13, sigma23), u_ref the peak of the Poiseuille
 * profile the drive sustains: drive_G = 8 rho_3 nu_3 u_ref / ny^2 with nu_3 = tau_3 / 3
 * (the pressure-driven flow of Sec. 2.5 as a uniform body force).  Hand-written reverse
 * of the whole coupled step: transposed streaming, node collisions and forces, stencils,
 * the potential solve (adjoint equation L lambda = psi'-bar, L symmetric, solved by the
 * configured solver to pot_tol relative to max |psi'-bar|) and the mixing rules.
 * Checkpointing: the forward keeps the state every ckpt_every steps in `work`; the
 * backward recomputes each segment (keeping its states) and runs the adjoint steps in
 * reverse.  When the forward starts from fcd_init_compound_droplet with no step since,
 * the u_ref gradient includes the initial Poiseuille velocity's dependence on it.
 * --------------------------------------------------------------------------------- */

/* Device bytes of `work` for fcd_adjoint_forward / _backward.  Host only. */
size_t fcd_adjoint_bytes(const fcd_lattice* lat, int32_t nsteps, int32_t ckpt_every);

/* Run nsteps forward steps from the current state, keeping checkpoints in `work`
 * (caller-owned device buffer of fcd_adjoint_bytes, 256-byte aligned); D_out = {D_o, D_i}
 * of the final state.  Sync. */
fcd_status fcd_adjoint_forward(fcd_handle* h, int32_t nsteps, int32_t ckpt_every, void* work, double D_out[2]);

/* Gradient of J for the run of the last fcd_adjoint_forward (same `work`, untouched
 * since): grad = dJ/d(H0, alpha, u_ref, sigma12, sigma13, sigma23).  Sync.  Leaves the
 * handle on the forward's final state. */
fcd_status fcd_adjoint_backward(fcd_handle* h, const double dJ_dD[2], double grad[6]);

/* ---------------------------------------------------------------------------------
 * Batches: n independent channels of uneven size (e.g. a regime-map sweep over Bo_m and
 * Ca) stepped together.  Every kernel of a step is launched once for the whole batch;
 * per-channel lattices and parameters are honoured.  The potential of every channel is
 * solved to its own pot_tol * H0, with channels that have converged left untouched; a
 * batch step ends when every channel has converged.  Solver (channel 0's pot_solver):
 * FCD_SOLVER_MG gives batched multigrid V-cycles (each channel's single-channel
 * hierarchy and V-cycle, finest tiles 64 x 16, channel 0's pot_smooth and its own
 * pot_coarse_sweeps; one launch per level for all channels, each channel's convergence
 * decided on the device, so a channel's result does not depend on the rest of the
 * batch) when
 * every channel's lattice has a coarse level and an LDS tail (nx, ny >= 4 and a small
 * enough coarsest level), else, and for FCD_SOLVER_SOR, four-colour SOR per channel
 * (the SOR factors, schedule and tuners below apply to it only).  The batched adjoint's
 * potential solves use the same solver.  All lattices must share one precision.
 * Caller-owned buffers, sizes from fcd_batch_sizes: `state` (both state buffers of every
 * channel), `aux` (phi1, phi2, mu_r, psi' and psi' history planes), `scratch`
 * (descriptors, tile and job tables, reductions, the coarse multigrid levels); each at
 * least 256-byte aligned.
 * --------------------------------------------------------------------------------- */
typedef struct fcd_batch fcd_batch;

/* bytes_out[0..2] = state, aux and scratch bytes for these n lattices.  Host only. */
fcd_status fcd_batch_sizes(int32_t n, const fcd_lattice* lats, size_t bytes_out[3]);

/* Carve the caller's buffers, upload the per-channel descriptors and tile tables
 * (synchronously), and bind the batch to `hip_stream`. */
fcd_status fcd_batch_create(int32_t n, const fcd_lattice* lats, const fcd_params* prms, void* state,
                            void* aux, void* scratch, void* hip_stream, fcd_batch** out);

/* Initial compound droplet of every channel; geom is a host array of n rows
 * {xc, yc, r_core, r_shell} (the same initial state as fcd_init_compound_droplet). */
fcd_status fcd_batch_init_compound_droplet(fcd_batch* b, const double* geom);

/* Advance every channel by nsteps coupled steps.  Synchronises at residual tests.  Each
 * channel has its own divergence flag (as fcd_step; u_limit per channel, the check
 * interval of channel 0); a set flag makes this call, fcd_batch_deformation and the
 * batched adjoint return FCD_ERR_DIVERGED naming the first such channel. */
fcd_status fcd_batch_step(fcd_batch* b, int32_t nsteps);

/* Deformation and masses of every channel: out is a host array of n rows
 * {D_o, D_i, mass1, mass2} (as fcd_deformation).  Sync. */
fcd_status fcd_batch_deformation(fcd_batch* b, double* out);

/* State (dense [27][ny][nx] FP64) and moments (as fcd_read_moments) of channel k into
 * device buffers.  Async. */
fcd_status fcd_batch_read_state(fcd_batch* b, int32_t k, double* out);
fcd_status fcd_batch_read_moments(fcd_batch* b, int32_t k, uint32_t mask, double* out);

/* Launch schedule of the batch: kernels run over 64 x tile_rows tiles (tile_rows 1, 2,
 * 4 or 8), the potential sweeps are replayed as HIP graphs of block_sweeps sweeps (a
 * multiple of pot_check_every of channel 0, the interval of the device-side convergence
 * test, at most 2^20), and fused_sweeps > 0 runs that many four-colour SOR sweeps per
 * launch on 64 x 32 tiles with their halo in LDS (1 or 2 with pot_check_every a multiple
 * of 2 fused_sweeps, or 4 with pot_check_every a multiple of 4; block_sweeps a multiple
 * of 2 fused_sweeps), 0 one launch per colour.  The schedule changes launch geometry
 * only: states are bitwise the same under every schedule.  Default: tile_rows 4,
 * block_sweeps 8 * pot_check_every, the largest of fused_sweeps 2 and 1 allowed.
 * FCD_ERR_ARG for any other value. */
fcd_status fcd_batch_set_schedule(fcd_batch* b, int32_t tile_rows, int32_t block_sweeps, int32_t fused_sweeps);

/* Tail fusion: the graph blocks of a potential solve that start at or after
 * after_sweeps sweeps run fused_sweeps sweeps per fused launch instead of the
 * schedule's (deep fusion repeats halo work, which costs most while many channels are
 * active; late in a solve, when few are, the number of launches dominates).
 * fused_sweeps 0 turns it off; otherwise a value fcd_batch_set_schedule would accept for
 * the test interval.  Applies only while the schedule fuses (fused_sweeps > 0) and to
 * block sizes that are a multiple of 2 fused_sweeps.  States are bitwise unchanged.
 * Default: 4 after 16 * pot_check_every sweeps where 4 is allowed, else off.
 * FCD_ERR_ARG for any other value. */
fcd_status fcd_batch_set_tail_fusion(fcd_batch* b, int32_t fused_sweeps, int32_t after_sweeps);

/* Autotuner: tries every tile_rows in {1, 2, 4, 8} with block_sweeps in
 * {2, 8, 32} * pot_check_every and every allowed fused_sweeps in {0, 1, 2, 4}, each for
 * one untimed step (capturing its graphs) and steps_per_candidate real steps of the batch
 * timed with HIP events, keeps the fastest; then, where 4 sweeps per launch are allowed,
 * tries the tail fusion off and 4 after {8, 16, 32} * pot_check_every sweeps the same
 * way.  Writes choice = {tile_rows, block_sweeps, fused_sweeps, tail fused_sweeps, tail
 * after_sweeps}.  Advances the batch by 12 F (1 + steps_per_candidate) steps, F the
 * number of allowed fusions, plus 4 (1 + steps_per_candidate) for the tail fusion when
 * 4 is allowed.  Sync. */
fcd_status fcd_batch_autotune(fcd_batch* b, int32_t steps_per_candidate, int32_t choice[5]);

/* SOR factor tuner: for each of the ncand (1..16) candidate scales s in scale[], every
 * channel relaxes with 2 / (1 + s sin(pi / (ny + 1))) for `steps` real steps while the
 * device counts the sweeps each channel receives; each channel then keeps (as its
 * pot_omega) the factor with its smallest count, the earlier candidate on ties, written
 * to omega_out[k] (host, n values).  The choice depends on the channels' states only,
 * not on timing.  Advances the batch by ncand * steps steps (callers that want the
 * tuned factors from the initial state initialise again).  Sync.  FCD_ERR_ARG for a
 * scale outside (0, 10). */
fcd_status fcd_batch_tune_omega(fcd_batch* b, int32_t steps, int32_t ncand, const double* scale, double* omega_out);

/* Batched adjoint: the adjoint of fcd_adjoint_forward / _backward for every channel of
 * the batch at once (one launch per kernel for all channels, the adjoint potential
 * solves by the batch's solver with per-channel thresholds pot_tol * max |psi'-bar|).
 * fcd_batch_adjoint_bytes: device bytes of `work` (host only).
 * fcd_batch_adjoint_forward: nsteps steps from the current state, checkpoints every
 * ckpt_every steps in `work` (caller-owned, 256-byte aligned); D_out[2k..2k+1] =
 * {D_o, D_i} of channel k after the run.  Sync.
 * fcd_batch_adjoint_backward: grad[6k..6k+5] = dJ_k/d(H0, alpha, u_ref, sigma12,
 * sigma13, sigma23) of channel k for J_k = dJ_dD[2k] D_o + dJ_dD[2k+1] D_i.  Sync; leaves
 * the batch on the forward's final state. */
size_t fcd_batch_adjoint_bytes(fcd_batch* b, int32_t nsteps, int32_t ckpt_every);
fcd_status fcd_batch_adjoint_forward(fcd_batch* b, int32_t nsteps, int32_t ckpt_every, void* work, double* D_out);
fcd_status fcd_batch_adjoint_backward(fcd_batch* b, const double* dJ_dD, double* grad);

/* out = {steps, SOR sweeps launched, largest final residual of the last solve}. */
fcd_status fcd_batch_stats(fcd_batch* b, double out[3]);

/* Free the batch (not the caller's buffers).  Waits for the stream. */
fcd_status fcd_batch_destroy(fcd_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* FCD_H */
