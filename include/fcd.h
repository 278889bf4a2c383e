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
    double sor_omega; /* over-relaxation factor of the potential solve in (0, 2); 0 selects
                         2 / (1 + sin(pi / (ny + 1))), optimal for the constant-mu channel */
    double sor_tol;   /* potential solve stops when max |L(psi0 + psi')| <= sor_tol * H0 */
    int32_t sor_check_every; /* sweeps between residual tests */
    int32_t sor_max_sweeps;  /* sweeps allowed per solve before FCD_ERR_NOT_CONVERGED */
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

/* Bytes of device scratch the handle needs for this lattice (reductions). */
size_t fcd_scratch_bytes(const fcd_lattice* lat);

/* Validate the lattice and buffers and build a handle bound to `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Enqueues no work. */
fcd_status fcd_create(const fcd_lattice* lat, const fcd_params* prm, const fcd_buffers* buf,
                      void* hip_stream, fcd_handle** out);

/* Replace the parameters (takes effect for work enqueued afterwards). */
fcd_status fcd_set_params(fcd_handle* h, const fcd_params* prm);

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

/* Solve the potential for the current state (Eq. 6) by four-colour SOR, warm-started
 * from the stored psi', until max |L(psi0 + psi')| <= tol * H0 or max_sweeps.  Sync.
 * sweeps_out / resid_out (nullable) receive the sweep count and the final residual.
 * Returns FCD_ERR_NOT_CONVERGED if the tolerance was not met. */
fcd_status fcd_solve_potential(fcd_handle* h, double tol, int32_t max_sweeps,
                               int32_t* sweeps_out, double* resid_out);

/* Advance nsteps coupled time steps: phases and mu_r, potential solve (sor_tol,
 * sor_max_sweeps), then the fused collide-and-stream of f, g1, g2 with all forces.
 * The potential solve synchronises the stream at each residual test. */
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

/* Counters since creation: out = {steps, potential sweeps, last residual}.  Host only. */
fcd_status fcd_stats(fcd_handle* h, double out[3]);

/* Per-kernel timing with HIP events recorded on the handle's stream around every
 * launch of the step's kernels.  fcd_timing(h, 1) clears the totals and starts
 * recording; fcd_timing(h, 0) stops.  fcd_timing_read (sync) fills out[2*k] with the
 * total milliseconds and out[2*k+1] with the launch count of kernel class k:
 * 0 fused collide-stream, 1 one four-colour SOR sweep (four launches), 2 potential
 * residual, 3 phase moments.  out must hold 8 doubles. */
fcd_status fcd_timing(fcd_handle* h, int32_t enable);
fcd_status fcd_timing_read(fcd_handle* h, double out[8]);

/* Wait for the stream and report any asynchronous HIP error.  Sync. */
fcd_status fcd_sync(fcd_handle* h);

/* Free the handle (not the caller's buffers).  Waits for the stream. */
fcd_status fcd_destroy(fcd_handle* h);

/* Message of the calling thread's last error ("" if none). */
const char* fcd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FCD_H */
