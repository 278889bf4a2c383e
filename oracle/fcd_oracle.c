/*
 * fcd_oracle.c -- plain, slow, FP64 CPU oracle of the coupled step of the hybrid
 * finite-difference / phase-field MRT lattice Boltzmann method for a ferrofluid
 * compound droplet in a channel (Poureslami, Majidi, Ranjbar Kermani, Bijarchi,
 * arXiv:2410.11129, Sections 2.1-2.5).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no code, header, table or
 * helper with the HIP library; it is written directly from the paper's equations.
 * Where the printed text is garbled or silent, the reading taken is stated at the
 * point of use ("Reading:").
 *
 * Conventions.  Node (i, j) sits at x = i, y = j, 0 <= i < nx, 0 <= j < ny.  Every
 * plane is row-major [ny][nx] (x fastest); distributions are [9][ny][nx].  The
 * channel is periodic in x, or open (Eq. 37 inlet at i = 0, convective outlet at
 * i = nx - 1) when open_x is set; no-slip walls lie half a cell outside the first and
 * last rows (y = -1/2 and y = ny - 1/2).
 *
 * Parity status: every exported function below is pinned by a CPU test against
 * closed forms, invariants or brute force.  The long-run coupled trajectory of
 * orc_step as a whole has no value printed in the paper (parity unpinned for the
 * trajectory itself; each of its parts is pinned).  The complex-step build (see the
 * scalar type below) is the reference gradient of the adjoint; it is pinned against
 * central differences of this real build and the exact zeros at H0 = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Scalar type.  The method's arithmetic is written over `real`, which is      */
/* double in the oracle proper.  Built with ORC_COMPLEX_STEP, real is          */
/* double _Complex: a parameter given a tiny imaginary part i h then carries   */
/* h times its first derivative through every step, and dJ/dtheta =           */
/* Im J(theta + i h) / h holds to rounding, with no difference of nearby      */
/* values (complex-step differentiation: Squire and Trapp, SIAM Review 40,     */
/* 1998; Martins, Sturdza and Alonso, ACM TOMS 29, 2003).  That requires every */
/* operation on a real to be the analytic continuation of the real one:        */
/* sums, products, quotients, sqrt, tanh, cos, sin are; comparisons and        */
/* floor act on the real part (they select a branch, whose derivative is that  */
/* of the branch); |x| is x times the sign of its real part; atan2 takes its   */
/* first-order continuation, exact for h far below the rounding of the real    */
/* part.  Lattice constants and the solver's settings stay double.            */
/* ------------------------------------------------------------------------- */
#ifdef ORC_COMPLEX_STEP
#include <complex.h>
typedef double _Complex real;
#define RE(x) creal(x)
#define r_sqrt csqrt
#define r_tanh ctanh
#define r_cos ccos
#define r_sin csin
static inline real r_abs(real x) { return creal(x) < 0.0 ? -x : x; }
/* atan2(y, x) + i (x Im y - y Im x) / (x^2 + y^2) with x, y the real parts. */
static inline real r_atan2(real y, real x) {
    double a = creal(x), b = creal(y);
    return atan2(b, a) + I * ((a * cimag(y) - b * cimag(x)) / (a * a + b * b));
}
/* magnitude for stop tests and maxima */
static inline double r_mag(real x) { return cabs(x); }
#else
typedef double real;
#define RE(x) (x)
#define r_sqrt sqrt
#define r_tanh tanh
#define r_cos cos
#define r_sin sin
#define r_abs fabs
#define r_atan2 atan2
#define r_mag fabs
#endif

/* ------------------------------------------------------------------------- */
/* Lattice (Eq. 17 weights, Eq. 20 velocities; delta x = delta t = 1, c = 1). */
/* ------------------------------------------------------------------------- */
#define NQ 9
static const int EX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0; /* c_s^2 (Section 2.2, after Eq. 14) */

/* Orthogonal moment matrix M of the D2Q9 MRT model in the Lallemand-Luo order
 * (density, energy, energy squared, j_x, q_x, j_y, q_y, p_xx, p_xy).  Reading: Eq. 13
 * prints eight rates for nine moments; the missing one is a further unit rate. */
static const double MM[NQ][NQ] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},         {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},     {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},      {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},      {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
static double MINV[NQ][NQ];
static int minv_ready = 0;

/* M^{-1} by Gauss-Jordan elimination with partial pivoting (no use is made of the
 * orthogonality of M, so a typo in M shows up as M^{-1} M != I in the tests). */
static void build_minv(void) {
    double a[NQ][2 * NQ];
    for (int r = 0; r < NQ; ++r)
        for (int c = 0; c < 2 * NQ; ++c) a[r][c] = c < NQ ? MM[r][c] : (c - NQ == r ? 1.0 : 0.0);
    for (int c = 0; c < NQ; ++c) {
        int piv = c;
        for (int r = c + 1; r < NQ; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k < 2 * NQ; ++k) {
                double t = a[c][k];
                a[c][k] = a[piv][k];
                a[piv][k] = t;
            }
        double d = a[c][c];
        for (int k = 0; k < 2 * NQ; ++k) a[c][k] /= d;
        for (int r = 0; r < NQ; ++r)
            if (r != c) {
                double m = a[r][c];
                for (int k = 0; k < 2 * NQ; ++k) a[r][k] -= m * a[c][k];
            }
    }
    for (int r = 0; r < NQ; ++r)
        for (int c = 0; c < NQ; ++c) MINV[r][c] = a[r][NQ + c];
    minv_ready = 1;
}

/* ------------------------------------------------------------------------- */
/* Parameters.                                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny;
    int32_t open_x; /* 0: periodic channel; 1: Eq. 37 inlet at i = 0, convective outlet at i = nx - 1 */
    int32_t pad1;
    real rho[3], tau[3], chi[3]; /* phase 1 = core, 2 = shell, 3 = ambient   */
    real sigma12, sigma13, sigma23, eta;
    real xi, mobility;
    real H0, alpha, mu0;
    real drive_G, grav_x, grav_y;
    real eps_n; /* n = grad phi / sqrt(|grad phi|^2 + eps_n^2); the paper leaves |grad phi| = 0 open */
    real u_inlet; /* open channel: u_avg of Eq. 37 (the centreline value of the inlet profile) */
} orc_params;

typedef struct {
    int32_t mode;        /* 0: direct banded Cholesky, 1: four-colour SOR */
    int32_t max_sweeps;  /* SOR only */
    int32_t check_every; /* SOR only: residual test every this many sweeps */
    int32_t every;       /* orc_step: potential solved on steps 0, K, 2K, ... (K = every; 0, 1: all) */
    double omega; /* SOR relaxation factor */
    double tol;   /* SOR stop: max |L_mu(psi0 + psi')| <= tol * H0 */
} orc_solver;

#define IDX(i, j, nx) ((size_t)(j) * (size_t)(nx) + (size_t)(i))

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Value of a plane at (i + dx, j + dy): periodic in x (or, with clamp_x, columns
 * beyond the inlet and outlet take the value of the end column); rows outside the
 * channel take the value of the nearest row (reading: zero normal gradient of phi and
 * mu_r at the walls, i.e. neutral wetting; the paper names no wetting condition). */
static inline real nb_mirror(const real* a, int nx, int ny, int i, int j, int dx, int dy, int clamp_x) {
    int ii = i + dx;
    if (clamp_x)
        ii = ii < 0 ? 0 : (ii > nx - 1 ? nx - 1 : ii);
    else
        ii = wrap(ii, nx);
    int jj = j + dy;
    if (jj < 0) jj = 0;
    if (jj > ny - 1) jj = ny - 1;
    return a[IDX(ii, jj, nx)];
}

/* Value of psi' at (i + dx, j + dy): periodic in x; zero in the ghost rows,
 * unless ghost data are given (used only by the potential tests).  Reading: the paper
 * gives no boundary condition for psi; the applied potential psi0 is imposed in the
 * ghost rows, i.e. psi' = 0 there. */
static inline real nb_psi(const real* a, int nx, int ny, int i, int j, int dx, int dy,
                            const real* lo, const real* hi) {
    int ii = wrap(i + dx, nx);
    int jj = j + dy;
    if (jj < 0) return lo ? lo[ii] : 0.0;
    if (jj > ny - 1) return hi ? hi[ii] : 0.0;
    return a[IDX(ii, jj, nx)];
}

/* ------------------------------------------------------------------------- */
/* Equilibria and forcing.                                                    */
/* ------------------------------------------------------------------------- */

/* Gamma_alpha(u), Eq. 18.  Reading: the last term is -u.u/(2 c_s^2) (the printed
 * -u.u/c_s^2 would break sum_alpha Gamma_alpha = 1). */
void orc_gamma(const real u[2], real out[NQ]) {
    real uu = u[0] * u[0] + u[1] * u[1];
    for (int a = 0; a < NQ; ++a) {
        real eu = EX[a] * u[0] + EY[a] * u[1];
        out[a] = WQ[a] * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* f^eq_alpha = p* w_alpha + (Gamma_alpha - w_alpha), Eq. 16. */
void orc_feq(real pstar, const real u[2], real out[NQ]) {
    real G[NQ];
    orc_gamma(u, G);
    for (int a = 0; a < NQ; ++a) out[a] = pstar * WQ[a] + (G[a] - WQ[a]);
}

/* F_alpha = w_alpha e_alpha . F_t / (rho c_s^2), Eq. 19. */
void orc_forcing(const real Ft[2], real rho, real out[NQ]) {
    for (int a = 0; a < NQ; ++a) out[a] = WQ[a] * (EX[a] * Ft[0] + EY[a] * Ft[1]) / (rho * CS2);
}

/* Apply M^{-1} Lambda M to a 9-vector; Lambda = diag(1,1,1,1,1,1,1,s_nu,s_nu) (Eq. 13). */
static void mrt_apply(const real d[NQ], real s_nu, real out[NQ]) {
    if (!minv_ready) build_minv();
    real m[NQ];
    for (int r = 0; r < NQ; ++r) {
        real acc = 0.0;
        for (int c = 0; c < NQ; ++c) acc += MM[r][c] * d[c];
        m[r] = acc;
    }
    m[7] *= s_nu;
    m[8] *= s_nu;
    for (int r = 0; r < NQ; ++r) {
        real acc = 0.0;
        for (int c = 0; c < NQ; ++c) acc += MINV[r][c] * m[c];
        out[r] = acc;
    }
}

/* MRT collision with forcing at one node, Eq. 12 with Eq. 15:
 * f* = f - M^{-1} Lambda M (f - fbar^eq) + F,  fbar^eq = f^eq(p*, u) - F/2. */
void orc_collide_f(const real f[NQ], real pstar, const real u[2], const real Ft[2],
                   real rho, real tau, real out[NQ]) {
    real feq[NQ], F[NQ], d[NQ], r[NQ];
    orc_feq(pstar, u, feq);
    orc_forcing(Ft, rho, F);
    for (int a = 0; a < NQ; ++a) d[a] = f[a] - (feq[a] - 0.5 * F[a]);
    real s_nu = 1.0 / (0.5 + tau); /* Eq. 13 */
    mrt_apply(d, s_nu, r);
    for (int a = 0; a < NQ; ++a) out[a] = f[a] - r[a] + F[a];
}

/* Exported for the tests: M, M^{-1} (row-major 9x9). */
void orc_mrt_matrices(double m_out[NQ * NQ], double minv_out[NQ * NQ]) {
    if (!minv_ready) build_minv();
    for (int r = 0; r < NQ; ++r)
        for (int c = 0; c < NQ; ++c) {
            m_out[r * NQ + c] = MM[r][c];
            minv_out[r * NQ + c] = MINV[r][c];
        }
}

void orc_lattice(int32_t ex[NQ], int32_t ey[NQ], double w[NQ]) {
    for (int a = 0; a < NQ; ++a) {
        ex[a] = EX[a];
        ey[a] = EY[a];
        w[a] = WQ[a];
    }
}

/* ------------------------------------------------------------------------- */
/* Free energy and chemical potentials (Eq. 25-28).                           */
/* ------------------------------------------------------------------------- */

/* gamma_i = sigma_ij + sigma_ik - sigma_jk (Eq. 27); 3/gamma_T = sum 1/gamma_i (Eq. 26). */
static void spreading_coeffs(const orc_params* P, real gam[3], real* gT) {
    gam[0] = P->sigma12 + P->sigma13 - P->sigma23;
    gam[1] = P->sigma12 + P->sigma23 - P->sigma13;
    gam[2] = P->sigma13 + P->sigma23 - P->sigma12;
    *gT = 3.0 / (1.0 / gam[0] + 1.0 / gam[1] + 1.0 / gam[2]);
}

/* Bulk free energy H(phi1, phi2, phi3), Eq. 28. */
real orc_free_energy(const orc_params* P, const real ph[3]) {
    real gam[3], gT;
    spreading_coeffs(P, gam, &gT);
    real p1 = ph[0], p2 = ph[1], p3 = ph[2];
    return P->sigma12 * p1 * p1 * p2 * p2 + P->sigma13 * p1 * p1 * p3 * p3 +
           P->sigma23 * p2 * p2 * p3 * p3 +
           p1 * p2 * p3 * (gam[0] * p1 + gam[1] * p2 + gam[2] * p3) +
           P->eta * p1 * p1 * p2 * p2 * p3 * p3;
}

/* Partial derivatives dH/dphi_k of Eq. 28 with the three phi treated as
 * independent variables. */
void orc_free_energy_grad(const orc_params* P, const real ph[3], real dH[3]) {
    real gam[3], gT;
    spreading_coeffs(P, gam, &gT);
    real p1 = ph[0], p2 = ph[1], p3 = ph[2];
    real s12 = P->sigma12, s13 = P->sigma13, s23 = P->sigma23, eta = P->eta;
    dH[0] = 2.0 * s12 * p1 * p2 * p2 + 2.0 * s13 * p1 * p3 * p3 +
            p2 * p3 * (gam[0] * p1 + gam[1] * p2 + gam[2] * p3) + p1 * p2 * p3 * gam[0] +
            2.0 * eta * p1 * p2 * p2 * p3 * p3;
    dH[1] = 2.0 * s12 * p1 * p1 * p2 + 2.0 * s23 * p2 * p3 * p3 +
            p1 * p3 * (gam[0] * p1 + gam[1] * p2 + gam[2] * p3) + p1 * p2 * p3 * gam[1] +
            2.0 * eta * p1 * p1 * p2 * p3 * p3;
    dH[2] = 2.0 * s13 * p1 * p1 * p3 + 2.0 * s23 * p2 * p2 * p3 +
            p1 * p2 * (gam[0] * p1 + gam[1] * p2 + gam[2] * p3) + p1 * p2 * p3 * gam[2] +
            2.0 * eta * p1 * p1 * p2 * p2 * p3;
}

/* Chemical potentials, Eq. 25.  Reading: the "gamma_t" of the Laplacian term is
 * gamma_i, as in the Boyer-Lapuerta form the paper cites (equal to gamma_T when the
 * three surface tensions are equal). */
void orc_chem_potential(const orc_params* P, const real ph[3], const real lap[3], real mu[3]) {
    real gam[3], gT, dH[3];
    spreading_coeffs(P, gam, &gT);
    orc_free_energy_grad(P, ph, dH);
    for (int k = 0; k < 3; ++k) {
        real s = 0.0;
        for (int j = 0; j < 3; ++j)
            if (j != k) s += (dH[k] - dH[j]) / gam[j];
        mu[k] = 4.0 * gT / P->xi * s - 0.75 * P->xi * gam[k] * lap[k];
    }
}

/* ------------------------------------------------------------------------- */
/* Phase fields and the isotropic stencils (Eq. 24, 32-35, 8).                */
/* ------------------------------------------------------------------------- */

/* phi_i = sum_alpha g^i_alpha (Eq. 32). */
static void phase_from_g(int nx, int ny, const real* g, real* phi) {
    size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        real s = 0.0;
        for (int a = 0; a < NQ; ++a) s += g[a * n + k];
        phi[k] = s;
    }
}

/* mu_r = 1 + chi with 1/(1+chi) = sum_i phi_i/(1+chi_i): Eq. 8 read with the index
 * on chi that the printed formula drops (harmonic mean, as the text says). */
static void mu_r_from_phi(const orc_params* P, const real* phi1, const real* phi2, real* mur) {
    size_t n = (size_t)P->nx * P->ny;
    for (size_t k = 0; k < n; ++k) {
        real p3 = 1.0 - phi1[k] - phi2[k];
        real s = phi1[k] / (1.0 + P->chi[0]) + phi2[k] / (1.0 + P->chi[1]) + p3 / (1.0 + P->chi[2]);
        mur[k] = 1.0 / s;
    }
}

/* Isotropic gradient, Eq. 34: grad a = (1/c_s^2) sum_alpha w_alpha e_alpha a(x + e_alpha). */
static void iso_grad(const real* a, int nx, int ny, int i, int j, int clamp_x, real g[2]) {
    real gx = 0.0, gy = 0.0;
    for (int q = 0; q < NQ; ++q) {
        real v = nb_mirror(a, nx, ny, i, j, EX[q], EY[q], clamp_x);
        gx += WQ[q] * EX[q] * v;
        gy += WQ[q] * EY[q] * v;
    }
    g[0] = gx / CS2;
    g[1] = gy / CS2;
}

/* Isotropic Laplacian, Eq. 35: lap a = (2/c_s^2) sum_alpha w_alpha [a(x+e_alpha) - a(x)]. */
static real iso_lap(const real* a, int nx, int ny, int i, int j, int clamp_x) {
    real c = a[IDX(i, j, nx)];
    real s = 0.0;
    for (int q = 0; q < NQ; ++q) s += WQ[q] * (nb_mirror(a, nx, ny, i, j, EX[q], EY[q], clamp_x) - c);
    return 2.0 * s / CS2;
}

/* Interface normals and the counter-diffusion magnitude of Eq. 23 for the three
 * phases: n_k = grad phi_k / sqrt(|grad phi_k|^2 + eps_n^2) (reading: the paper leaves
 * n undefined where grad phi vanishes), theta_k = (4/xi) phi_k (1 - phi_k). */
static void interface_terms(const orc_params* P, const real* phi, const real (*gphi)[2], real* theta,
                            real (*nrm)[2]) {
    for (int s = 0; s < 3; ++s) {
        real gx = gphi[s][0], gy = gphi[s][1];
        real nn = r_sqrt(gx * gx + gy * gy + P->eps_n * P->eps_n);
        nrm[s][0] = gx / nn;
        nrm[s][1] = gy / nn;
        theta[s] = 4.0 / P->xi * phi[s] * (1.0 - phi[s]);
    }
}

/* Source term of the phase-field LBE of component comp (Eq. 29).  Reading: the paper
 * only cites it; taken as the term whose first moment is c_s^2 times the
 * counter-diffusion flux of Eq. 23 for that component,
 *   F^{phi,i}_alpha = w_alpha e_alpha . [theta_i n_i - (1/3) sum_k theta_k n_k],
 * the inner sum over all three phases (Eq. 23 with its reused index read as a sum over
 * k), so that the three right-hand sides of Eq. 23 add up to zero as phi_1 + phi_2 +
 * phi_3 = 1 requires. */
static void phase_source(const real theta[3], const real nrm[3][2], int comp, real F[NQ]) {
    real sx = 0.0, sy = 0.0;
    for (int s = 0; s < 3; ++s) {
        sx += theta[s] * nrm[s][0];
        sy += theta[s] * nrm[s][1];
    }
    real vx = theta[comp] * nrm[comp][0] - sx / 3.0;
    real vy = theta[comp] * nrm[comp][1] - sy / 3.0;
    for (int a = 0; a < NQ; ++a) F[a] = WQ[a] * (EX[a] * vx + EY[a] * vy);
}

/* Exported for the tests: the sources of all three components at one node from phi_k and
 * grad phi_k (k = 1..3), out[k * 9 + alpha]. */
void orc_phase_source(const orc_params* P, const real phi[3], const real gphi[6], real out[3 * NQ]) {
    real g[3][2] = {{gphi[0], gphi[1]}, {gphi[2], gphi[3]}, {gphi[4], gphi[5]}};
    real theta[3], nrm[3][2];
    interface_terms(P, phi, g, theta, nrm);
    for (int c = 0; c < 3; ++c) phase_source(theta, nrm, c, out + c * NQ);
}

/* Everything the collision at one node needs. */
typedef struct {
    real phi[3], gphi[3][2], lphi[3], nrm[3][2], theta[3];
    real rho, tau, grho[2], gchi[2], mu[3];
    real Fs[2], H[2], Fm[2], Fp[2], Fd[2], Fb[2], Fmu[2], Ft[2];
    real pstar, u0[2], u[2];
} nodeq;

/* Stencils, forces and velocity at node (i, j) given phi planes, psi' and the local f. */
static void node_quantities(const orc_params* P, const real* phi1, const real* phi2,
                            const real* psi, const real* fnode, int i, int j, nodeq* q) {
    int nx = P->nx, ny = P->ny;
    size_t k = IDX(i, j, nx);
    /* Phase fields, Eq. 24; gradients and Laplacians, Eq. 34-35; those of phi_3 follow
     * from phi_3 = 1 - phi_1 - phi_2 by linearity. */
    q->phi[0] = phi1[k];
    q->phi[1] = phi2[k];
    q->phi[2] = 1.0 - phi1[k] - phi2[k];
    /* Open channel, reading: zero normal gradient of phi at the inlet and outlet (the
     * paper names no phase-field condition there; as at the walls). */
    iso_grad(phi1, nx, ny, i, j, P->open_x, q->gphi[0]);
    iso_grad(phi2, nx, ny, i, j, P->open_x, q->gphi[1]);
    q->gphi[2][0] = -q->gphi[0][0] - q->gphi[1][0];
    q->gphi[2][1] = -q->gphi[0][1] - q->gphi[1][1];
    q->lphi[0] = iso_lap(phi1, nx, ny, i, j, P->open_x);
    q->lphi[1] = iso_lap(phi2, nx, ny, i, j, P->open_x);
    q->lphi[2] = -q->lphi[0] - q->lphi[1];
    interface_terms(P, q->phi, q->gphi, q->theta, q->nrm);
    /* Mixture closure: Eq. 33 for rho.  Reading: the paper does not say how the
     * viscosity is mixed; tau = sum phi_i tau_i (linear). */
    q->rho = 0.0;
    q->tau = 0.0;
    q->grho[0] = q->grho[1] = 0.0;
    for (int s = 0; s < 3; ++s) {
        q->rho += P->rho[s] * q->phi[s];
        q->tau += P->tau[s] * q->phi[s];
        q->grho[0] += P->rho[s] * q->gphi[s][0];
        q->grho[1] += P->rho[s] * q->gphi[s][1];
    }
    /* Eq. 9: grad chi = -[sum grad phi_i/(1+chi_i)] / [sum phi_i/(1+chi_i)]^2. */
    real S = 0.0, gS[2] = {0.0, 0.0};
    for (int s = 0; s < 3; ++s) {
        S += q->phi[s] / (1.0 + P->chi[s]);
        gS[0] += q->gphi[s][0] / (1.0 + P->chi[s]);
        gS[1] += q->gphi[s][1] / (1.0 + P->chi[s]);
    }
    q->gchi[0] = -gS[0] / (S * S);
    q->gchi[1] = -gS[1] / (S * S);
    /* Chemical potentials (Eq. 25) and surface tension force (Eq. 36). */
    orc_chem_potential(P, q->phi, q->lphi, q->mu);
    q->Fs[0] = q->Fs[1] = 0.0;
    for (int s = 0; s < 3; ++s) {
        q->Fs[0] += q->mu[s] * q->gphi[s][0];
        q->Fs[1] += q->mu[s] * q->gphi[s][1];
    }
    /* H = -grad(psi0 + psi') = H0 (cos a, sin a) - grad psi' (Eq. 5 with the Eq. 34
     * stencil); Kelvin force, Eq. 7, with mu0 in lattice units. */
    real gpx = 0.0, gpy = 0.0;
    for (int a = 0; a < NQ; ++a) {
        real v = nb_psi(psi, nx, ny, i, j, EX[a], EY[a], NULL, NULL);
        gpx += WQ[a] * EX[a] * v;
        gpy += WQ[a] * EY[a] * v;
    }
    q->H[0] = P->H0 * r_cos(P->alpha) - gpx / CS2;
    q->H[1] = P->H0 * r_sin(P->alpha) - gpy / CS2;
    real H2 = q->H[0] * q->H[0] + q->H[1] * q->H[1];
    q->Fm[0] = -0.5 * P->mu0 * H2 * q->gchi[0];
    q->Fm[1] = -0.5 * P->mu0 * H2 * q->gchi[1];
    /* Pressure (Eq. 21), pressure force F_p = -(p/rho) grad rho = -p* c_s^2 grad rho,
     * gravity F_b = rho g.  Reading: the pressure-driven flow of the periodic channel is
     * driven by a uniform force density drive_G along x. */
    real ps = 0.0, jx = 0.0, jy = 0.0;
    size_t n = (size_t)nx * ny;
    (void)n;
    for (int a = 0; a < NQ; ++a) {
        ps += fnode[a];
        jx += fnode[a] * EX[a];
        jy += fnode[a] * EY[a];
    }
    q->pstar = ps;
    q->Fp[0] = -ps * CS2 * q->grho[0];
    q->Fp[1] = -ps * CS2 * q->grho[1];
    q->Fd[0] = P->drive_G;
    q->Fd[1] = 0.0;
    q->Fb[0] = q->rho * P->grav_x;
    q->Fb[1] = q->rho * P->grav_y;
    real F0[2];
    for (int c = 0; c < 2; ++c) F0[c] = q->Fs[c] + q->Fp[c] + q->Fm[c] + q->Fd[c] + q->Fb[c];
    /* Eq. 22 without the viscous force.  Reading: F_mu needs grad u, which needs u;
     * the viscous force is taken from the local non-equilibrium stress instead, as in
     * the velocity-based model the paper follows (Fakhari et al.). */
    q->u0[0] = jx + F0[0] / (2.0 * q->rho);
    q->u0[1] = jy + F0[1] / (2.0 * q->rho);
    /* Viscous force from the non-equilibrium stress:
     * Pi_ij = sum_b e_bi e_bj [M^-1 Lambda M (f - f^eq(p*, u0))]_b,
     * F_mu,i = -(nu / c_s^2) Pi_ij d_j rho, with nu = c_s^2 tau (Eq. 14). */
    real feq0[NQ], d[NQ], r[NQ];
    orc_feq(ps, q->u0, feq0);
    for (int a = 0; a < NQ; ++a) d[a] = fnode[a] - feq0[a];
    mrt_apply(d, 1.0 / (0.5 + q->tau), r);
    real Pxx = 0.0, Pxy = 0.0, Pyy = 0.0;
    for (int a = 0; a < NQ; ++a) {
        Pxx += EX[a] * EX[a] * r[a];
        Pxy += EX[a] * EY[a] * r[a];
        Pyy += EY[a] * EY[a] * r[a];
    }
    real nu = CS2 * q->tau;
    q->Fmu[0] = -(nu / CS2) * (Pxx * q->grho[0] + Pxy * q->grho[1]);
    q->Fmu[1] = -(nu / CS2) * (Pxy * q->grho[0] + Pyy * q->grho[1]);
    for (int c = 0; c < 2; ++c) q->Ft[c] = F0[c] + q->Fmu[c];
    /* Eq. 22 with the total force. */
    q->u[0] = jx + q->Ft[0] / (2.0 * q->rho);
    q->u[1] = jy + q->Ft[1] / (2.0 * q->rho);
}

/* Phase-field collision, Eq. 29-31, with the source term of phase_source.  phi in
 * Eq. 31 is phi_i and Gamma uses the final velocity of the step. */
static void collide_g(const orc_params* P, const nodeq* q, int comp, const real g[NQ], real out[NQ]) {
    real Gm[NQ], Fphi[NQ];
    orc_gamma(q->u, Gm);
    phase_source(q->theta, q->nrm, comp, Fphi);
    real tau_phi = P->mobility / CS2; /* Eq. 30, its "c_s^s" read as c_s^2 */
    for (int a = 0; a < NQ; ++a) {
        real geq = q->phi[comp] * Gm[a] - 0.5 * Fphi[a]; /* Eq. 31 */
        out[a] = g[a] - (g[a] - geq) / (0.5 + tau_phi) + Fphi[a];
    }
}

/* ------------------------------------------------------------------------- */
/* Magnetic scalar potential (Eq. 6).                                         */
/* ------------------------------------------------------------------------- */
/* Reading: the paper names a second-order isotropic finite-difference scheme and no
 * more.  The discrete operator taken is the conservative nine-point flux form
 *   (L u)(x) = (1/c_s^2) sum_{a=1..8} w_a (mu(x) + mu(x+e_a)) (u(x+e_a) - u(x)),
 * which equals mu * (Eq. 35 Laplacian) when mu is constant and is symmetric.  The total potential is
 * psi = psi0 + psi', psi0 = -H0 (x cos a + y sin a); psi' is periodic in x and zero in
 * the ghost rows.  In the open channel too (reading: the paper gives the potential no
 * condition at the inlet or outlet; psi' is the droplet's perturbation of the applied
 * field and decays away from it, so the periodic closure is kept there).  The equation L(psi0 + psi') = 0 reads
 *   sum_a c_a (psi'(x+e_a) - psi'(x)) = H0 sum_a c_a (e_a . h),   c_a = 3 w_a (mu + mu_a). */

static inline real coef(const real* mur, int nx, int ny, int i, int j, int a) {
    return (WQ[a] / CS2) * (mur[IDX(i, j, nx)] + nb_mirror(mur, nx, ny, i, j, EX[a], EY[a], 0));
}

/* Residual r = L(psi0 + psi') at every node; returns max |r|. */
static double potential_residual(int nx, int ny, const real* mur, real H0, real alpha,
                                   const real* psi, const real* lo, const real* hi, real* r) {
    real hx = r_cos(alpha), hy = r_sin(alpha);
    double mx = 0.0;
#pragma omp parallel for schedule(static) reduction(max : mx)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real c0 = psi[IDX(i, j, nx)], acc = 0.0;
            for (int a = 1; a < NQ; ++a) {
                real c = coef(mur, nx, ny, i, j, a);
                acc += c * (nb_psi(psi, nx, ny, i, j, EX[a], EY[a], lo, hi) - c0);
                acc -= H0 * c * (EX[a] * hx + EY[a] * hy);
            }
            if (r) r[IDX(i, j, nx)] = acc;
            if (r_mag(acc) > mx) mx = r_mag(acc);
        }
    return mx;
}

/* Column order that keeps the periodic matrix banded: 0, nx-1, 1, nx-2, ... */
static inline int fold(int i, int nx) { return i < nx / 2 ? 2 * i : 2 * (nx - 1 - i) + 1; }

/* Exact solve of -L psi' = -H0 sum c (e.h) (+ ghost data) by banded Cholesky. */
static int potential_direct(int nx, int ny, const real* mur, real H0, real alpha, real* psi,
                            const real* lo, const real* hi) {
    size_t n = (size_t)nx * ny;
    int bw = 2 * ny + 1; /* half bandwidth under the folded ordering */
    real* L = (real*)calloc(n * (size_t)(bw + 1), sizeof(real));
    real* b = (real*)calloc(n, sizeof(real));
    int* inv = (int*)malloc(n * sizeof(int)); /* ordered index -> plane index */
    if (!L || !b || !inv) {
        free(L);
        free(b);
        free(inv);
        return -3;
    }
    real hx = r_cos(alpha), hy = r_sin(alpha);
    /* Assemble A = -L (lower band, row-wise: L[k*(bw+1) + (k-m)] = A[k][m]) and b. */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)fold(i, nx) * ny + j;
            inv[k] = (int)IDX(i, j, nx);
            real diag = 0.0, rhs = 0.0;
            for (int a = 1; a < NQ; ++a) {
                real c = coef(mur, nx, ny, i, j, a);
                diag += c;
                rhs -= H0 * c * (EX[a] * hx + EY[a] * hy);
                int jj = j + EY[a];
                if (jj < 0 || jj > ny - 1) {
                    real gv = jj < 0 ? (lo ? lo[wrap(i + EX[a], nx)] : 0.0)
                                       : (hi ? hi[wrap(i + EX[a], nx)] : 0.0);
                    rhs += c * gv;
                    continue;
                }
                size_t m = (size_t)fold(wrap(i + EX[a], nx), nx) * ny + jj;
                if (m < k) L[k * (bw + 1) + (k - m)] -= c;
            }
            L[k * (bw + 1)] += diag;
            b[k] = rhs;
        }
    /* In-place Cholesky A = C C^T on the band. */
    for (size_t k = 0; k < n; ++k) {
        size_t lo_k = k > (size_t)bw ? k - bw : 0;
        for (size_t m = lo_k; m <= k; ++m) {
            size_t lo_m = m > (size_t)bw ? m - bw : 0;
            size_t start = lo_k > lo_m ? lo_k : lo_m;
            real s = L[k * (bw + 1) + (k - m)];
            for (size_t p = start; p < m; ++p) s -= L[k * (bw + 1) + (k - p)] * L[m * (bw + 1) + (m - p)];
            if (m == k) {
                if (RE(s) <= 0.0) {
                    free(L);
                    free(b);
                    free(inv);
                    return -5;
                }
                L[k * (bw + 1)] = r_sqrt(s);
            } else {
                L[k * (bw + 1) + (k - m)] = s / L[m * (bw + 1)];
            }
        }
    }
    /* Forward substitution C y = b. */
    for (size_t k = 0; k < n; ++k) {
        size_t lo_k = k > (size_t)bw ? k - bw : 0;
        real s = b[k];
        for (size_t p = lo_k; p < k; ++p) s -= L[k * (bw + 1) + (k - p)] * b[p];
        b[k] = s / L[k * (bw + 1)];
    }
    /* Back substitution C^T x = y. */
    for (size_t kk = n; kk-- > 0;) {
        real s = b[kk];
        size_t hi_k = kk + bw < n - 1 ? kk + bw : n - 1;
        for (size_t p = kk + 1; p <= hi_k; ++p) s -= L[p * (bw + 1) + (p - kk)] * b[p];
        b[kk] = s / L[kk * (bw + 1)];
    }
    for (size_t k = 0; k < n; ++k) psi[inv[k]] = b[k];
    free(L);
    free(b);
    free(inv);
    return 0;
}

/* Four-colour SOR: colour (i mod 2) + 2 (j mod 2), colours in the order 0, 1, 2, 3;
 * nodes of one colour never neighbour each other (nx even), so their order within a
 * colour does not matter.  Warm-started from the psi' passed in. */
static int potential_sor(int nx, int ny, const real* mur, real H0, real alpha, real* psi,
                         const orc_solver* S, int* sweeps, double* resid) {
    real hx = r_cos(alpha), hy = r_sin(alpha);
    double thr = S->tol * RE(H0);
    int every = S->check_every > 0 ? S->check_every : 1;
    int sw = 0;
    double rmax = potential_residual(nx, ny, mur, H0, alpha, psi, NULL, NULL, NULL);
    while (rmax > thr && sw < S->max_sweeps) {
        for (int colour = 0; colour < 4; ++colour)
#pragma omp parallel for schedule(static)
            for (int j = colour / 2; j < ny; j += 2)
                for (int i = colour % 2; i < nx; i += 2) {
                    real C = 0.0, acc = 0.0;
                    for (int a = 1; a < NQ; ++a) {
                        real c = coef(mur, nx, ny, i, j, a);
                        C += c;
                        acc += c * nb_psi(psi, nx, ny, i, j, EX[a], EY[a], NULL, NULL);
                        acc -= H0 * c * (EX[a] * hx + EY[a] * hy);
                    }
                    real gs = acc / C;
                    real* p = &psi[IDX(i, j, nx)];
                    *p += S->omega * (gs - *p);
                }
        ++sw;
        if (sw % every == 0 || sw == S->max_sweeps)
            rmax = potential_residual(nx, ny, mur, H0, alpha, psi, NULL, NULL, NULL);
    }
    if (sweeps) *sweeps = sw;
    if (resid) *resid = rmax;
    return rmax <= thr ? 0 : -5;
}

static int solve_mu(const orc_params* P, const real* mur, const orc_solver* S, real* psi,
                    const real* lo, const real* hi, int* sweeps, double* resid) {
    int nx = P->nx, ny = P->ny;
    if (sweeps) *sweeps = 0;
    if (P->H0 == 0.0 && !lo && !hi) { /* no field: psi' = 0 exactly */
        memset(psi, 0, sizeof(real) * (size_t)nx * ny);
        if (resid) *resid = 0.0;
        return 0;
    }
    int rc;
    if (S->mode == 0) {
        rc = potential_direct(nx, ny, mur, P->H0, P->alpha, psi, lo, hi);
        if (resid) *resid = potential_residual(nx, ny, mur, P->H0, P->alpha, psi, lo, hi, NULL);
    } else {
        if (lo || hi) return -1;
        rc = potential_sor(nx, ny, mur, P->H0, P->alpha, psi, S, sweeps, resid);
    }
    return rc;
}

/* Exported: solve for psi' given phi1, phi2 planes (ghost data optional). */
int orc_solve_potential_phi(const orc_params* P, const real* phi1, const real* phi2,
                            const orc_solver* S, real* psi, const real* ghost_lo,
                            const real* ghost_hi, int32_t* sweeps, double* resid) {
    size_t n = (size_t)P->nx * P->ny;
    real* mur = (real*)malloc(n * sizeof(real));
    if (!mur) return -3;
    mu_r_from_phi(P, phi1, phi2, mur);
    int sw = 0;
    int rc = solve_mu(P, mur, S, psi, ghost_lo, ghost_hi, &sw, resid);
    if (sweeps) *sweeps = sw;
    free(mur);
    return rc;
}

/* Exported: residual max |L(psi0+psi')| for given phi planes and psi'. */
double orc_potential_residual_phi(const orc_params* P, const real* phi1, const real* phi2,
                                  const real* psi, real* r_out) {
    size_t n = (size_t)P->nx * P->ny;
    real* mur = (real*)malloc(n * sizeof(real));
    if (!mur) return -1.0;
    mu_r_from_phi(P, phi1, phi2, mur);
    double m = potential_residual(P->nx, P->ny, mur, P->H0, P->alpha, psi, NULL, NULL, r_out);
    free(mur);
    return m;
}

/* Exported: apply the discrete operator L_mu (without psi0) to u; ghost rows of u are 0. */
void orc_apply_L(const orc_params* P, const real* mur, const real* u, real* out) {
    int nx = P->nx, ny = P->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real c0 = u[IDX(i, j, nx)], acc = 0.0;
            for (int a = 1; a < NQ; ++a)
                acc += coef(mur, nx, ny, i, j, a) * (nb_psi(u, nx, ny, i, j, EX[a], EY[a], NULL, NULL) - c0);
            out[IDX(i, j, nx)] = acc;
        }
}

/* ------------------------------------------------------------------------- */
/* Initial state (reading: the paper gives no initial profile, pressure or     */
/* velocity; tanh interfaces, p* = 0, f = f^eq, g = phi Gamma).                */
/* ------------------------------------------------------------------------- */

/* f = f^eq(p*, u), g^i = phi_i Gamma(u). */
int orc_init_fields(const orc_params* P, const real* phi1, const real* phi2, const real* ux,
                    const real* uy, const real* pstar, real* f, real* g1, real* g2) {
    size_t n = (size_t)P->nx * P->ny;
    for (size_t k = 0; k < n; ++k) {
        real u[2] = {ux[k], uy[k]}, fe[NQ], G[NQ];
        orc_feq(pstar ? pstar[k] : 0.0, u, fe);
        orc_gamma(u, G);
        for (int a = 0; a < NQ; ++a) {
            f[a * n + k] = fe[a];
            g1[a * n + k] = phi1[k] * G[a];
            g2[a * n + k] = phi2[k] * G[a];
        }
    }
    return 0;
}

/* Eq. 37: inlet velocity u_avg 4 (y/H)(1 - y/H) with the walls at y = 0 and y = H = ny,
 * i.e. y = j + 1/2 at row j.  Reading: taken as printed, so u_avg is the centreline value
 * and the mean over the section is (2/3) u_avg. */
static real inlet_u(const orc_params* P, int j) {
    real s = (j + 0.5) / P->ny;
    return 4.0 * P->u_inlet * s * (1.0 - s);
}

/* Concentric tanh profiles (width xi) about (xc, yc), minimum image in x (plain distance
 * in the open channel); ambient velocity: the Poiseuille profile under the drive, or the
 * Eq. 37 profile in every column of the open channel; p* = 0. Writes phi1, phi2 too. */
int orc_init_droplet(const orc_params* P, double xc, double yc, double r_core, double r_shell,
                     real* f, real* g1, real* g2, real* phi1, real* phi2) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    real* ux = (real*)malloc(n * sizeof(real));
    real* uy = (real*)calloc(n, sizeof(real));
    if (!ux || !uy) {
        free(ux);
        free(uy);
        return -3;
    }
    real nu3 = CS2 * P->tau[2];
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double dx = (double)i - xc;
            if (!P->open_x) dx -= nx * floor(dx / nx + 0.5);
            double dy = (double)j - yc;
            double d = sqrt(dx * dx + dy * dy);
            real pin = 0.5 * (1.0 + r_tanh(2.0 * (r_core - d) / P->xi));
            real pout = 0.5 * (1.0 + r_tanh(2.0 * (r_shell - d) / P->xi));
            phi1[IDX(i, j, nx)] = pin;
            phi2[IDX(i, j, nx)] = pout - pin;
            ux[IDX(i, j, nx)] = P->open_x ? inlet_u(P, j)
                                          : P->drive_G / (2.0 * P->rho[2] * nu3) * (j + 0.5) * (ny - 0.5 - j);
        }
    orc_init_fields(P, phi1, phi2, ux, uy, NULL, f, g1, g2);
    free(ux);
    free(uy);
    return 0;
}

/* Open channel: the populations that streaming cannot supply at the end columns.
 * Inlet i = 0 (unknown directions 1, 5, 8, i.e. e_x = +1), the velocity condition of
 * Eq. 37 in the Zou-He manner: the first moment of f is set to j = (u_in(y), 0) and the
 * non-equilibrium part of f_1 equals that of its opposite f_3; f_eq,1 - f_eq,3 =
 * Gamma_1 - Gamma_3 = (2/3) u_x (Eq. 16, 18).  The two first-moment equations then fix
 * f_5 and f_8.  p* needs no closure: it is whatever the sum of the completed set gives.
 * Reading: the prescribed velocity is the first moment of f, which equals the u of
 * Eq. 22 where the inflowing fluid carries no force.
 * The order parameters enter at equilibrium with the inflow's composition (reading:
 * carrier only, phi_1 = phi_2 = 0): g^i_a = phi_in Gamma_a(u_in) (Eq. 31 without the
 * interface term, which vanishes in a uniform phase).
 * Outlet i = nx - 1 (unknown directions 3, 6, 7), the convective condition
 * d f/dt + U d f/dx = 0 discretised as f(t+1, N) = [f(t, N) + U f(t+1, N-1)] / (1 + U)
 * for f, g1 and g2.  Reading: U, which the paper does not give, is the mean inlet
 * velocity over the section (by continuity the mean outflow velocity). */
static void open_boundaries(const orc_params* P, const real* out_old, real* f, real* g1, real* g2) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    real U = 0.0;
    for (int j = 0; j < ny; ++j) U += inlet_u(P, j);
    U /= ny;
    const real phi_in[2] = {0.0, 0.0};
    for (int j = 0; j < ny; ++j) {
        /* inlet */
        size_t k = IDX(0, j, nx);
        real ux = inlet_u(P, j), uy = 0.0;
        real f2 = f[2 * n + k], f3 = f[3 * n + k], f4 = f[4 * n + k], f6 = f[6 * n + k], f7 = f[7 * n + k];
        f[1 * n + k] = f3 + (2.0 / 3.0) * ux;
        f[5 * n + k] = f7 - 0.5 * (f2 - f4) + ux / 6.0 + 0.5 * uy;
        f[8 * n + k] = f6 + 0.5 * (f2 - f4) + ux / 6.0 - 0.5 * uy;
        real u[2] = {ux, uy}, G[NQ];
        orc_gamma(u, G);
        const int in_dirs[3] = {1, 5, 8};
        for (int d = 0; d < 3; ++d) {
            int a = in_dirs[d];
            g1[a * n + k] = phi_in[0] * G[a];
            g2[a * n + k] = phi_in[1] * G[a];
        }
        /* outlet */
        size_t ko = IDX(nx - 1, j, nx), kb = IDX(nx - 2, j, nx);
        const int out_dirs[3] = {3, 6, 7};
        for (int d = 0; d < 3; ++d) {
            int a = out_dirs[d];
            f[a * n + ko] = (out_old[(0 * NQ + a) * ny + j] + U * f[a * n + kb]) / (1.0 + U);
            g1[a * n + ko] = (out_old[(1 * NQ + a) * ny + j] + U * g1[a * n + kb]) / (1.0 + U);
            g2[a * n + ko] = (out_old[(2 * NQ + a) * ny + j] + U * g2[a * n + kb]) / (1.0 + U);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* The coupled step.  Reading: the algorithm figure is missing; the order is   */
/* phases -> potential -> stencils and forces -> collisions -> streaming.      */
/* ------------------------------------------------------------------------- */
int orc_step(const orc_params* P, const orc_solver* S, int32_t nsteps, int32_t step0, real* f, real* g1,
             real* g2, real* psi, int32_t* total_sweeps, double* last_resid) {
    int nx = P->nx, ny = P->ny;
    if (nx < 4 || ny < 2 || (nx % 2)) return -1;
    size_t n = (size_t)nx * ny;
    real* phi1 = (real*)malloc(n * sizeof(real));
    real* phi2 = (real*)malloc(n * sizeof(real));
    real* mur = (real*)malloc(n * sizeof(real));
    real* fp = (real*)malloc(NQ * n * sizeof(real));
    real* g1p = (real*)malloc(NQ * n * sizeof(real));
    real* g2p = (real*)malloc(NQ * n * sizeof(real));
    real* out_old = (real*)malloc(3 * NQ * (size_t)ny * sizeof(real));
    int rc = 0;
    if (!phi1 || !phi2 || !mur || !fp || !g1p || !g2p || !out_old) {
        rc = -3;
        goto done;
    }
    if (total_sweeps) *total_sweeps = 0;
    if (!minv_ready) build_minv(); /* before any threads share it */
    for (int step = 0; step < nsteps; ++step) {
        /* Order parameters (Eq. 32, 24) and mu_r (Eq. 8). */
        phase_from_g(nx, ny, g1, phi1);
        phase_from_g(nx, ny, g2, phi2);
        mu_r_from_phi(P, phi1, phi2, mur);
        /* Potential from phi(t), warm start from the previous psi'.  Quasi-static option
         * (not the paper's coupling, which solves every step): solved only on the steps
         * step0 + step = 0, K, 2K, ... counted from the initial state, psi' held between. */
        if ((step0 + step) % (S->every > 1 ? S->every : 1) == 0) {
            int sw = 0;
            double res = 0.0;
            rc = solve_mu(P, mur, S, psi, NULL, NULL, &sw, &res);
            if (total_sweeps) *total_sweeps += sw;
            if (last_resid) *last_resid = res;
            if (rc != 0) goto done;
        }
        /* Stencils, forces and both collisions at every node (rows independent: with
         * OpenMP they are shared out among threads, the arithmetic per node unchanged). */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = IDX(i, j, nx);
                real fn[NQ], gn1[NQ], gn2[NQ], fo[NQ], go1[NQ], go2[NQ];
                for (int a = 0; a < NQ; ++a) {
                    fn[a] = f[a * n + k];
                    gn1[a] = g1[a * n + k];
                    gn2[a] = g2[a * n + k];
                }
                nodeq q;
                node_quantities(P, phi1, phi2, psi, fn, i, j, &q);
                orc_collide_f(fn, q.pstar, q.u, q.Ft, q.rho, q.tau, fo);
                collide_g(P, &q, 0, gn1, go1);
                collide_g(P, &q, 1, gn2, go2);
                for (int a = 0; a < NQ; ++a) {
                    fp[a * n + k] = fo[a];
                    g1p[a * n + k] = go1[a];
                    g2p[a * n + k] = go2[a];
                }
            }
        /* Open channel: the outlet column before streaming, for the convective condition. */
        if (P->open_x)
            for (int j = 0; j < ny; ++j)
                for (int a = 0; a < NQ; ++a) {
                    size_t k = IDX(nx - 1, j, nx);
                    out_old[(0 * NQ + a) * ny + j] = f[a * n + k];
                    out_old[(1 * NQ + a) * ny + j] = g1[a * n + k];
                    out_old[(2 * NQ + a) * ny + j] = g2[a * n + k];
                }
        /* Pull streaming; halfway bounce-back when the source lies beyond a wall
         * (reading: the paper says bounce-back without naming the variant).  In the open
         * channel a source beyond the inlet or outlet is unknown: set just below. */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = IDX(i, j, nx);
                for (int a = 0; a < NQ; ++a) {
                    int js = j - EY[a], is = i - EX[a];
                    size_t src;
                    int as;
                    if (js < 0 || js > ny - 1) {
                        src = k;
                        as = OPP[a];
                    } else if (P->open_x && (is < 0 || is > nx - 1)) {
                        continue;
                    } else {
                        src = IDX(wrap(is, nx), js, nx);
                        as = a;
                    }
                    f[a * n + k] = fp[as * n + src];
                    g1[a * n + k] = g1p[as * n + src];
                    g2[a * n + k] = g2p[as * n + src];
                }
            }
        if (P->open_x) open_boundaries(P, out_old, f, g1, g2);
    }
done:
    free(phi1);
    free(phi2);
    free(mur);
    free(fp);
    free(g1p);
    free(g2p);
    free(out_old);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Moments and diagnostics.                                                   */
/* ------------------------------------------------------------------------- */

/* Planes [10][ny][nx]: p*, ux, uy, phi1, phi2, phi3, rho, psi', Hx, Hy, with u the
 * force-corrected velocity of Eq. 22 evaluated from the stored psi'. */
int orc_moments(const orc_params* P, const real* f, const real* g1, const real* g2,
                const real* psi, real* out) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    real* phi1 = (real*)malloc(n * sizeof(real));
    real* phi2 = (real*)malloc(n * sizeof(real));
    if (!phi1 || !phi2) {
        free(phi1);
        free(phi2);
        return -3;
    }
    phase_from_g(nx, ny, g1, phi1);
    phase_from_g(nx, ny, g2, phi2);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = IDX(i, j, nx);
            real fn[NQ];
            for (int a = 0; a < NQ; ++a) fn[a] = f[a * n + k];
            nodeq q;
            node_quantities(P, phi1, phi2, psi, fn, i, j, &q);
            out[0 * n + k] = q.pstar;
            out[1 * n + k] = q.u[0];
            out[2 * n + k] = q.u[1];
            out[3 * n + k] = q.phi[0];
            out[4 * n + k] = q.phi[1];
            out[5 * n + k] = q.phi[2];
            out[6 * n + k] = q.rho;
            out[7 * n + k] = psi[k];
            out[8 * n + k] = q.H[0];
            out[9 * n + k] = q.H[1];
        }
    free(phi1);
    free(phi2);
    return 0;
}

/* Forces at every node (for the force tests): planes [8][ny][nx] =
 * Fs_x, Fs_y, Fm_x, Fm_y, Fmu_x, Fmu_y, Ft_x, Ft_y. */
int orc_forces(const orc_params* P, const real* f, const real* g1, const real* g2,
               const real* psi, real* out) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    real* phi1 = (real*)malloc(n * sizeof(real));
    real* phi2 = (real*)malloc(n * sizeof(real));
    if (!phi1 || !phi2) {
        free(phi1);
        free(phi2);
        return -3;
    }
    phase_from_g(nx, ny, g1, phi1);
    phase_from_g(nx, ny, g2, phi2);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = IDX(i, j, nx);
            real fn[NQ];
            for (int a = 0; a < NQ; ++a) fn[a] = f[a * n + k];
            nodeq q;
            node_quantities(P, phi1, phi2, psi, fn, i, j, &q);
            out[0 * n + k] = q.Fs[0];
            out[1 * n + k] = q.Fs[1];
            out[2 * n + k] = q.Fm[0];
            out[3 * n + k] = q.Fm[1];
            out[4 * n + k] = q.Fmu[0];
            out[5 * n + k] = q.Fmu[1];
            out[6 * n + k] = q.Ft[0];
            out[7 * n + k] = q.Ft[1];
        }
    free(phi1);
    free(phi2);
    return 0;
}

/* Second-moment deformation of a weight field w (a differentiable stand-in for the
 * extent-based index of Eq. 42, equal to it for an ellipse): centroid with a circular mean
 * in periodic x, I_xx and I_yy about it, D = (sqrt Iyy - sqrt Ixx)/(sqrt Iyy + sqrt Ixx). */
real orc_deformation_w(int32_t nx, int32_t ny, const real* w) {
    const double twopi = 6.283185307179586476925286766559;
    real sw = 0.0, sc = 0.0, ss = 0.0, sy = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real v = w[IDX(i, j, nx)];
            sw += v;
            sc += v * cos(twopi * i / nx);
            ss += v * sin(twopi * i / nx);
            sy += v * j;
        }
    real xc = nx * r_atan2(ss, sc) / twopi;
    real yc = sy / sw;
    real ixx = 0.0, iyy = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real v = w[IDX(i, j, nx)];
            real dx = (double)i - xc;
            dx -= nx * floor(RE(dx) / nx + 0.5);
            real dy = (double)j - yc;
            ixx += v * dx * dx;
            iyy += v * dy * dy;
        }
    ixx /= sw;
    iyy /= sw;
    return (r_sqrt(iyy) - r_sqrt(ixx)) / (r_sqrt(iyy) + r_sqrt(ixx));
}

/* out = {D_o (w = 1 - phi3), D_i (w = phi1), sum phi1, sum phi2}. */
int orc_diagnostics(const orc_params* P, const real* g1, const real* g2, real out[4]) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    real* phi1 = (real*)malloc(n * sizeof(real));
    real* phi2 = (real*)malloc(n * sizeof(real));
    real* wo = (real*)malloc(n * sizeof(real));
    if (!phi1 || !phi2 || !wo) {
        free(phi1);
        free(phi2);
        free(wo);
        return -3;
    }
    phase_from_g(nx, ny, g1, phi1);
    phase_from_g(nx, ny, g2, phi2);
    real m1 = 0.0, m2 = 0.0;
    for (size_t k = 0; k < n; ++k) {
        wo[k] = phi1[k] + phi2[k];
        m1 += phi1[k];
        m2 += phi2[k];
    }
    out[0] = orc_deformation_w(nx, ny, wo);
    out[1] = orc_deformation_w(nx, ny, phi1);
    out[2] = m1;
    out[3] = m2;
    free(phi1);
    free(phi2);
    free(wo);
    return 0;
}

#ifndef ORC_COMPLEX_STEP
/* Extent-based deformation index of Eq. 42, T = (l_y - l_x) / (l_y + l_x), of the
 * outer droplet (w = phi1 + phi2) and the inner one (w = phi1), the interface at w = 1/2.
 * Reading: l_y is the largest vertical extent over the columns: in each column the longest
 * run of rows with w >= 1/2, from its linearly interpolated lower crossing to its upper one
 * (a run reaching a wall row ends at the wall, half a node beyond the row); l_x is the
 * length of the longest run with w >= 1/2 of the centreline profile (the middle row, or the
 * mean of the two middle rows when ny is even), periodic in x, between its interpolated
 * crossings (nx when the run closes on itself).  T = 0 when both extents vanish. */
static double run_crossing(double wa, double wb) { return (0.5 - wa) / (wb - wa); }

static double column_extent(int nx, int ny, const double* w, int i) {
    double best = 0.0;
    int j = 0;
    while (j < ny) {
        if (w[IDX(i, j, nx)] < 0.5) {
            ++j;
            continue;
        }
        int j0 = j;
        while (j < ny && w[IDX(i, j, nx)] >= 0.5) ++j;
        int j1 = j - 1; /* last row of the run */
        double lo = j0 == 0 ? -0.5 : (j0 - 1) + run_crossing(w[IDX(i, j0 - 1, nx)], w[IDX(i, j0, nx)]);
        double hi = j1 == ny - 1 ? ny - 0.5 : j1 + 1.0 - run_crossing(w[IDX(i, j1 + 1, nx)], w[IDX(i, j1, nx)]);
        if (hi - lo > best) best = hi - lo;
    }
    return best;
}

static double centreline_extent(int nx, const double* c) {
    int all = 1;
    for (int i = 0; i < nx; ++i)
        if (c[i] < 0.5) all = 0;
    if (all) return (double)nx;
    double best = 0.0;
    /* start every run scan just after a node below 1/2, so runs are never cut by the seam */
    int s = 0;
    while (c[s] >= 0.5) ++s;
    for (int t = 1; t <= nx; ++t) {
        int i = (s + t) % nx;
        if (c[i] < 0.5) continue;
        int prev = (i - 1 + nx) % nx; /* below 1/2: a run starts at i */
        if (c[prev] >= 0.5) continue;
        int len = 0;
        while (c[(i + len) % nx] >= 0.5) ++len;
        int last = (i + len - 1) % nx, next = (i + len) % nx;
        double left = run_crossing(c[prev], c[i]);          /* fraction of the gap before i */
        double right = run_crossing(c[next], c[last]);      /* fraction of the gap after last */
        double ext = (len - 1) + (1.0 - left) + (1.0 - right);
        if (ext > best) best = ext;
    }
    return best;
}

int orc_extent_deformation(const orc_params* P, const double* g1, const double* g2, double out[6]) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    double* phi1 = (double*)malloc(n * sizeof(double));
    double* phi2 = (double*)malloc(n * sizeof(double));
    double* wo = (double*)malloc(n * sizeof(double));
    double* cl = (double*)malloc(2 * (size_t)nx * sizeof(double));
    if (!phi1 || !phi2 || !wo || !cl) {
        free(phi1);
        free(phi2);
        free(wo);
        free(cl);
        return -3;
    }
    phase_from_g(nx, ny, g1, phi1);
    phase_from_g(nx, ny, g2, phi2);
    for (size_t k = 0; k < n; ++k) wo[k] = phi1[k] + phi2[k];
    const double* w[2] = {wo, phi1};
    for (int d = 0; d < 2; ++d) {
        double ly = 0.0;
        for (int i = 0; i < nx; ++i) {
            double e = column_extent(nx, ny, w[d], i);
            if (e > ly) ly = e;
        }
        double* c = cl + (size_t)d * nx;
        for (int i = 0; i < nx; ++i)
            c[i] = (ny % 2) ? w[d][IDX(i, ny / 2, nx)] : 0.5 * (w[d][IDX(i, ny / 2 - 1, nx)] + w[d][IDX(i, ny / 2, nx)]);
        double lx = centreline_extent(nx, c);
        out[2 + 2 * d] = ly;
        out[3 + 2 * d] = lx;
        out[d] = (ly + lx > 0.0) ? (ly - lx) / (ly + lx) : 0.0;
    }
    free(phi1);
    free(phi2);
    free(wo);
    free(cl);
    return 0;
}

/* Breakup probe (Sec. 2.5: breakup is the inner droplet touching the shell's interface).
 * Reading: a contact node is a node of the core (phi1 >= 1/2) with a nine-point neighbour
 * in the carrier (phi3 >= 1/2; columns periodic, no neighbours beyond the walls): no shell
 * node separates them there.  out = {number of contact nodes, their mean y, their circular
 * mean x (angle 2 pi x / nx), the circular mean x of the outer droplet weighted by
 * phi1 + phi2}; the two x means are -1 where their weights vanish. */
int orc_breakup_probe(const orc_params* P, const double* g1, const double* g2, double out[4]) {
    int nx = P->nx, ny = P->ny;
    size_t n = (size_t)nx * ny;
    double* phi1 = (double*)malloc(n * sizeof(double));
    double* phi2 = (double*)malloc(n * sizeof(double));
    if (!phi1 || !phi2) {
        free(phi1);
        free(phi2);
        return -3;
    }
    phase_from_g(nx, ny, g1, phi1);
    phase_from_g(nx, ny, g2, phi2);
    const double two_pi = 6.283185307179586;
    double cnt = 0.0, sy = 0.0, sc = 0.0, ss = 0.0, oc = 0.0, os = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = IDX(i, j, nx);
            double th = two_pi * i / nx;
            double wo = phi1[k] + phi2[k];
            oc += wo * cos(th);
            os += wo * sin(th);
            if (phi1[k] < 0.5) continue;
            int touch = 0;
            for (int dj = -1; dj <= 1 && !touch; ++dj)
                for (int di = -1; di <= 1 && !touch; ++di) {
                    int jj = j + dj;
                    if ((di == 0 && dj == 0) || jj < 0 || jj >= ny) continue;
                    size_t kk = IDX(wrap(i + di, nx), jj, nx);
                    if (1.0 - phi1[kk] - phi2[kk] >= 0.5) touch = 1;
                }
            if (!touch) continue;
            cnt += 1.0;
            sy += j;
            sc += cos(th);
            ss += sin(th);
        }
    out[0] = cnt;
    out[1] = cnt > 0.0 ? sy / cnt : -1.0;
    double a = atan2(ss, sc), ao = atan2(os, oc);
    out[2] = cnt > 0.0 ? (a < 0.0 ? a + two_pi : a) * nx / two_pi : -1.0;
    out[3] = (oc != 0.0 || os != 0.0) ? (ao < 0.0 ? ao + two_pi : ao) * nx / two_pi : -1.0;
    free(phi1);
    free(phi2);
    return 0;
}

#endif /* ORC_COMPLEX_STEP */

/* Exported for the stencil tests: Eq. 34 gradient and Eq. 35 Laplacian of a plane
 * with the mirror ghost rule. */
void orc_stencils(int32_t nx, int32_t ny, const real* a, real* gx, real* gy, real* lap) {
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real g[2];
            iso_grad(a, nx, ny, i, j, 0, g);
            gx[IDX(i, j, nx)] = g[0];
            gy[IDX(i, j, nx)] = g[1];
            lap[IDX(i, j, nx)] = iso_lap(a, nx, ny, i, j, 0);
        }
}

/* Exported: mu_r plane from phi planes (Eq. 8). */
void orc_mu_r(const orc_params* P, const real* phi1, const real* phi2, real* mur) {
    mu_r_from_phi(P, phi1, phi2, mur);
}

/* Threads the row loops use (1 without OpenMP): reported beside CPU timings. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
