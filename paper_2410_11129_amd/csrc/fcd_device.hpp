// fcd_device.hpp -- per-node physics of the coupled step, as device functions shared
// by the step, moment and diagnostic kernels (gfx950, wave64).
//
// The node update follows arXiv:2410.11129 Sec. 2.1-2.4:
//   order parameters (Eq. 32, 24), isotropic gradient / Laplacian (Eq. 34-35),
//   Boyer-Lapuerta chemical potentials (Eq. 25-28) and surface tension (Eq. 36),
//   field H = -grad psi (Eq. 5) and Kelvin force (Eq. 7, 9),
//   pressure and viscous forces (Sec. 2.2 after Eq. 19), velocity (Eq. 21-22),
//   MRT collision with forcing (Eq. 12-19), phase-field collision (Eq. 29-31).
// Where the paper is garbled or silent the same readings as the library documents
// are taken: Gamma with -u.u/(2 c_s^2); Lambda = diag(1,...,1, s_nu, s_nu); gamma_i in
// the Laplacian term of Eq. 25; harmonic mixing of 1 + chi; linear mixing of tau;
// F_mu from the local non-equilibrium stress; phase-field source
// w e.[theta_i n_i - (1/3) sum_k theta_k n_k]; mirror ghost rows for phi, zero psi'.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcd {

// Constants of one step in the working precision T, prepared on the host.
template <typename T>
struct StepConst {
    int nx, ny, pitch;
    int pad;
    long long plane;  // ny * pitch
    T rho0, rho1, rho2;
    T tau0, tau1, tau2;
    T ic0, ic1, ic2;          // 1 / (1 + chi_i)
    T gam0, gam1, gam2;       // gamma_i of Eq. 27
    T igam0, igam1, igam2;    // 1 / gamma_i
    T s12, s13, s23, eta;     // surface tensions, total-spreading coefficient
    T c_bulk;                 // 4 gamma_T / xi (Eq. 25-26)
    T c_lap;                  // 3 xi / 4 (Eq. 25)
    T four_over_xi;           // theta = (4/xi) phi (1 - phi)
    T omega_phi;              // 1 / (tau_phi + 1/2), tau_phi = M / c_s^2 (Eq. 29-30)
    T H0x, H0y;               // H0 (cos alpha, sin alpha)
    T half_mu0;
    T drive, grav_x, grav_y;
    T eps2;                   // eps_n^2
    T u_limit;                // divergence guard: largest admissible max(|u_x|, |u_y|)
};

// The outcome of a residual test, read on the device from the test's two words (max
// |residual| and max |C psi'| as bit patterns of non-negative doubles; both zero when the
// test did not run): passed when r <= max(thr0, floor_factor * scale).  A NaN residual
// does not pass.  res == nullptr: no test (nothing is gated).  The words are written and
// cleared by earlier kernels on the same stream only.
struct ResGate {
    const unsigned long long* res;
    double thr0, floor_factor;
    __device__ __forceinline__ bool passed() const {
        const double r = __longlong_as_double((long long)res[0]);
        const double sc = __longlong_as_double((long long)res[1]);
        return r <= fmax(thr0, floor_factor * sc);
    }
};

// One level of the potential problem (see fcd_potential.hip).  f == nullptr marks the
// finest level, whose right-hand side H0 sum_a c_a (e_a . h) is formed on the fly.
template <typename T>
struct PotLevel {
    T* u;         // unknown: psi' on the finest level, the correction on coarse levels
    const T* mu;  // mu_r (finest) or its cell averages (coarse)
    T* f;         // right-hand side, nullptr on the finest level
    // a kernel given this level does nothing when gate.res is set and that test passed
    // (the V-cycle it belongs to is not needed)
    ResGate gate;
    int nx, ny, pitch, pad;
    T inv_h2;     // 1 / h^2, h = 2^level
    T kappa;      // the ghost row below the first row carries -kappa times it: (h - 1) / (h + 1)
    T kappa_top;  // the ghost row above the last row carries -kappa_top times it (wall distance)
    T H0x, H0y;   // applied field (finest level only)
};

// The residual tests of a time step's solve (the rotating slots), the number of tests that
// ran since the last publication and the divergence flag word, as the step's
// collide-and-stream publishes them to pinned host memory; seq is stored last.
constexpr int SOLVE_SLOTS = 8;
struct SolveMirror {
    unsigned long long seq;
    double r[SOLVE_SLOTS], scale[SOLVE_SLOTS];
    unsigned tests, pad_;
    unsigned long long div;
};

// The launch that ends a batch of a solve decided on the device (the collide-and-stream
// of a time step, or a one-lane publication): with gate.res set, the collide-and-stream
// runs only if that test passed; one lane first publishes the slots, the test count
// (then zeroed) and the divergence word to m under the sequence number seq, and zeroes
// the two words at clear (the next test's).
struct StepGate {
    ResGate gate;
    const unsigned long long* slots;
    unsigned long long* clear;
    unsigned* tests;
    SolveMirror* m;
    const unsigned long long* div;
    unsigned long long seq;
};

// The publication of a StepGate, by one lane; the host polls m->seq (stored last).
__device__ __forceinline__ void publish_tests(const StepGate& sg) {
    SolveMirror* m = sg.m;
    for (int q = 0; q < SOLVE_SLOTS; ++q) {
        m->r[q] = __longlong_as_double((long long)sg.slots[2 * q]);
        m->scale[q] = __longlong_as_double((long long)sg.slots[2 * q + 1]);
    }
    m->tests = *sg.tests;
    m->div = *sg.div;
    *sg.tests = 0u;
    sg.clear[0] = 0ULL;
    sg.clear[1] = 0ULL;
    __hip_atomic_store(&m->seq, sg.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The coarsest levels of a V-cycle, solved in LDS by one block (levels lv[0..n), finest
// first; lv[0].f holds the restricted residual, lv[0].u receives the correction).
constexpr int MG_MAX_TAIL = 8;
// Up to four successive coarse mu levels (cell averages) written by one launch.
template <typename T>
struct MuLevels {
    T* mu[4];
    int nx[4], ny[4], pitch[4];
    int n;
};

template <typename T>
struct MgTail {
    PotLevel<T> lv[MG_MAX_TAIL];
    int n, nu1, nu2, coarse_sweeps;
    T omega;  // SOR factor of the coarsest-level sweeps
};

// ceil(2^32 / nx) of every tail level (see fcd_potential.hip).
struct TailDiv {
    unsigned inv[MG_MAX_TAIL];
};

// Levels of a multigrid hierarchy at most.
constexpr int MG_MAX_LEVELS = 16;

// One channel's multigrid hierarchy as the batched multigrid kernels see it (device
// memory): the finest level (u = psi', mu = mu_r, f = nullptr) and its ping-pong plane,
// the FP32 coarse levels 1 .. levels-1 with the smoothers' second planes, and the tail
// (levels tail .. levels-1) with its divisors.  Levels 1 .. tail-1 are smoothed by tiles.
template <typename T, typename TC>
struct MgChan {
    PotLevel<T> L0;
    T* t0;
    PotLevel<TC> C[MG_MAX_LEVELS];
    TC* t[MG_MAX_LEVELS];
    MgTail<TC> tl;
    TailDiv dv;
    MuLevels<TC> mu4[4];  // coarse mu written from level 4g: levels 4g+1 .. 4g+4 (those that exist)
    int levels, tail;
    double thr;  // the channel stops when max |residual| <= max(thr, rounding floor)
};

// A block's work in a batched multigrid launch: channel k, level l, tile (bx, by).
struct MgJob {
    int k, l, bx, by;
};

template <typename T>
__global__ void k_fill(T* __restrict__ a, long long n, T v) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// Values of a plane on the 3x3 neighbourhood of a node.
template <typename T>
struct Nb9 {
    T c, e, n, w, s, ne, nw, sw, se;
};

// Row offsets of the neighbourhood: periodic columns, rows clamped to the channel
// (the clamp realises the mirror ghost rule for phi and mu_r).
struct NbIdx {
    long long c, e, w, n, s, ne, nw, sw, se;
};

__device__ __forceinline__ NbIdx nb_index(int i, int j, int nx, int ny, int pitch) {
    int im = i == 0 ? nx - 1 : i - 1;
    int ip = i == nx - 1 ? 0 : i + 1;
    int jm = j == 0 ? 0 : j - 1;
    int jp = j == ny - 1 ? ny - 1 : j + 1;
    long long r0 = (long long)j * pitch, rm = (long long)jm * pitch, rp = (long long)jp * pitch;
    NbIdx x;
    x.c = r0 + i;
    x.e = r0 + ip;
    x.w = r0 + im;
    x.n = rp + i;
    x.s = rm + i;
    x.ne = rp + ip;
    x.nw = rp + im;
    x.sw = rm + im;
    x.se = rm + ip;
    return x;
}

template <typename T>
__device__ __forceinline__ Nb9<T> load_nb(const T* __restrict__ a, const NbIdx& x) {
    Nb9<T> v;
    v.c = a[x.c];
    v.e = a[x.e];
    v.w = a[x.w];
    v.n = a[x.n];
    v.s = a[x.s];
    v.ne = a[x.ne];
    v.nw = a[x.nw];
    v.sw = a[x.sw];
    v.se = a[x.se];
    return v;
}

// psi' neighbourhood: rows beyond the walls hold psi' = 0.
template <typename T>
__device__ __forceinline__ Nb9<T> load_nb_psi(const T* __restrict__ a, const NbIdx& x, int j, int ny) {
    Nb9<T> v = load_nb(a, x);
    if (j == 0) v.s = v.sw = v.se = T(0);
    if (j == ny - 1) v.n = v.ne = v.nw = T(0);
    return v;
}

// Eq. 34: grad a = 3 sum w e a(x+e): axis weight 1/9 -> 1/3, diagonal 1/36 -> 1/12.
template <typename T>
__host__ __device__ __forceinline__ void iso_grad(const Nb9<T>& v, T& gx, T& gy) {
    const T third = T(1) / T(3), twelfth = T(1) / T(12);
    T d1 = v.ne - v.sw, d2 = v.se - v.nw;
    gx = third * (v.e - v.w) + twelfth * (d1 + d2);
    gy = third * (v.n - v.s) + twelfth * (d1 - d2);
}

// Eq. 35: lap a = 6 sum w (a(x+e) - a(x)) = 2/3 sum_axis + 1/6 sum_diag - 10/3 a.
template <typename T>
__host__ __device__ __forceinline__ T iso_lap(const Nb9<T>& v) {
    return T(2) / T(3) * ((v.e + v.w) + (v.n + v.s)) + T(1) / T(6) * ((v.ne + v.sw) + (v.nw + v.se)) -
           T(10) / T(3) * v.c;
}

// Everything the two collisions need at one node.
template <typename T>
struct NodeOut {
    T pstar, ux, uy;       // p* (Eq. 21), u (Eq. 22)
    T Ftx, Fty;            // total force F_t
    T rho, tau;            // mixture density and relaxation time
    T inv_rho, snu;        // 1 / rho, s_nu = 1 / (tau + 1/2)
    T phi1, phi2;          // order parameters
    T v1x, v1y, v2x, v2y;  // theta_i n_i - (1/3) sum_k theta_k n_k for i = 1, 2
    T Hx, Hy;              // magnetic field
};

template <typename T>
__host__ __device__ __forceinline__ T rsqrt_t(T x);
template <>
__host__ __device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }
template <>
__host__ __device__ __forceinline__ float rsqrt_t<float>(float x) { return 1.0f / sqrtf(x); }

// Stencils, forces and velocity at one node from the local f, the phi1 / phi2 and
// psi' neighbourhoods.
template <typename T>
__host__ __device__ __forceinline__ NodeOut<T> node_physics(const StepConst<T>& P, const T f[9], const Nb9<T>& a1,
                                                   const Nb9<T>& a2, const Nb9<T>& ps) {
    NodeOut<T> o;
    const T p1 = a1.c, p2 = a2.c, p3 = T(1) - p1 - p2;  // Eq. 24
    T g1x, g1y, g2x, g2y;
    iso_grad(a1, g1x, g1y);
    iso_grad(a2, g2x, g2y);
    const T l1 = iso_lap(a1), l2 = iso_lap(a2);
    const T g3x = -(g1x + g2x), g3y = -(g1y + g2y), l3 = -(l1 + l2);

    // Interface normals (regularised) and the counter-diffusion fluxes of Eq. 23.
    const T t1 = P.four_over_xi * p1 * (T(1) - p1);
    const T t2 = P.four_over_xi * p2 * (T(1) - p2);
    const T t3 = P.four_over_xi * p3 * (T(1) - p3);
    const T r1 = t1 * rsqrt_t(g1x * g1x + g1y * g1y + P.eps2);
    const T r2 = t2 * rsqrt_t(g2x * g2x + g2y * g2y + P.eps2);
    const T r3 = t3 * rsqrt_t(g3x * g3x + g3y * g3y + P.eps2);
    const T sx = (r1 * g1x + r2 * g2x + r3 * g3x) * (T(1) / T(3));
    const T sy = (r1 * g1y + r2 * g2y + r3 * g3y) * (T(1) / T(3));
    o.v1x = r1 * g1x - sx;
    o.v1y = r1 * g1y - sy;
    o.v2x = r2 * g2x - sx;
    o.v2y = r2 * g2y - sy;

    // Mixture closure (Eq. 33; linear tau).
    const T rho = P.rho0 * p1 + P.rho1 * p2 + P.rho2 * p3;
    const T tau = P.tau0 * p1 + P.tau1 * p2 + P.tau2 * p3;
    const T grx = P.rho0 * g1x + P.rho1 * g2x + P.rho2 * g3x;
    const T gry = P.rho0 * g1y + P.rho1 * g2y + P.rho2 * g3y;

    // Eq. 9: grad chi = -[sum grad phi_i/(1+chi_i)] / [sum phi_i/(1+chi_i)]^2.
    const T S = P.ic0 * p1 + P.ic1 * p2 + P.ic2 * p3;
    const T iS2 = T(1) / (S * S);
    const T gcx = -(P.ic0 * g1x + P.ic1 * g2x + P.ic2 * g3x) * iS2;
    const T gcy = -(P.ic0 * g1y + P.ic1 * g2y + P.ic2 * g3y) * iS2;

    // Eq. 28 derivatives, phi_k independent; Eq. 25 chemical potentials.
    const T q = P.gam0 * p1 + P.gam1 * p2 + P.gam2 * p3;
    const T p123 = p1 * p2 * p3;
    const T e2 = T(2) * P.eta * p123;
    const T dH1 = T(2) * p1 * (P.s12 * p2 * p2 + P.s13 * p3 * p3) + p2 * p3 * q + p123 * P.gam0 + e2 * p2 * p3;
    const T dH2 = T(2) * p2 * (P.s12 * p1 * p1 + P.s23 * p3 * p3) + p1 * p3 * q + p123 * P.gam1 + e2 * p1 * p3;
    const T dH3 = T(2) * p3 * (P.s13 * p1 * p1 + P.s23 * p2 * p2) + p1 * p2 * q + p123 * P.gam2 + e2 * p1 * p2;
    const T m1 = P.c_bulk * ((dH1 - dH2) * P.igam1 + (dH1 - dH3) * P.igam2) - P.c_lap * P.gam0 * l1;
    const T m2 = P.c_bulk * ((dH2 - dH1) * P.igam0 + (dH2 - dH3) * P.igam2) - P.c_lap * P.gam1 * l2;
    const T m3 = P.c_bulk * ((dH3 - dH1) * P.igam0 + (dH3 - dH2) * P.igam1) - P.c_lap * P.gam2 * l3;
    const T Fsx = m1 * g1x + m2 * g2x + m3 * g3x;  // Eq. 36
    const T Fsy = m1 * g1y + m2 * g2y + m3 * g3y;

    // Field and Kelvin force (Eq. 5, 7).
    T gpx, gpy;
    iso_grad(ps, gpx, gpy);
    o.Hx = P.H0x - gpx;
    o.Hy = P.H0y - gpy;
    const T kel = -P.half_mu0 * (o.Hx * o.Hx + o.Hy * o.Hy);
    const T Fmx = kel * gcx, Fmy = kel * gcy;

    // Zeroth, first and second moments of f.
    const T pstar = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const T jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const T jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const T dd = (f[5] + f[6]) + (f[7] + f[8]);
    const T sxx = (f[1] + f[3]) + dd;
    const T syy = (f[2] + f[4]) + dd;
    const T sxy = (f[5] - f[6]) + (f[7] - f[8]);

    // Pressure force -(p/rho) grad rho = -p* c_s^2 grad rho; drive and gravity.
    const T cp = -pstar * (T(1) / T(3));
    const T F0x = Fsx + Fmx + cp * grx + P.drive + rho * P.grav_x;
    const T F0y = Fsy + Fmy + cp * gry + rho * P.grav_y;
    const T inv_rho = T(1) / rho;
    const T ihr = T(0.5) * inv_rho;
    const T u0x = jx + F0x * ihr, u0y = jy + F0y * ihr;

    // Viscous force from the non-equilibrium stress of f - f^eq(p*, u0); the second
    // moments of f^eq are p* c_s^2 I + u0 u0.  Only p_xx, p_xy relax at s_nu.
    const T A = sxx - pstar * (T(1) / T(3)) - u0x * u0x;
    const T B = syy - pstar * (T(1) / T(3)) - u0y * u0y;
    const T C = sxy - u0x * u0y;
    const T snu = T(1) / (tau + T(0.5));
    const T half_om = T(0.5) * (T(1) - snu) * (A - B);
    const T Pxx = A - half_om, Pyy = B + half_om, Pxy = snu * C;
    const T Fmux = -tau * (Pxx * grx + Pxy * gry);
    const T Fmuy = -tau * (Pxy * grx + Pyy * gry);

    o.Ftx = F0x + Fmux;
    o.Fty = F0y + Fmuy;
    o.ux = jx + o.Ftx * ihr;
    o.uy = jy + o.Fty * ihr;
    o.pstar = pstar;
    o.rho = rho;
    o.tau = tau;
    o.inv_rho = inv_rho;
    o.snu = snu;
    o.phi1 = p1;
    o.phi2 = p2;
    return o;
}

// MRT collision with forcing, in projection form: all non-conserved moments except
// p_xx, p_xy relax to fbar^eq at unit rate, so
//   f* = fbar^eq + (1 - s_nu)/4 [(ex^2 - ey^2) m_xx + ex ey m_xy] + F,
// with m the p_xx, p_xy moments of f - fbar^eq and fbar^eq = f^eq - F/2 (Eq. 15).
template <typename T>
__host__ __device__ __forceinline__ void collide_f(const NodeOut<T>& o, const T f[9], T out[9]) {
    const T ux = o.ux, uy = o.uy;
    const T usq = T(1.5) * (ux * ux + uy * uy);
    const T fr = T(3) * o.inv_rho;
    const T fx = fr * o.Ftx, fy = fr * o.Fty;  // 3 F/rho
    const T w0 = T(4) / T(9), wa = T(1) / T(9), wd = T(1) / T(36);
    T fb[9], F[9];
    // rest
    F[0] = T(0);
    fb[0] = w0 * (o.pstar - usq);
    // axes and diagonals: e.u, e.F
    const T eu[9] = {T(0), ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
    const T ef[9] = {T(0), fx, fy, -fx, -fy, fx + fy, fy - fx, -fx - fy, fx - fy};
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const T w = a < 5 ? wa : wd;
        F[a] = w * ef[a];
        fb[a] = w * (o.pstar + T(3) * eu[a] + T(4.5) * eu[a] * eu[a] - usq) - T(0.5) * F[a];
    }
    const T mxx = ((f[1] + f[3]) - (f[2] + f[4])) - ((fb[1] + fb[3]) - (fb[2] + fb[4]));
    const T mxy = ((f[5] + f[7]) - (f[6] + f[8])) - ((fb[5] + fb[7]) - (fb[6] + fb[8]));
    const T k = T(0.25) * (T(1) - o.snu);
    const T kx = k * mxx, ky = k * mxy;
    out[0] = fb[0];
    out[1] = fb[1] + kx + F[1];
    out[3] = fb[3] + kx + F[3];
    out[2] = fb[2] - kx + F[2];
    out[4] = fb[4] - kx + F[4];
    out[5] = fb[5] + ky + F[5];
    out[7] = fb[7] + ky + F[7];
    out[6] = fb[6] - ky + F[6];
    out[8] = fb[8] - ky + F[8];
}

// Phase-field collision (Eq. 29-31) written as
//   g* = (1 - omega) g + omega phi Gamma(u) + (1 - omega/2) F^phi,
// F^phi_a = w_a e_a . v.
template <typename T>
__host__ __device__ __forceinline__ void collide_g(const NodeOut<T>& o, T om, T phi, T vx, T vy, const T g[9], T out[9]) {
    const T ux = o.ux, uy = o.uy;
    const T usq = T(1.5) * (ux * ux + uy * uy);
    const T w0 = T(4) / T(9), wa = T(1) / T(9), wd = T(1) / T(36);
    const T keep = T(1) - om, op = om * phi, fs = T(1) - T(0.5) * om;
    const T eu[9] = {T(0), ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
    const T ev[9] = {T(0), vx, vy, -vx, -vy, vx + vy, vy - vx, -vx - vy, vx - vy};
    out[0] = keep * g[0] + op * w0 * (T(1) - usq);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const T w = a < 5 ? wa : wd;
        const T gam = w * (T(1) + T(3) * eu[a] + T(4.5) * eu[a] * eu[a] - usq);
        out[a] = keep * g[a] + op * gam + fs * (w * ev[a]);
    }
}

}  // namespace fcd
