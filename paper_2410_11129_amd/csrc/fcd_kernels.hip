// fcd_kernels.hip -- gfx950 kernels of the coupled ferrofluid compound-droplet step.
//
// Layout: every plane is [ny][pitch] (x fastest).  A state buffer is 27 planes
// (f_0..8, g1_0..8, g2_0..8); the stored state is post-streaming.  The phase buffer is
// 3 planes (phi1, phi2, mu_r); psi' is one plane.  One work-item owns one node; a
// wavefront covers 64 consecutive nodes of one row, so every load and store of a
// plane is coalesced and wall rows are wave-uniform branches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fcd_device.hpp"
#include "fcd_kernels.hpp"

namespace fcd {

constexpr int BX = 64;  // one wavefront per row segment
constexpr int BY = 4;

// ---------------------------------------------------------------------------------
// Initial state: f = f^eq(p*, u) (Eq. 16), g^i = phi_i Gamma(u) (Eq. 18).
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void write_equilibrium(T* __restrict__ dist, long long plane, long long k, double p,
                                                  double ux, double uy, double phi1, double phi2) {
    const double usq = 1.5 * (ux * ux + uy * uy);
    const double eu[9] = {0.0, ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double w = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const double gmw = w * (3.0 * eu[a] + 4.5 * eu[a] * eu[a] - usq);  // Gamma - w
        dist[a * plane + k] = T(p * w + gmw);
        dist[(9 + a) * plane + k] = T(phi1 * (w + gmw));
        dist[(18 + a) * plane + k] = T(phi2 * (w + gmw));
    }
}

template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_init_fields(T* __restrict__ dist, const double* __restrict__ phi1, const double* __restrict__ phi2,
                  const double* __restrict__ ux, const double* __restrict__ uy, const double* __restrict__ ps,
                  int nx, int ny, int pitch) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const long long d = (long long)j * nx + i;
    write_equilibrium(dist, (long long)ny * pitch, (long long)j * pitch + i, ps ? ps[d] : 0.0, ux[d], uy[d],
                      phi1[d], phi2[d]);
}

template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_init_droplet(T* __restrict__ dist, int nx, int ny, int pitch, double xc, double yc, double rc, double rs,
                   double xi, double u_scale) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    double dx = (double)i - xc;
    dx -= nx * floor(dx / nx + 0.5);  // minimum image in periodic x
    const double dy = (double)j - yc;
    const double d = sqrt(dx * dx + dy * dy);
    const double pin = 0.5 * (1.0 + tanh(2.0 * (rc - d) / xi));
    const double pout = 0.5 * (1.0 + tanh(2.0 * (rs - d) / xi));
    const double ux = u_scale * (j + 0.5) * (ny - 0.5 - j);  // Poiseuille profile
    write_equilibrium(dist, (long long)ny * pitch, (long long)j * pitch + i, 0.0, ux, 0.0, pin, pout - pin);
}

// ---------------------------------------------------------------------------------
// Order parameters (Eq. 32, 24) and mu_r = 1 / sum phi_i/(1+chi_i) (Eq. 8).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_phase(const T* __restrict__ dist, T* __restrict__ phi, StepConst<T> P) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const long long k = (long long)j * P.pitch + i, pl = P.plane;
    T g1[9], g2[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        g1[a] = dist[(9 + a) * pl + k];
        g2[a] = dist[(18 + a) * pl + k];
    }
    const T p1 = ((g1[0] + g1[1]) + (g1[2] + g1[3])) + ((g1[4] + g1[5]) + (g1[6] + g1[7])) + g1[8];
    const T p2 = ((g2[0] + g2[1]) + (g2[2] + g2[3])) + ((g2[4] + g2[5]) + (g2[6] + g2[7])) + g2[8];
    const T p3 = T(1) - p1 - p2;
    phi[k] = p1;
    phi[pl + k] = p2;
    phi[2 * pl + k] = T(1) / (P.ic0 * p1 + P.ic1 * p2 + P.ic2 * p3);
}

// ---------------------------------------------------------------------------------
// Magnetic potential, Eq. 6, conservative nine-point flux form:
//   sum_a c_a (psi'(x+e_a) - psi'(x)) = H0 sum_a c_a (e_a . h),  c_a = 3 w_a (mu + mu_a).
// One launch relaxes one of the four colours (i mod 2) + 2 (j mod 2); nodes of a colour
// never neighbour each other, so the update is race-free and order-independent.
// ---------------------------------------------------------------------------------
template <typename T>
struct PotNode {
    T C, acc, src;  // sum c, sum c psi'_nb, H0 sum c (e.h)
};

template <typename T>
__device__ __forceinline__ PotNode<T> pot_node(const T* __restrict__ psi, const T* __restrict__ mur, int i, int j,
                                               const StepConst<T>& P) {
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    const Nb9<T> m = load_nb(mur, x);
    const Nb9<T> u = load_nb_psi(psi, x, j, P.ny);
    const T a = T(1) / T(3), d = T(1) / T(12);
    const T ce = a * (m.c + m.e), cw = a * (m.c + m.w), cn = a * (m.c + m.n), cs = a * (m.c + m.s);
    const T cne = d * (m.c + m.ne), cnw = d * (m.c + m.nw), csw = d * (m.c + m.sw), cse = d * (m.c + m.se);
    PotNode<T> r;
    r.C = ((ce + cw) + (cn + cs)) + ((cne + csw) + (cnw + cse));
    r.acc = ((ce * u.e + cw * u.w) + (cn * u.n + cs * u.s)) + ((cne * u.ne + csw * u.sw) + (cnw * u.nw + cse * u.se));
    const T sx = (ce - cw) + (cne - csw) + (cse - cnw);
    const T sy = (cn - cs) + (cne - csw) + (cnw - cse);
    r.src = P.H0x * sx + P.H0y * sy;
    return r;
}

template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_sor_colour(T* __restrict__ psi, const T* __restrict__ mur, StepConst<T> P, int colour, T omega) {
    const int i = 2 * (blockIdx.x * BX + threadIdx.x) + (colour & 1);
    const int j = 2 * (blockIdx.y * BY + threadIdx.y) + (colour >> 1);
    if (i >= P.nx || j >= P.ny) return;
    const PotNode<T> r = pot_node(psi, mur, i, j, P);
    const long long k = (long long)j * P.pitch + i;
    const T old = psi[k];
    psi[k] = old + omega * ((r.acc - r.src) / r.C - old);
}

// Max-norm of the residual L(psi0 + psi').  Grid-stride over nodes with a capped grid;
// wave64 shuffle max, then the block's four wave maxima through LDS, then one
// atomicMax per block on the bit pattern (monotone for non-negative doubles; a NaN
// propagates as the largest pattern).
constexpr int RES_T = 256;
constexpr int RES_MAX_BLOCKS = 1024;

__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

template <typename T>
__global__ void __launch_bounds__(RES_T)
    k_residual(const T* __restrict__ psi, const T* __restrict__ mur, StepConst<T> P,
               unsigned long long* __restrict__ out) {
    __shared__ double wmax[RES_T / 64];
    double v = 0.0;
    const long long n = (long long)P.nx * P.ny;
    for (long long t = (long long)blockIdx.x * RES_T + threadIdx.x; t < n; t += (long long)gridDim.x * RES_T) {
        const int j = (int)(t / P.nx), i = (int)(t - (long long)j * P.nx);
        const PotNode<T> r = pot_node(psi, mur, i, j, P);
        const T c = psi[(long long)j * P.pitch + i];
        v = nan_max(v, fabs((double)(r.acc - r.C * c - r.src)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
        for (int w = 1; w < RES_T / 64; ++w) m = nan_max(m, wmax[w]);
        atomicMax(out, (unsigned long long)__double_as_longlong(m));
    }
}

// ---------------------------------------------------------------------------------
// Fused step: stencils + forces + MRT collision of f + phase-field collision of g1, g2,
// then push streaming with halfway bounce-back at the walls.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_collide_stream(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ phi,
                     const T* __restrict__ psi, StepConst<T> P) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const long long pl = P.plane;
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    const long long k = x.c;
    T f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = src[a * pl + k];
    const Nb9<T> a1 = load_nb(phi, x);
    const Nb9<T> a2 = load_nb(phi + pl, x);
    const Nb9<T> ps = load_nb_psi(psi, x, j, P.ny);
    const NodeOut<T> o = node_physics(P, f, a1, a2, ps);

    // Destinations of the push: (i + ex, j + ey); a population that would cross a wall
    // returns to its own node in the opposite direction (halfway bounce-back).
    const bool bot = j == 0, top = j == P.ny - 1;
    const long long dE = x.e, dW = x.w, dN = x.n, dS = x.s, dNE = x.ne, dNW = x.nw, dSW = x.sw, dSE = x.se;
    // plane and node of each direction's destination
    const int pN = top ? 4 : 2, pNE = top ? 7 : 5, pNW = top ? 8 : 6;
    const int pS = bot ? 2 : 4, pSW = bot ? 5 : 7, pSE = bot ? 6 : 8;
    const long long nN = top ? k : dN, nNE = top ? k : dNE, nNW = top ? k : dNW;
    const long long nS = bot ? k : dS, nSW = bot ? k : dSW, nSE = bot ? k : dSE;

    {
        T out[9];
        collide_f(o, f, out);
        T* D = dst;
        D[k] = out[0];
        D[1 * pl + dE] = out[1];
        D[3 * pl + dW] = out[3];
        D[pN * pl + nN] = out[2];
        D[pS * pl + nS] = out[4];
        D[pNE * pl + nNE] = out[5];
        D[pNW * pl + nNW] = out[6];
        D[pSW * pl + nSW] = out[7];
        D[pSE * pl + nSE] = out[8];
    }
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        T g[9], out[9];
        const T* S = src + (9 + 9 * comp) * pl;
#pragma unroll
        for (int a = 0; a < 9; ++a) g[a] = S[a * pl + k];
        collide_g(o, P.omega_phi, comp == 0 ? o.phi1 : o.phi2, comp == 0 ? o.v1x : o.v2x,
                  comp == 0 ? o.v1y : o.v2y, g, out);
        T* D = dst + (9 + 9 * comp) * pl;
        D[k] = out[0];
        D[1 * pl + dE] = out[1];
        D[3 * pl + dW] = out[3];
        D[pN * pl + nN] = out[2];
        D[pS * pl + nS] = out[4];
        D[pNE * pl + nNE] = out[5];
        D[pNW * pl + nNW] = out[6];
        D[pSW * pl + nSW] = out[7];
        D[pSE * pl + nSE] = out[8];
    }
}

// ---------------------------------------------------------------------------------
// Moments of the current state (FP64 dense planes selected by a bit mask).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_moments(const T* __restrict__ src, const T* __restrict__ phi, const T* __restrict__ psi, StepConst<T> P,
              unsigned mask, double* __restrict__ out) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const long long pl = P.plane;
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    T f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = src[a * pl + x.c];
    const NodeOut<T> o = node_physics(P, f, load_nb(phi, x), load_nb(phi + pl, x), load_nb_psi(psi, x, j, P.ny));
    const double vals[10] = {(double)o.pstar, (double)o.ux, (double)o.uy, (double)o.phi1, (double)o.phi2,
                             (double)(T(1) - o.phi1 - o.phi2), (double)o.rho, (double)psi[x.c], (double)o.Hx,
                             (double)o.Hy};
    const long long dn = (long long)P.nx * P.ny, d = (long long)j * P.nx + i;
    int slot = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q)
        if (mask & (1u << q)) out[slot++ * dn + d] = vals[q];
}

// ---------------------------------------------------------------------------------
// State and psi' copies between the pitched planes and dense FP64 arrays.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_planes_to_dense(const T* __restrict__ src, double* __restrict__ out, int nplanes, int nx, int ny, int pitch) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    for (int q = 0; q < nplanes; ++q)
        out[((long long)q * ny + j) * nx + i] = (double)src[((long long)q * ny + j) * pitch + i];
}

template <typename T>
__global__ void __launch_bounds__(BX* BY)
    k_dense_to_planes(const double* __restrict__ in, T* __restrict__ dst, int nplanes, int nx, int ny, int pitch) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    for (int q = 0; q < nplanes; ++q)
        dst[((long long)q * ny + j) * pitch + i] = T(in[((long long)q * ny + j) * nx + i]);
}

template <typename T>
__global__ void k_fill(T* __restrict__ a, long long n, T v) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// ---------------------------------------------------------------------------------
// Deformation diagnostics, deterministic two-level reductions (one block per row,
// then one block over rows in a fixed order).
//   pass 0 per row: for w_o = phi1 + phi2 and w_i = phi1: sum w, sum w cos, sum w sin,
//                   sum w y  (8 values)
//   pass 1 per row: sum w dx^2, sum w dy^2 about the centroids (4 values)
// ---------------------------------------------------------------------------------
constexpr int DIAG_T = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = DIAG_T / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <typename T>
__global__ void __launch_bounds__(DIAG_T)
    k_diag_rows(const T* __restrict__ phi, StepConst<T> P, int pass, const double* __restrict__ cent,
                double* __restrict__ rows) {
    __shared__ double sh[DIAG_T];
    const int j = blockIdx.x;
    const double twopi = 6.283185307179586476925286766559;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < P.nx; i += DIAG_T) {
        const long long k = (long long)j * P.pitch + i;
        const double wi = (double)phi[k];
        const double wo = wi + (double)phi[P.plane + k];
        if (pass == 0) {
            double sn, cs;
            sincos(twopi * i / P.nx, &sn, &cs);
            acc[0] += wo;
            acc[1] += wo * cs;
            acc[2] += wo * sn;
            acc[3] += wo * j;
            acc[4] += wi;
            acc[5] += wi * cs;
            acc[6] += wi * sn;
            acc[7] += wi * j;
        } else {
            double dxo = (double)i - cent[0], dxi = (double)i - cent[2];
            dxo -= P.nx * floor(dxo / P.nx + 0.5);
            dxi -= P.nx * floor(dxi / P.nx + 0.5);
            const double dyo = (double)j - cent[1], dyi = (double)j - cent[3];
            acc[0] += wo * dxo * dxo;
            acc[1] += wo * dyo * dyo;
            acc[2] += wi * dxi * dxi;
            acc[3] += wi * dyi * dyi;
        }
    }
    const int nv = pass == 0 ? 8 : 4;
    for (int q = 0; q < nv; ++q) {
        const double s = block_sum(acc[q], sh);
        if (threadIdx.x == 0) rows[(long long)j * 8 + q] = s;
    }
}

// Sums the per-row values in row order; pass 0 writes the centroids, pass 1 the result
// {D_o, D_i, mass1, mass2} (masses kept from pass 0 in cent[4], cent[5]).
__global__ void k_diag_final(const double* __restrict__ rows, int ny, int nx, int pass, double* __restrict__ cent,
                             double* __restrict__ result) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int nv = pass == 0 ? 8 : 4;
    for (int j = 0; j < ny; ++j)
        for (int q = 0; q < nv; ++q) s[q] += rows[(long long)j * 8 + q];
    const double twopi = 6.283185307179586476925286766559;
    if (pass == 0) {
        cent[0] = nx * atan2(s[2], s[1]) / twopi;
        cent[1] = s[3] / s[0];
        cent[2] = nx * atan2(s[6], s[5]) / twopi;
        cent[3] = s[7] / s[4];
        cent[4] = s[4];           // mass of phase 1
        cent[5] = s[0] - s[4];    // mass of phase 2
        cent[6] = s[0];
        cent[7] = s[4];
    } else {
        const double ixo = s[0] / cent[6], iyo = s[1] / cent[6];
        const double ixi = s[2] / cent[7], iyi = s[3] / cent[7];
        result[0] = (sqrt(iyo) - sqrt(ixo)) / (sqrt(iyo) + sqrt(ixo));
        result[1] = (sqrt(iyi) - sqrt(ixi)) / (sqrt(iyi) + sqrt(ixi));
        result[2] = cent[4];
        result[3] = cent[5];
    }
}

// ---------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------
static inline dim3 grid2(int nx, int ny) { return dim3((nx + BX - 1) / BX, (ny + BY - 1) / BY); }

template <typename T>
void launch_init_fields(T* dist, const double* phi1, const double* phi2, const double* ux, const double* uy,
                        const double* ps, int nx, int ny, int pitch, hipStream_t s) {
    hipLaunchKernelGGL(k_init_fields<T>, grid2(nx, ny), dim3(BX, BY), 0, s, dist, phi1, phi2, ux, uy, ps, nx, ny,
                       pitch);
}

template <typename T>
void launch_init_droplet(T* dist, int nx, int ny, int pitch, double xc, double yc, double rc, double rs, double xi,
                         double u_scale, hipStream_t s) {
    hipLaunchKernelGGL(k_init_droplet<T>, grid2(nx, ny), dim3(BX, BY), 0, s, dist, nx, ny, pitch, xc, yc, rc, rs,
                       xi, u_scale);
}

template <typename T>
void launch_phase(const T* dist, T* phi, const StepConst<T>& P, hipStream_t s) {
    hipLaunchKernelGGL(k_phase<T>, grid2(P.nx, P.ny), dim3(BX, BY), 0, s, dist, phi, P);
}

template <typename T>
void launch_sor_sweep(T* psi, const T* mur, const StepConst<T>& P, T omega, hipStream_t s) {
    const dim3 g = grid2((P.nx + 1) / 2, (P.ny + 1) / 2);
    for (int c = 0; c < 4; ++c) hipLaunchKernelGGL(k_sor_colour<T>, g, dim3(BX, BY), 0, s, psi, mur, P, c, omega);
}

template <typename T>
void launch_residual(const T* psi, const T* mur, const StepConst<T>& P, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, out, 1LL, 0ULL);
    const long long n = (long long)P.nx * P.ny;
    long long blocks = (n + RES_T - 1) / RES_T;
    if (blocks > RES_MAX_BLOCKS) blocks = RES_MAX_BLOCKS;
    hipLaunchKernelGGL(k_residual<T>, dim3((unsigned)blocks), dim3(RES_T), 0, s, psi, mur, P, out);
}

template <typename T>
void launch_collide_stream(const T* src, T* dst, const T* phi, const T* psi, const StepConst<T>& P, hipStream_t s) {
    hipLaunchKernelGGL(k_collide_stream<T>, grid2(P.nx, P.ny), dim3(BX, BY), 0, s, src, dst, phi, psi, P);
}

template <typename T>
void launch_moments(const T* src, const T* phi, const T* psi, const StepConst<T>& P, unsigned mask, double* out,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_moments<T>, grid2(P.nx, P.ny), dim3(BX, BY), 0, s, src, phi, psi, P, mask, out);
}

template <typename T>
void launch_to_dense(const T* src, double* out, int nplanes, int nx, int ny, int pitch, hipStream_t s) {
    hipLaunchKernelGGL(k_planes_to_dense<T>, grid2(nx, ny), dim3(BX, BY), 0, s, src, out, nplanes, nx, ny, pitch);
}

template <typename T>
void launch_from_dense(const double* in, T* dst, int nplanes, int nx, int ny, int pitch, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_to_planes<T>, grid2(nx, ny), dim3(BX, BY), 0, s, in, dst, nplanes, nx, ny, pitch);
}

template <typename T>
void launch_fill(T* a, long long n, T v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n, v);
}

template <typename T>
void launch_diagnostics(const T* phi, const StepConst<T>& P, double* rows, double* cent, double* result,
                        hipStream_t s) {
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_diag_rows<T>, dim3(P.ny), dim3(DIAG_T), 0, s, phi, P, pass, cent, rows);
        hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, rows, P.ny, P.nx, pass, cent, result);
    }
}

#define FCD_INSTANTIATE(T)                                                                                        \
    template void launch_init_fields<T>(T*, const double*, const double*, const double*, const double*,         \
                                        const double*, int, int, int, hipStream_t);                              \
    template void launch_init_droplet<T>(T*, int, int, int, double, double, double, double, double, double,     \
                                         hipStream_t);                                                           \
    template void launch_phase<T>(const T*, T*, const StepConst<T>&, hipStream_t);                               \
    template void launch_sor_sweep<T>(T*, const T*, const StepConst<T>&, T, hipStream_t);                        \
    template void launch_residual<T>(const T*, const T*, const StepConst<T>&, unsigned long long*, hipStream_t); \
    template void launch_collide_stream<T>(const T*, T*, const T*, const T*, const StepConst<T>&, hipStream_t);  \
    template void launch_moments<T>(const T*, const T*, const T*, const StepConst<T>&, unsigned, double*,        \
                                    hipStream_t);                                                                \
    template void launch_to_dense<T>(const T*, double*, int, int, int, int, hipStream_t);                        \
    template void launch_from_dense<T>(const double*, T*, int, int, int, int, hipStream_t);                      \
    template void launch_fill<T>(T*, long long, T, hipStream_t);                                                 \
    template void launch_diagnostics<T>(const T*, const StepConst<T>&, double*, double*, double*, hipStream_t);

FCD_INSTANTIATE(double)
FCD_INSTANTIATE(float)

}  // namespace fcd
