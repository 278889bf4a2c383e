// fcd_kernels.hip -- gfx950 kernels of the coupled ferrofluid compound-droplet step.
//
// Layout: every plane is [ny][pitch] (x fastest).  A state buffer is 27 planes
// (f_0..8, g1_0..8, g2_0..8); the stored state is post-streaming.  The phase buffer is
// 3 planes (phi1, phi2, mu_r); psi' is one plane.  One work-item owns one node; a
// wavefront covers 64 consecutive nodes of one row, so every load and store of a
// plane is coalesced and wall rows are wave-uniform branches.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fcd_device.hpp"
#include "fcd_kernels.hpp"
#include "fcd_step.hpp"

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
    phase_node(dist, phi, P, i, j);
}

// ---------------------------------------------------------------------------------
// Fused step: stencils + forces + MRT collision of f + phase-field collision of g1, g2,
// then push streaming with halfway bounce-back.  The phi1, phi2 and psi' neighbourhoods
// are staged through LDS: a block loads its (64 + 2) x (CY + 2) tile of the three planes
// once (coalesced rows; columns wrap, rows beyond the walls mirrored for phi and zero
// for psi'), then every node reads its nine-point neighbourhoods from LDS.
// ---------------------------------------------------------------------------------
constexpr int CY = 4;

template <typename T>
__device__ __forceinline__ Nb9<T> lds_nb(const T (*t)[BX + 2], int lx, int ly) {
    Nb9<T> v;
    v.c = t[ly][lx];
    v.e = t[ly][lx + 1];
    v.w = t[ly][lx - 1];
    v.n = t[ly + 1][lx];
    v.s = t[ly - 1][lx];
    v.ne = t[ly + 1][lx + 1];
    v.nw = t[ly + 1][lx - 1];
    v.sw = t[ly - 1][lx - 1];
    v.se = t[ly - 1][lx + 1];
    return v;
}

template <typename T>
__global__ void __launch_bounds__(BX* CY)
    k_collide_stream(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ phi,
                         const T* __restrict__ psi, StepConst<T> P, unsigned long long* __restrict__ div,
                         StepGate sg) {
    if (sg.gate.res) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) publish_tests(sg);
        if (!sg.gate.passed()) return;
    }
    __shared__ T t1[CY + 2][BX + 2], t2[CY + 2][BX + 2], tp[CY + 2][BX + 2];
    const int i0 = blockIdx.x * BX, j0 = blockIdx.y * CY;
    const int tid = threadIdx.y * BX + threadIdx.x;
    for (int q = tid; q < (BX + 2) * (CY + 2); q += BX * CY) {
        const int ly = q / (BX + 2), lx = q - ly * (BX + 2);
        int i = i0 + lx - 1;
        while (i < 0) i += P.nx;
        while (i >= P.nx) i -= P.nx;
        const int jr = j0 + ly - 1;
        const int j = jr < 0 ? 0 : (jr >= P.ny ? P.ny - 1 : jr);
        const long long k = (long long)j * P.pitch + i;
        t1[ly][lx] = phi[k];
        t2[ly][lx] = phi[P.plane + k];
        tp[ly][lx] = (jr < 0 || jr >= P.ny) ? T(0) : psi[k];
    }
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const int lx = threadIdx.x + 1, ly = threadIdx.y + 1;
    collide_stream_nb(src, dst, lds_nb<T>(t1, lx, ly), lds_nb<T>(t2, lx, ly), lds_nb<T>(tp, lx, ly), P, i, j, div);
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
            acc[4] += wo * dxo;
            acc[5] += wi * dxi;
        }
    }
    const int nv = pass == 0 ? 8 : 6;
    for (int q = 0; q < nv; ++q) {
        const double s = block_sum(acc[q], sh);
        if (threadIdx.x == 0) rows[(long long)j * 8 + q] = s;
    }
}

// Sums the per-row values in row order; pass 0 writes the centroids, pass 1 the result
// {D_o, D_i, mass1, mass2} (masses kept from pass 0 in cent[4], cent[5]).  cent[8..23]
// receive, for the shell weight (8..15) and the core weight (16..23): S, C, Sn, y_c, x_c,
// I_xx, I_yy, sum w dx -- what the adjoint of D needs.
__global__ void k_diag_final(const double* __restrict__ rows, int ny, int nx, int pass, double* __restrict__ cent,
                             double* __restrict__ result) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int nv = pass == 0 ? 8 : 6;
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
        double* dg = cent + 8;
        dg[0] = s[0];
        dg[1] = s[1];
        dg[2] = s[2];
        dg[3] = cent[1];
        dg[4] = cent[0];
        dg[8] = s[4];
        dg[9] = s[5];
        dg[10] = s[6];
        dg[11] = cent[3];
        dg[12] = cent[2];
    } else {
        const double ixo = s[0] / cent[6], iyo = s[1] / cent[6];
        const double ixi = s[2] / cent[7], iyi = s[3] / cent[7];
        double* dg = cent + 8;
        dg[5] = ixo;
        dg[6] = iyo;
        dg[7] = s[4];
        dg[13] = ixi;
        dg[14] = iyi;
        dg[15] = s[5];
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
void launch_phase(const T* dist, T* phi, const StepConst<T>& P, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    // with events, the launch itself records the kernel's start and end (no host gap inside)
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(k_phase<T>, grid2(P.nx, P.ny), dim3(BX, BY), 0, s, ev0, ev1, 0, dist, phi, P);
    else
        hipLaunchKernelGGL(k_phase<T>, grid2(P.nx, P.ny), dim3(BX, BY), 0, s, dist, phi, P);
}

template <typename T>
void launch_collide_stream(const T* src, T* dst, const T* phi, const T* psi, const StepConst<T>& P,
                           unsigned long long* div, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, const StepGate& sg) {
    const dim3 g((P.nx + BX - 1) / BX, (P.ny + CY - 1) / CY);
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(k_collide_stream<T>, g, dim3(BX, CY), 0, s, ev0, ev1, 0, src, dst, phi, psi, P, div,
                              sg);
    else
        hipLaunchKernelGGL(k_collide_stream<T>, g, dim3(BX, CY), 0, s, src, dst, phi, psi, P, div, sg);
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
    template void launch_phase<T>(const T*, T*, const StepConst<T>&, hipStream_t, hipEvent_t, hipEvent_t);       \
    template void launch_collide_stream<T>(const T*, T*, const T*, const T*, const StepConst<T>&,                \
                                           unsigned long long*, hipStream_t, hipEvent_t, hipEvent_t,              \
                                           const StepGate&);                                                      \
    template void launch_moments<T>(const T*, const T*, const T*, const StepConst<T>&, unsigned, double*,        \
                                    hipStream_t);                                                                \
    template void launch_to_dense<T>(const T*, double*, int, int, int, int, hipStream_t);                        \
    template void launch_from_dense<T>(const double*, T*, int, int, int, int, hipStream_t);                      \
    template void launch_fill<T>(T*, long long, T, hipStream_t);                                                 \
    template void launch_diagnostics<T>(const T*, const StepConst<T>&, double*, double*, double*, hipStream_t);

FCD_INSTANTIATE(double)
FCD_INSTANTIATE(float)
template void launch_fill<int>(int*, long long, int, hipStream_t);

}  // namespace fcd
