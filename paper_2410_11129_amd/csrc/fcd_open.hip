// fcd_open.hip -- open-channel boundaries of the single-channel step: the Eq. 37 velocity
// inlet at x = 0 and the convective outflow condition at x = nx - 1 (Sec. 2.5).
//
// The fused collide-and-stream kernel treats x as periodic.  Every (destination node,
// direction) slot of the post-streaming state is written by exactly one source node, so
// the open channel is obtained after that kernel by two small launches on the same stream:
//  1. the two end columns are collided again with their phi stencils closed by zero normal
//     gradient (the column beyond an end takes the end column's value) and pushed again;
//     this overwrites exactly the slots they wrote before.  psi' keeps its periodic closure.
//  2. the populations streaming cannot supply are set: directions 1, 5, 8 at the inlet
//     (Zou-He velocity condition for f, carrier-only equilibrium inflow for g1, g2) and
//     3, 6, 7 at the outlet (convective condition for f, g1, g2).
// The wrapped values that step 1 and the fused kernel push across the ends land only in
// those unknown slots and are replaced by step 2.  Both launches touch 2 ny nodes.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fcd_device.hpp"
#include "fcd_kernels.hpp"
#include "fcd_step.hpp"

namespace fcd {

constexpr int OPEN_T = 64;

// Neighbour offsets at (i, j) with the columns beyond the inlet and outlet replaced by the
// end column (zero normal gradient), rows clamped as in the interior.
__device__ __forceinline__ NbIdx nb_index_open(int i, int j, int nx, int ny, int pitch) {
    NbIdx x = nb_index(i, j, nx, ny, pitch);
    if (i == 0) {
        x.w = x.c;
        x.nw = x.n;
        x.sw = x.s;
    }
    if (i == nx - 1) {
        x.e = x.c;
        x.ne = x.n;
        x.se = x.s;
    }
    return x;
}

// Thread q < 2 ny: column 0 for q < ny, column nx - 1 otherwise.
__device__ __forceinline__ bool edge_node(int q, int nx, int ny, int& i, int& j) {
    if (q >= 2 * ny) return false;
    j = q < ny ? q : q - ny;
    i = q < ny ? 0 : nx - 1;
    return true;
}

template <typename T>
__global__ void __launch_bounds__(OPEN_T)
    k_open_edge_collide(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ phi,
                        const T* __restrict__ psi, StepConst<T> P, ResGate gate) {
    if (gate.res && !gate.passed()) return;
    int i, j;
    if (!edge_node(blockIdx.x * OPEN_T + threadIdx.x, P.nx, P.ny, i, j)) return;
    const NbIdx c = nb_index_open(i, j, P.nx, P.ny, P.pitch);
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    // the end columns were collided (and checked for divergence) by the main kernel
    collide_stream_nb(src, dst, load_nb(phi, c), load_nb(phi + P.plane, c), load_nb_psi(psi, x, j, P.ny), P, i, j,
                      nullptr);
}

// One thread per row.  Inlet: the first moment of f is set to (u_in(y), 0) and the
// non-equilibrium part of f_1 to that of f_3 (f_eq,1 - f_eq,3 = (2/3) u_x from Eq. 16, 18);
// the two first-moment equations then give f_5 and f_8; the inflow is carrier only, so
// the entering g populations phi_in Gamma_a(u_in) are zero.  Outlet: f(t+1, N) =
// [f(t, N) + U f(t+1, N-1)] / (1 + U) for f, g1, g2, with f(t, N) read from the state
// the step started from.
template <typename T>
__global__ void __launch_bounds__(OPEN_T)
    k_open_bc(const T* __restrict__ src, T* __restrict__ dst, StepConst<T> P, double u_in, double U,
              ResGate gate) {
    if (gate.res && !gate.passed()) return;
    const int j = blockIdx.x * OPEN_T + threadIdx.x;
    if (j >= P.ny) return;
    const long long pl = P.plane, k0 = (long long)j * P.pitch, kN = k0 + P.nx - 1, kB = kN - 1;
    const double s = (j + 0.5) / P.ny;
    const T ux = T(4.0 * u_in * s * (1.0 - s));  // Eq. 37 at y = j + 1/2, H = ny
    const T f2 = dst[2 * pl + k0], f3 = dst[3 * pl + k0], f4 = dst[4 * pl + k0];
    const T f6 = dst[6 * pl + k0], f7 = dst[7 * pl + k0];
    dst[1 * pl + k0] = f3 + T(2.0 / 3.0) * ux;
    dst[5 * pl + k0] = f7 - T(0.5) * (f2 - f4) + ux / T(6);
    dst[8 * pl + k0] = f6 + T(0.5) * (f2 - f4) + ux / T(6);
#pragma unroll
    for (int comp = 1; comp <= 2; ++comp) {
        dst[(9 * comp + 1) * pl + k0] = T(0);
        dst[(9 * comp + 5) * pl + k0] = T(0);
        dst[(9 * comp + 8) * pl + k0] = T(0);
    }
    const T Ut = T(U), inv = T(1) / (T(1) + Ut);
    const int out_dirs[3] = {3, 6, 7};
#pragma unroll
    for (int comp = 0; comp < 3; ++comp)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const long long p = (long long)(9 * comp + out_dirs[d]) * pl;
            dst[p + kN] = (src[p + kN] + Ut * dst[p + kB]) * inv;
        }
}

// Moments of the end columns with the open-channel stencils (overwrites what the periodic
// moments kernel wrote there); same planes and mask order.
template <typename T>
__global__ void __launch_bounds__(OPEN_T)
    k_open_edge_moments(const T* __restrict__ src, const T* __restrict__ phi, const T* __restrict__ psi,
                        StepConst<T> P, unsigned mask, double* __restrict__ out) {
    int i, j;
    if (!edge_node(blockIdx.x * OPEN_T + threadIdx.x, P.nx, P.ny, i, j)) return;
    const long long pl = P.plane;
    const NbIdx c = nb_index_open(i, j, P.nx, P.ny, P.pitch);
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    T f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = src[a * pl + x.c];
    const NodeOut<T> o = node_physics(P, f, load_nb(phi, c), load_nb(phi + pl, c), load_nb_psi(psi, x, j, P.ny));
    const double vals[10] = {(double)o.pstar, (double)o.ux, (double)o.uy, (double)o.phi1, (double)o.phi2,
                             (double)(T(1) - o.phi1 - o.phi2), (double)o.rho, (double)psi[x.c], (double)o.Hx,
                             (double)o.Hy};
    const long long dn = (long long)P.nx * P.ny, d = (long long)j * P.nx + i;
    int slot = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q)
        if (mask & (1u << q)) out[slot++ * dn + d] = vals[q];
}

// Initial state of the open channel: concentric tanh profiles about (xc, yc) by plain
// distance (no periodic image) and the Eq. 37 profile in every column; p* = 0;
// f = f^eq (Eq. 16), g^i = phi_i Gamma(u) (Eq. 18).
template <typename T>
__global__ void __launch_bounds__(OPEN_T)
    k_open_init_droplet(T* __restrict__ dist, int nx, int ny, int pitch, double xc, double yc, double rc, double rs,
                        double xi, double u_in) {
    const long long q = (long long)blockIdx.x * OPEN_T + threadIdx.x;
    if (q >= (long long)nx * ny) return;
    const int j = (int)(q / nx), i = (int)(q - (long long)j * nx);
    const double dx = (double)i - xc, dy = (double)j - yc;
    const double d = sqrt(dx * dx + dy * dy);
    const double pin = 0.5 * (1.0 + tanh(2.0 * (rc - d) / xi));
    const double pout = 0.5 * (1.0 + tanh(2.0 * (rs - d) / xi));
    const double s = (j + 0.5) / ny;
    const double ux = 4.0 * u_in * s * (1.0 - s);
    const double usq = 1.5 * ux * ux;
    const double eu[9] = {0.0, ux, 0.0, -ux, 0.0, ux, -ux, -ux, ux};
    const long long plane = (long long)ny * pitch, k = (long long)j * pitch + i;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const double w = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const double gmw = w * (3.0 * eu[a] + 4.5 * eu[a] * eu[a] - usq);  // Gamma - w
        dist[a * plane + k] = T(gmw);
        dist[(9 + a) * plane + k] = T(pin * (w + gmw));
        dist[(18 + a) * plane + k] = T((pout - pin) * (w + gmw));
    }
}

static inline unsigned open_grid(long long n) { return (unsigned)((n + OPEN_T - 1) / OPEN_T); }

template <typename T>
void launch_open_boundaries(const T* src, T* dst, const T* phi, const T* psi, const StepConst<T>& P, double u_in,
                            double U, hipStream_t s, const ResGate& gate) {
    hipLaunchKernelGGL(k_open_edge_collide<T>, dim3(open_grid(2LL * P.ny)), dim3(OPEN_T), 0, s, src, dst, phi, psi,
                       P, gate);
    hipLaunchKernelGGL(k_open_bc<T>, dim3(open_grid(P.ny)), dim3(OPEN_T), 0, s, src, dst, P, u_in, U, gate);
}

template <typename T>
void launch_open_edge_moments(const T* src, const T* phi, const T* psi, const StepConst<T>& P, unsigned mask,
                              double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_open_edge_moments<T>, dim3(open_grid(2LL * P.ny)), dim3(OPEN_T), 0, s, src, phi, psi, P,
                       mask, out);
}

template <typename T>
void launch_open_init_droplet(T* dist, int nx, int ny, int pitch, double xc, double yc, double rc, double rs,
                              double xi, double u_in, hipStream_t s) {
    hipLaunchKernelGGL(k_open_init_droplet<T>, dim3(open_grid((long long)nx * ny)), dim3(OPEN_T), 0, s, dist, nx, ny,
                       pitch, xc, yc, rc, rs, xi, u_in);
}

#define FCD_OPEN_INST(T)                                                                                          \
    template void launch_open_boundaries<T>(const T*, T*, const T*, const T*, const StepConst<T>&, double, double, \
                                            hipStream_t, const ResGate&);                                         \
    template void launch_open_edge_moments<T>(const T*, const T*, const T*, const StepConst<T>&, unsigned,         \
                                              double*, hipStream_t);                                              \
    template void launch_open_init_droplet<T>(T*, int, int, int, double, double, double, double, double, double,   \
                                              hipStream_t);
FCD_OPEN_INST(double)
FCD_OPEN_INST(float)

}  // namespace fcd
