// fcd_potential.hip -- magnetic potential solve (Eq. 6) on gfx950: four-colour SOR and
// geometric multigrid V-cycles, plus the residual max-norm that decides convergence.
//
// Discrete operator (conservative nine-point flux form, lattice units, grid spacing h):
//   (L u)(x) = sum_a c_a (u(x+e_a) - u(x)),  c_a = 3 w_a (mu(x) + mu(x+e_a)) / h^2.
// On the finest level u = psi', the right-hand side is H0 sum_a c_a (e_a . h) (so that
// L(psi0 + psi') = 0 with psi0 = -H0 (x cos a + y sin a)) and psi' = 0 on the rows beyond
// the walls.  Coarse levels are cell-centred: coarse node (I, J) is the average of fine
// nodes (2I..2I+1, 2J..2J+1) and sits (h-1)/2 fine cells inside the wall line, so its
// ghost row must carry -kappa times the edge row, kappa = (h-1)/(h+1), for the
// correction to vanish on the true wall line (linear extrapolation); kappa = 0 on the
// finest level.  mu_r is mirrored beyond the walls on every level.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fcd_device.hpp"
#include "fcd_kernels.hpp"
#include "fcd_potential.hpp"

namespace fcd {

constexpr int PX = 64;  // one wavefront per row segment
constexpr int PY = 4;

template <typename T>
__global__ void __launch_bounds__(PX* PY) k_pot_relax_colour(PotLevel<T> L, int colour, T omega) {
    const int i = 2 * (blockIdx.x * PX + threadIdx.x) + (colour & 1);
    const int j = 2 * (blockIdx.y * PY + threadIdx.y) + (colour >> 1);
    if (i >= L.nx || j >= L.ny) return;
    relax_node(L, i, j, omega);
}

// Max-norms of the residual of a level (out[0]) and of the diagonal term C u (out[1],
// the scale that bounds the residual's rounding floor).  Grid-stride with a capped grid,
// wave64 shuffle max, block max through LDS, one atomicMax per block and quantity on
// the bit pattern (monotone for non-negative doubles; a NaN propagates as the largest
// pattern).
constexpr int RES_T = 256;
constexpr int RES_MAX_BLOCKS = 1024;


template <typename T>
__global__ void __launch_bounds__(RES_T) k_pot_residual(PotLevel<T> L, unsigned long long* __restrict__ out) {
    __shared__ double wmax[2][RES_T / 64];
    double v = 0.0, sc = 0.0;
    const long long n = (long long)L.nx * L.ny;
    for (long long t = (long long)blockIdx.x * RES_T + threadIdx.x; t < n; t += (long long)gridDim.x * RES_T) {
        const int j = (int)(t / L.nx), i = (int)(t - (long long)j * L.nx);
        const MgEval<T> r = mg_eval(L, i, j);
        const T c = L.u[(long long)j * L.pitch + i];
        v = nan_max(v, fabs((double)(r.acc - r.C * c - r.rhs)));
        sc = nan_max(sc, fabs((double)(r.C * c)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v = nan_max(v, __shfl_xor(v, off, 64));
        sc = nan_max(sc, __shfl_xor(sc, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wmax[0][threadIdx.x >> 6] = v;
        wmax[1][threadIdx.x >> 6] = sc;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double m = wmax[threadIdx.x][0];
        for (int w = 1; w < RES_T / 64; ++w) m = nan_max(m, wmax[threadIdx.x][w]);
        atomicMax(out + threadIdx.x, (unsigned long long)__double_as_longlong(m));
    }
}

// Coarse mu: average of the four fine nodes.
template <typename T>
__global__ void __launch_bounds__(PX* PY) k_mg_restrict_mu(const T* __restrict__ muf, int pitchf,
                                                           T* __restrict__ muc, int nxc, int nyc, int pitchc) {
    const int I = blockIdx.x * PX + threadIdx.x, J = blockIdx.y * PY + threadIdx.y;
    if (I >= nxc || J >= nyc) return;
    const long long r0 = (long long)(2 * J) * pitchf + 2 * I, r1 = r0 + pitchf;
    muc[(long long)J * pitchc + I] = T(0.25) * ((muf[r0] + muf[r0 + 1]) + (muf[r1] + muf[r1 + 1]));
}

// Coarse right-hand side = average of the four fine residuals; coarse correction = 0.
template <typename T>
__global__ void __launch_bounds__(PX* PY) k_mg_restrict_residual(PotLevel<T> F, PotLevel<T> Cl) {
    const int I = blockIdx.x * PX + threadIdx.x, J = blockIdx.y * PY + threadIdx.y;
    if (I >= Cl.nx || J >= Cl.ny) return;
    T s = T(0);
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const int i = 2 * I + di, j = 2 * J + dj;
            const MgEval<T> r = mg_eval(F, i, j);
            s += r.rhs - (r.acc - r.C * F.u[(long long)j * F.pitch + i]);
        }
    const long long k = (long long)J * Cl.pitch + I;
    Cl.f[k] = T(0.25) * s;
    Cl.u[k] = T(0);
}

// Fine correction += bilinear interpolation of the coarse correction (weights 9/16,
// 3/16, 3/16, 1/16 of the four nearest coarse nodes; coarse ghost rows by the kappa rule).
template <typename T>
__global__ void __launch_bounds__(PX* PY) k_mg_prolong(PotLevel<T> Cl, PotLevel<T> F) {
    const int i = blockIdx.x * PX + threadIdx.x, j = blockIdx.y * PY + threadIdx.y;
    if (i >= F.nx || j >= F.ny) return;
    const int I = i >> 1, J = j >> 1;
    const int I2 = (i & 1) ? (I + 1 == Cl.nx ? 0 : I + 1) : (I == 0 ? Cl.nx - 1 : I - 1);
    int J2 = (j & 1) ? J + 1 : J - 1;
    T gy = T(1);
    if (J2 < 0) {
        J2 = 0;
        gy = -Cl.kappa;
    } else if (J2 >= Cl.ny) {
        J2 = Cl.ny - 1;
        gy = -Cl.kappa;
    }
    const T* e = Cl.u;
    const long long rJ = (long long)J * Cl.pitch, rJ2 = (long long)J2 * Cl.pitch;
    const T v = T(9) / T(16) * e[rJ + I] + T(3) / T(16) * (gy * e[rJ2 + I] + e[rJ + I2]) +
                T(1) / T(16) * gy * e[rJ2 + I2];
    F.u[(long long)j * F.pitch + i] += v;
}

// Coarsest level: the whole level in LDS, `iters` four-colour SOR sweeps by one block.
constexpr int COARSE_T = 256;

template <typename T>
__global__ void __launch_bounds__(COARSE_T) k_mg_coarse_solve(PotLevel<T> L, int iters, T omega) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* su = reinterpret_cast<T*>(lds_raw);
    const int n = L.nx * L.ny;
    T* sf = su + n;
    T* smu = sf + n;
    for (int t = threadIdx.x; t < n; t += COARSE_T) {
        const int j = t / L.nx, i = t - j * L.nx;
        const long long k = (long long)j * L.pitch + i;
        su[t] = L.u[k];
        sf[t] = L.f[k];
        smu[t] = L.mu[k];
    }
    __syncthreads();
    PotLevel<T> S = L;
    S.u = su;
    S.f = sf;
    S.mu = smu;
    S.pitch = L.nx;
    const int hx = (L.nx + 1) / 2, hy = (L.ny + 1) / 2;
    for (int it = 0; it < iters; ++it)
        for (int colour = 0; colour < 4; ++colour) {
            for (int t = threadIdx.x; t < hx * hy; t += COARSE_T) {
                const int tj = t / hx, ti = t - tj * hx;
                const int i = 2 * ti + (colour & 1), j = 2 * tj + (colour >> 1);
                if (i < L.nx && j < L.ny) relax_node(S, i, j, omega);
            }
            __syncthreads();
        }
    for (int t = threadIdx.x; t < n; t += COARSE_T) {
        const int j = t / L.nx, i = t - j * L.nx;
        L.u[(long long)j * L.pitch + i] = su[t];
    }
}

// Warm start: mode 0 keeps psi' and records it; mode 1 replaces psi' by the linear
// extrapolation 2 psi'(t-1) - psi'(t-2) and records psi'(t-1).
template <typename T>
__global__ void __launch_bounds__(PX* PY) k_psi_history(T* __restrict__ psi, T* __restrict__ prev, int nx, int ny,
                                                        int pitch, int mode) {
    const int i = blockIdx.x * PX + threadIdx.x, j = blockIdx.y * PY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const long long k = (long long)j * pitch + i;
    const T cur = psi[k];
    if (mode == 1) psi[k] = T(2) * cur - prev[k];
    prev[k] = cur;
}

// ---------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------
static inline dim3 pgrid(int nx, int ny) { return dim3((nx + PX - 1) / PX, (ny + PY - 1) / PY); }

template <typename T>
void launch_pot_sweep(const PotLevel<T>& L, T omega, hipStream_t s) {
    const dim3 g = pgrid((L.nx + 1) / 2, (L.ny + 1) / 2);
    for (int c = 0; c < 4; ++c) hipLaunchKernelGGL(k_pot_relax_colour<T>, g, dim3(PX, PY), 0, s, L, c, omega);
}

template <typename T>
void launch_pot_residual(const PotLevel<T>& L, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, out, 2LL, 0ULL);
    const long long n = (long long)L.nx * L.ny;
    long long blocks = (n + RES_T - 1) / RES_T;
    if (blocks > RES_MAX_BLOCKS) blocks = RES_MAX_BLOCKS;
    hipLaunchKernelGGL(k_pot_residual<T>, dim3((unsigned)blocks), dim3(RES_T), 0, s, L, out);
}

template <typename T>
void launch_mg_restrict_mu(const T* muf, int pitchf, T* muc, int nxc, int nyc, int pitchc, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_restrict_mu<T>, pgrid(nxc, nyc), dim3(PX, PY), 0, s, muf, pitchf, muc, nxc, nyc, pitchc);
}

template <typename T>
void launch_mg_restrict_residual(const PotLevel<T>& F, const PotLevel<T>& C, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_restrict_residual<T>, pgrid(C.nx, C.ny), dim3(PX, PY), 0, s, F, C);
}

template <typename T>
void launch_mg_prolong(const PotLevel<T>& C, const PotLevel<T>& F, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_prolong<T>, pgrid(F.nx, F.ny), dim3(PX, PY), 0, s, C, F);
}

template <typename T>
size_t mg_coarse_lds_bytes(int nx, int ny) {
    return (size_t)3 * nx * ny * sizeof(T);
}

template <typename T>
void launch_mg_coarse_solve(const PotLevel<T>& L, int iters, T omega, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_coarse_solve<T>, dim3(1), dim3(COARSE_T), mg_coarse_lds_bytes<T>(L.nx, L.ny), s, L, iters,
                       omega);
}

template <typename T>
void launch_psi_history(T* psi, T* prev, int nx, int ny, int pitch, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_psi_history<T>, pgrid(nx, ny), dim3(PX, PY), 0, s, psi, prev, nx, ny, pitch, mode);
}

#define FCD_POT_INSTANTIATE(T)                                                                            \
    template void launch_pot_sweep<T>(const PotLevel<T>&, T, hipStream_t);                                \
    template void launch_pot_residual<T>(const PotLevel<T>&, unsigned long long*, hipStream_t);           \
    template void launch_mg_restrict_mu<T>(const T*, int, T*, int, int, int, hipStream_t);                \
    template void launch_mg_restrict_residual<T>(const PotLevel<T>&, const PotLevel<T>&, hipStream_t);    \
    template void launch_mg_prolong<T>(const PotLevel<T>&, const PotLevel<T>&, hipStream_t);              \
    template size_t mg_coarse_lds_bytes<T>(int, int);                                                     \
    template void launch_mg_coarse_solve<T>(const PotLevel<T>&, int, T, hipStream_t);                     \
    template void launch_psi_history<T>(T*, T*, int, int, int, int, hipStream_t);

FCD_POT_INSTANTIATE(double)
FCD_POT_INSTANTIATE(float)

}  // namespace fcd
