// fcd_step.hpp -- one node of the phase-moment pass and of the fused collide-and-stream
// pass (shared by the single-channel and batched kernels).
#pragma once

#include <hip/hip_runtime.h>

#include "fcd_device.hpp"


namespace fcd {

// Load of a state value read once per step.  In FP64 the two state buffers (2 x 27
// planes) exceed the 256 MB last-level cache of the 2048 x 512 channel, so the loads are
// marked non-temporal (they do not displace lines that are reused); in FP32 the state
// fits and the plain load lets the next step find it in the cache.
template <typename T>
__device__ __forceinline__ T ld_state(const T* p) {
    if constexpr (sizeof(T) == 8)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Order parameters (Eq. 32, 24) and mu_r = 1 / sum phi_i/(1+chi_i) (Eq. 8) at (i, j).
template <typename T>
__device__ __forceinline__ void phase_node(const T* __restrict__ dist, T* __restrict__ phi, const StepConst<T>& P,
                                           int i, int j) {
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

// Divergence guard: a node whose velocity exceeds the limit, or whose p*, phi1 or phi2
// (sums over every population of f, g1, g2, so any non-finite population shows) is not
// finite, raises the flag word `div` to the bit pattern of its max(|u_x|, |u_y|) (a
// quiet NaN for a non-finite node).  Patterns of non-negative doubles order like their
// values and NaN above them all, so atomicMax keeps the worst node.  The test is one
// comparison per node; the atomic runs only on a diverged node.
template <typename T>
__device__ __forceinline__ void note_divergence(unsigned long long* __restrict__ div, const NodeOut<T>& o,
                                                T limit) {
    const T um = fmax(fabs(o.ux), fabs(o.uy));
    const T chk = o.pstar + (o.phi1 + o.phi2);
    const bool finite = chk - chk == T(0);  // false for NaN and +-Inf
    if (!(um <= limit) || !finite) {
        const double v = finite ? (double)um : __longlong_as_double(0x7ff8000000000000LL);
        atomicMax(div, (unsigned long long)__double_as_longlong(v));
    }
}

// Stencils + forces + MRT collision of f + phase-field collisions of g1, g2 at (i, j),
// then push streaming with halfway bounce-back at the walls.  The phi1, phi2 and psi'
// neighbourhoods are given (from global memory or from an LDS tile).  div (nullable):
// the divergence flag word.
template <typename T>
__device__ __forceinline__ void collide_stream_nb(const T* __restrict__ src, T* __restrict__ dst,
                                                  const Nb9<T>& a1, const Nb9<T>& a2, const Nb9<T>& ps,
                                                  const StepConst<T>& P, int i, int j,
                                                  unsigned long long* __restrict__ div) {
    const long long pl = P.plane;
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    const long long k = x.c;
    T f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = ld_state(src + a * pl + k);
    const NodeOut<T> o = node_physics(P, f, a1, a2, ps);
    if (div) note_divergence(div, o, P.u_limit);

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
        for (int a = 0; a < 9; ++a) g[a] = ld_state(S + a * pl + k);
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

// The same with the neighbourhoods read from global memory.
template <typename T>
__device__ __forceinline__ void collide_stream_node(const T* __restrict__ src, T* __restrict__ dst,
                                                    const T* __restrict__ phi, const T* __restrict__ psi,
                                                    const StepConst<T>& P, int i, int j) {
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    collide_stream_nb(src, dst, load_nb(phi, x), load_nb(phi + P.plane, x), load_nb_psi(psi, x, j, P.ny), P, i, j,
                      nullptr);
}

}  // namespace fcd
