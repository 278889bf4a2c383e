// fcd_adjoint.hip -- kernels of the reverse (adjoint) coupled step.
//
// With s_{t+1} = S(s_t, p) the forward step, the adjoint step maps lambda_{t+1} (the
// adjoint of the post-streaming state s_{t+1}) to lambda_t and accumulates p-bar:
//   1. k_adj_node: the transpose of push streaming is a pull from lambda_{t+1} (halfway
//      bounce-back transposes to the opposite direction at the same node); the node
//      adjoint then gives the adjoint of the node's f, g1, g2, sensitivities to the
//      phi1/phi2 stencil quantities and to grad psi', and parameter partials.
//   2. k_adj_gather_psi: transpose of the grad psi' stencil -> right-hand side psi'-bar of
//      the adjoint potential equation L lambda_psi = psi'-bar (L symmetric).
//   3. (host) multigrid solve of that equation on the current mu_r.
//   4. k_adj_finish: transpose of the phi stencils (with the mirror ghost rows), the
//      bond terms of d(lambda_psi^T (s - L psi'))/d mu_r, the chain through
//      mu_r(phi1, phi2) (Eq. 8), and phi-bar -> g-bar (phi_i = sum g^i, Eq. 32).
//   5. k_adj_reduce: deterministic sum of per-block parameter partials.
#include <hip/hip_runtime.h>

#include "fcd_adjoint.hpp"
#include "fcd_adjoint_kernels.hpp"
#include "fcd_batch.hpp"
#include "fcd_device.hpp"
#include "fcd_step.hpp"

namespace fcd {

constexpr int AX = 64;
constexpr int AY = 4;
constexpr int AT = AX * AY;

// Deterministic block sum of NV values per thread into part[blk][0..NV) (64 x 4 blocks).
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* __restrict__ part, long long blk) {
    __shared__ double wsum[NV][AY];
    const int lane = threadIdx.x, wave = threadIdx.y;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) wsum[q][wave] = s;
    }
    __syncthreads();
    const int t = wave * AX + lane;
    if (t < NV) {
        double s = 0.0;
        for (int w = 0; w < AY; ++w) s += wsum[t][w];
        part[blk * ADJ_NPART + t] = s;
    }
}

// Adjoint of one node's update: pull of lambda_{t+1}, node adjoint, writes of lambda_t
// (local part), the ten stencil sensitivities and the 13 parameter partials into pv.
template <typename T>
__device__ __forceinline__ void adj_node_at(const StepConst<T>& P, const T* __restrict__ st,
                                            const T* __restrict__ phi, const T* __restrict__ psi,
                                            const T* __restrict__ lam_next, T* __restrict__ lam,
                                            T* __restrict__ sens, int i, int j, double (&pv)[13]) {
    const long long pl = P.plane;
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    const long long k = x.c;
    T f[9], g1[9], g2[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f[a] = st[a * pl + k];
        g1[a] = st[(9 + a) * pl + k];
        g2[a] = st[(18 + a) * pl + k];
    }
    // pull of the next adjoint: direction a came from (i + ex, j + ey), or from the
    // opposite direction at this node when that lies beyond a wall
    const bool bot = j == 0, top = j == P.ny - 1;
    const long long src[9] = {k, x.e, top ? k : x.n, x.w, bot ? k : x.s, top ? k : x.ne, top ? k : x.nw,
                              bot ? k : x.sw, bot ? k : x.se};
    const int pln[9] = {0, 1, top ? 4 : 2, 3, bot ? 2 : 4, top ? 7 : 5, top ? 8 : 6, bot ? 5 : 7, bot ? 6 : 8};
    T Yf[9], Yg1[9], Yg2[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        Yf[a] = lam_next[pln[a] * pl + src[a]];
        Yg1[a] = lam_next[(9 + pln[a]) * pl + src[a]];
        Yg2[a] = lam_next[(18 + pln[a]) * pl + src[a]];
    }
    const NodeAdj<T> R = node_adjoint(P, f, g1, g2, load_nb(phi, x), load_nb(phi + pl, x),
                                      load_nb_psi(psi, x, j, P.ny), Yf, Yg1, Yg2);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        lam[a * pl + k] = R.f[a];
        lam[(9 + a) * pl + k] = R.g1[a];
        lam[(18 + a) * pl + k] = R.g2[a];
    }
    const T sv[10] = {R.p1, R.gx1, R.gy1, R.l1, R.p2, R.gx2, R.gy2, R.l2, R.gpx, R.gpy};
#pragma unroll
    for (int q = 0; q < 10; ++q) sens[q * pl + k] = sv[q];
    const T pp[13] = {R.H0x, R.H0y, R.drive, R.s12, R.s13, R.s23, R.gam0,
                      R.gam1, R.gam2, R.igam0, R.igam1, R.igam2, R.cbulk};
#pragma unroll
    for (int q = 0; q < 13; ++q) pv[q] = (double)pp[q];
}

template <typename T>
__global__ void __launch_bounds__(AT) k_adj_node(const T* __restrict__ st, const T* __restrict__ phi,
                                                 const T* __restrict__ psi, const T* __restrict__ lam_next,
                                                 T* __restrict__ lam, T* __restrict__ sens,
                                                 double* __restrict__ part, StepConst<T> P) {
    const int i = blockIdx.x * AX + threadIdx.x, j = blockIdx.y * AY + threadIdx.y;
    double pv[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) pv[q] = 0.0;
    if (i < P.nx && j < P.ny) adj_node_at(P, st, phi, psi, lam_next, lam, sens, i, j, pv);
    block_partials<13>(pv, part, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// psi'-bar(y) = sum over x = y - e_a inside the channel of 3 w_a e_a . (grad psi')-bar(x)
// (rows beyond the walls hold psi' = 0, so they pass nothing on).  Also max |psi'-bar|.
template <typename T>
__device__ __forceinline__ double adj_gather_at(const StepConst<T>& P, const T* __restrict__ sens,
                                                T* __restrict__ rhs, int i, int j) {
    const long long pl = P.plane;
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    const T* gx = sens + 8 * pl;
    const T* gy = sens + 9 * pl;
    const bool hasS = j > 0, hasN = j < P.ny - 1;
    const T third = T(1) / T(3), tw = T(1) / T(12);
    T v = third * (gx[x.w] - gx[x.e]);
    if (hasS) v += third * gy[x.s] + tw * ((gx[x.sw] + gy[x.sw]) + (gy[x.se] - gx[x.se]));
    if (hasN) v += -third * gy[x.n] + tw * ((gx[x.nw] - gy[x.nw]) - (gx[x.ne] + gy[x.ne]));
    rhs[x.c] = v;
    return fabs((double)v);
}

// Block max of m, one atomicMax per block into *out.
__device__ __forceinline__ void block_max_to(double m, unsigned long long* __restrict__ out) {
    __shared__ double wmax[AY];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (threadIdx.x == 0) wmax[threadIdx.y] = m;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double r = wmax[0];
        for (int w = 1; w < AY; ++w) r = fmax(r, wmax[w]);
        atomicMax(out, (unsigned long long)__double_as_longlong(r));
    }
}

template <typename T>
__global__ void __launch_bounds__(AT) k_adj_gather_psi(const T* __restrict__ sens, T* __restrict__ rhs,
                                                       unsigned long long* __restrict__ rmax, StepConst<T> P) {
    const int i = blockIdx.x * AX + threadIdx.x, j = blockIdx.y * AY + threadIdx.y;
    double m = 0.0;
    if (i < P.nx && j < P.ny) m = adj_gather_at(P, sens, rhs, i, j);
    block_max_to(m, rmax);
}

// Transpose of one phi stencil (gradient weights 3 w_a e_a, Laplacian weights 6 w_a and
// -10/3 at the centre, rows beyond the walls mirrored onto the edge rows) at node y.
template <typename T>
__device__ __forceinline__ T phi_transpose(const T* __restrict__ sp, const T* __restrict__ sgx,
                                           const T* __restrict__ sgy, const T* __restrict__ sl, const NbIdx& x,
                                           int j, int ny) {
    const T third = T(1) / T(3), tw = T(1) / T(12), la = T(2) / T(3), ld = T(1) / T(6);
    T v = sp[x.c] - T(10) / T(3) * sl[x.c];
    v += third * (sgx[x.w] - sgx[x.e]) + la * (sl[x.w] + sl[x.e]);
    if (j > 0) {
        v += third * sgy[x.s] + la * sl[x.s];
        v += tw * (sgx[x.sw] + sgy[x.sw]) + ld * sl[x.sw];
        v += tw * (sgy[x.se] - sgx[x.se]) + ld * sl[x.se];
    } else {  // mirror: this row stands in for the ghost row below
        v += -third * sgy[x.c] + la * sl[x.c];
        v += -tw * (sgx[x.e] + sgy[x.e]) + ld * sl[x.e];
        v += tw * (sgx[x.w] - sgy[x.w]) + ld * sl[x.w];
    }
    if (j < ny - 1) {
        v += -third * sgy[x.n] + la * sl[x.n];
        v += -tw * (sgx[x.ne] + sgy[x.ne]) + ld * sl[x.ne];
        v += tw * (sgx[x.nw] - sgy[x.nw]) + ld * sl[x.nw];
    } else {  // mirror: this row stands in for the ghost row above
        v += third * sgy[x.c] + la * sl[x.c];
        v += tw * (sgx[x.w] + sgy[x.w]) + ld * sl[x.w];
        v += tw * (sgy[x.e] - sgx[x.e]) + ld * sl[x.e];
    }
    return v;
}

// Bond term of the adjoint potential for the bond from node y in direction a with
// coefficient c = 3 w_a (mu(y) + mu(z)): c-bar = (l_y - l_z)(H0 e_a.h - psi'_z + psi'_y),
// with l_z = psi'_z = 0 beyond a wall.
template <typename T>
__device__ __forceinline__ T bond_bar(T ly, T lz, T py, T pz, T eh) {
    return (ly - lz) * (eh - pz + py);
}

template <typename T>
__device__ __forceinline__ void adj_finish_at(const StepConst<T>& P, const T* __restrict__ sens,
                                              const T* __restrict__ phi, const T* __restrict__ psi,
                                              const T* __restrict__ lpsi, T* __restrict__ lam, int i, int j,
                                              double (&pv)[2]) {
    const long long pl = P.plane;
    const NbIdx x = nb_index(i, j, P.nx, P.ny, P.pitch);
    const long long k = x.c;
    T p1b = phi_transpose(sens, sens + pl, sens + 2 * pl, sens + 3 * pl, x, j, P.ny);
    T p2b = phi_transpose(sens + 4 * pl, sens + 5 * pl, sens + 6 * pl, sens + 7 * pl, x, j, P.ny);
    // adjoint potential: mu-bar from the bond terms
    const T* mu = phi + 2 * pl;
    const bool bot = j == 0, top = j == P.ny - 1;
    const T ly = lpsi[k], py = psi[k];
    const T hx = P.H0x, hy = P.H0y;
    const T wa = T(1) / T(3), wd = T(1) / T(12);
    // neighbour values (zero beyond the walls)
    const T lE = lpsi[x.e], lW = lpsi[x.w], pE = psi[x.e], pW = psi[x.w];
    const T lN = top ? T(0) : lpsi[x.n], pN = top ? T(0) : psi[x.n];
    const T lS = bot ? T(0) : lpsi[x.s], pS = bot ? T(0) : psi[x.s];
    const T lNE = top ? T(0) : lpsi[x.ne], pNE = top ? T(0) : psi[x.ne];
    const T lNW = top ? T(0) : lpsi[x.nw], pNW = top ? T(0) : psi[x.nw];
    const T lSW = bot ? T(0) : lpsi[x.sw], pSW = bot ? T(0) : psi[x.sw];
    const T lSE = bot ? T(0) : lpsi[x.se], pSE = bot ? T(0) : psi[x.se];
    T mub = wa * (bond_bar(ly, lE, py, pE, hx) + bond_bar(ly, lW, py, pW, -hx) + bond_bar(ly, lN, py, pN, hy) +
                  bond_bar(ly, lS, py, pS, -hy)) +
            wd * (bond_bar(ly, lNE, py, pNE, hx + hy) + bond_bar(ly, lNW, py, pNW, hy - hx) +
                  bond_bar(ly, lSW, py, pSW, -hx - hy) + bond_bar(ly, lSE, py, pSE, hx - hy));
    // ghost bonds of edge-row nodes whose mirrored mu is this node's
    if (bot) {
        mub += wa * bond_bar(ly, T(0), py, T(0), -hy);
        mub += wd * bond_bar(lpsi[x.e], T(0), psi[x.e], T(0), -hx - hy);  // SW bond of the east node
        mub += wd * bond_bar(lpsi[x.w], T(0), psi[x.w], T(0), hx - hy);   // SE bond of the west node
    }
    if (top) {
        mub += wa * bond_bar(ly, T(0), py, T(0), hy);
        mub += wd * bond_bar(lpsi[x.w], T(0), psi[x.w], T(0), hx + hy);   // NE bond of the west node
        mub += wd * bond_bar(lpsi[x.e], T(0), psi[x.e], T(0), hy - hx);   // NW bond of the east node
    }
    // mu_r = 1 / (ic0 phi1 + ic1 phi2 + ic2 phi3), phi3 = 1 - phi1 - phi2 (Eq. 8)
    const T m = mu[k];
    p1b += -mub * m * m * (P.ic0 - P.ic2);
    p2b += -mub * m * m * (P.ic1 - P.ic2);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        lam[(9 + a) * pl + k] += p1b;
        lam[(18 + a) * pl + k] += p2b;
    }
    // lambda_psi^T ds/dH0x, ds/dH0y with s = sum_a c_a (e_a . (H0x, H0y))
    const Nb9<T> mm = load_nb(mu, x);
    const T ce = wa * (mm.c + mm.e), cw = wa * (mm.c + mm.w), cn = wa * (mm.c + mm.n), cs = wa * (mm.c + mm.s);
    const T cne = wd * (mm.c + mm.ne), cnw = wd * (mm.c + mm.nw), csw = wd * (mm.c + mm.sw),
            cse = wd * (mm.c + mm.se);
    pv[0] = (double)(ly * ((ce - cw) + (cne - csw) + (cse - cnw)));
    pv[1] = (double)(ly * ((cn - cs) + (cne - csw) + (cnw - cse)));
}

template <typename T>
__global__ void __launch_bounds__(AT) k_adj_finish(const T* __restrict__ sens, const T* __restrict__ phi,
                                                   const T* __restrict__ psi, const T* __restrict__ lpsi,
                                                   T* __restrict__ lam, double* __restrict__ part, StepConst<T> P) {
    const int i = blockIdx.x * AX + threadIdx.x, j = blockIdx.y * AY + threadIdx.y;
    double pv[2] = {0.0, 0.0};
    if (i < P.nx && j < P.ny) adj_finish_at(P, sens, phi, psi, lpsi, lam, i, j, pv);
    block_partials<2>(pv, part, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// Sum of the per-block partials in a fixed order: acc[q] += sum_b part[b][q] for the
// first nq slots, into acc slots starting at dst.
// One block of RED_T threads: thread t sums the partials of blocks t, t + RED_T, ... for
// every quantity, then the threads' sums are combined by a fixed wave-shuffle and LDS
// tree, so the result does not depend on scheduling.
constexpr int RED_T = 256;

__global__ void __launch_bounds__(RED_T) k_adj_reduce(const double* __restrict__ part, int nblocks, int nq,
                                                      double* __restrict__ acc, int dst) {
    __shared__ double wsum[ADJ_NPART][RED_T / 64];
    double v[ADJ_NPART];
#pragma unroll
    for (int q = 0; q < ADJ_NPART; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_T) {
        const double* p = part + (long long)b * ADJ_NPART;
#pragma unroll
        for (int q = 0; q < ADJ_NPART; ++q)
            if (q < nq) v[q] += p[q];
    }
#pragma unroll
    for (int q = 0; q < ADJ_NPART; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & 63) == 0) wsum[q][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < nq) {
        double s = 0.0;
        for (int w = 0; w < RED_T / 64; ++w) s += wsum[q][w];
        acc[dst + q] += s;
    }
}

// Adjoint of the final state from J = dJ[0] D_o + dJ[1] D_i (second-moment deformation
// with a circular-mean centroid in x).  dg holds, for the shell weight w_o = phi1 + phi2
// and the core weight w_i = phi1: S, C, Sn, y_c, x_c, I_xx, I_yy, sum w dx (8 each).
template <typename T>
__global__ void __launch_bounds__(AT) k_adj_seed(const T* __restrict__ phi, const double* __restrict__ dg,
                                                 double dJo, double dJi, T* __restrict__ lam, StepConst<T> P) {
    const int i = blockIdx.x * AX + threadIdx.x, j = blockIdx.y * AY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const double twopi = 6.283185307179586476925286766559;
    double sn, cs;
    sincos(twopi * i / P.nx, &sn, &cs);
    double dw[2];
    for (int s = 0; s < 2; ++s) {
        const double* d = dg + 8 * s;
        const double S = d[0], C = d[1], Sn = d[2], yc = d[3], xc = d[4], Ixx = d[5], Iyy = d[6], Sdx = d[7];
        double dx = (double)i - xc;
        dx -= P.nx * floor(dx / P.nx + 0.5);
        const double dy = (double)j - yc;
        const double a = sqrt(Iyy), b = sqrt(Ixx), ab = (a + b) * (a + b);
        const double dD_dIyy = b / (a * ab), dD_dIxx = -a / (b * ab);
        const double dxc = P.nx / twopi * (C * sn - Sn * cs) / (C * C + Sn * Sn);
        const double dIxx = (dx * dx - Ixx) / S + (-2.0 * Sdx / S) * dxc;
        const double dIyy = (dy * dy - Iyy) / S;
        dw[s] = dD_dIxx * dIxx + dD_dIyy * dIyy;
    }
    const long long k = (long long)j * P.pitch + i, pl = P.plane;
    const T b1 = T(dJo * dw[0] + dJi * dw[1]), b2 = T(dJo * dw[0]);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        lam[a * pl + k] = T(0);
        lam[(9 + a) * pl + k] = b1;
        lam[(18 + a) * pl + k] = b2;
    }
}

// lambda_0 . d s_0 / d G for the initial state of the compound-droplet set-up, whose
// Poiseuille velocity U(y) = G (y + 1/2)(ny - 1/2 - y) / (2 rho_3 nu_3) enters f = f^eq(0, u)
// and g^i = phi_i Gamma(u).
template <typename T>
__global__ void __launch_bounds__(AT) k_adj_init_drive(const T* __restrict__ s0, const T* __restrict__ lam0,
                                                       double dU_dG_scale, double u_scale,
                                                       double* __restrict__ part, StepConst<T> P) {
    const int i = blockIdx.x * AX + threadIdx.x, j = blockIdx.y * AY + threadIdx.y;
    double pv[1] = {0.0};
    if (i < P.nx && j < P.ny) {
        const long long k = (long long)j * P.pitch + i, pl = P.plane;
        const double prof = (j + 0.5) * (P.ny - 0.5 - j);
        const double U = u_scale * prof, dUdG = dU_dG_scale * prof;
        double phi1 = 0.0, phi2 = 0.0;
        for (int a = 0; a < 9; ++a) {
            phi1 += (double)s0[(9 + a) * pl + k];
            phi2 += (double)s0[(18 + a) * pl + k];
        }
        const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        double acc = 0.0;
        for (int a = 0; a < 9; ++a) {
            const double w = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
            const double d = w * (3.0 * ex[a] + 9.0 * ex[a] * ex[a] * U - 3.0 * U);
            acc += d * ((double)lam0[a * pl + k] + phi1 * (double)lam0[(9 + a) * pl + k] +
                        phi2 * (double)lam0[(18 + a) * pl + k]);
        }
        pv[0] = acc * dUdG;
    }
    block_partials<1>(pv, part, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// ---------------------------------------------------------------------------------
// Batched adjoint: the same per-node functions over the batch's 64 x 4 tile list, each
// tile mapped to its channel; per-block partials indexed by the global tile.
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool batch_tile_node(const BatchInst<T>& B, int& i, int& j) {
    const int lt = blockIdx.x - B.tile0[2];
    const int ty = lt / B.tiles_x[2], tx = lt - ty * B.tiles_x[2];
    i = tx * AX + threadIdx.x;
    j = ty * AY + threadIdx.y;
    return i < B.P.nx && j < B.P.ny;
}

// what 0: the 27 state planes of dist[cur] into record r; what 1: psi' into record r.
template <typename T>
__global__ void __launch_bounds__(AT) kba_save(const BatchInst<T>* __restrict__ inst,
                                               const BatchAdj<T>* __restrict__ adj, const int* __restrict__ tiles,
                                               int cur, int r, int what) {
    const int k = tiles[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    if (!batch_tile_node(B, i, j)) return;
    const long long pl = B.P.plane, q = (long long)j * B.P.pitch + i;
    T* rec = adj[k].seg + (long long)r * adj[k].srec;
    if (what == 0) {
        const T* src = B.dist[cur];
#pragma unroll
        for (int a = 0; a < 27; ++a) rec[a * pl + q] = src[a * pl + q];
    } else {
        rec[27 * pl + q] = B.L0.u[q];
    }
}

template <typename T>
__global__ void __launch_bounds__(AT) kba_phase(const BatchInst<T>* __restrict__ inst,
                                                const BatchAdj<T>* __restrict__ adj, const int* __restrict__ tiles,
                                                int r) {
    const int k = tiles[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    if (!batch_tile_node(B, i, j)) return;
    phase_node(adj[k].seg + (long long)r * adj[k].srec, B.phi, B.P, i, j);
}

template <typename T>
__global__ void __launch_bounds__(AT) kba_node(const BatchInst<T>* __restrict__ inst,
                                               const BatchAdj<T>* __restrict__ adj, const int* __restrict__ tiles,
                                               int r, int A, double* __restrict__ part) {
    const int k = tiles[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    const BatchAdj<T>& D = adj[k];
    double pv[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) pv[q] = 0.0;
    int i, j;
    if (batch_tile_node(B, i, j)) {
        const T* rec = D.seg + (long long)r * D.srec;
        adj_node_at(B.P, rec, B.phi, rec + 27 * B.P.plane, D.lam[A], D.lam[1 - A], D.sens, i, j, pv);
    }
    block_partials<13>(pv, part, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(AT) kba_gather(const BatchInst<T>* __restrict__ inst,
                                                 const BatchAdj<T>* __restrict__ adj, const int* __restrict__ tiles,
                                                 unsigned long long* __restrict__ scale) {
    const int k = tiles[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    double m = 0.0;
    int i, j;
    if (batch_tile_node(B, i, j)) m = adj_gather_at(B.P, adj[k].sens, adj[k].rhs, i, j);
    block_max_to(m, scale + k);
}

template <typename T>
__global__ void __launch_bounds__(AT) kba_finish(const BatchInst<T>* __restrict__ inst,
                                                 const BatchInst<T>* __restrict__ ainst,
                                                 const BatchAdj<T>* __restrict__ adj, const int* __restrict__ tiles,
                                                 int r, int A, double* __restrict__ part) {
    const int k = tiles[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    const BatchAdj<T>& D = adj[k];
    double pv[2] = {0.0, 0.0};
    int i, j;
    if (batch_tile_node(B, i, j)) {
        const T* psi = D.seg + (long long)r * D.srec + 27 * B.P.plane;
        adj_finish_at(B.P, D.sens, B.phi, psi, ainst[k].L0.u, D.lam[1 - A], i, j, pv);
    }
    block_partials<2>(pv, part, blockIdx.x);
}

// One block per channel: acc[16 k + dst + q] += sum over the channel's tiles, in order.
template <typename T>
__global__ void kba_reduce(const BatchAdj<T>* __restrict__ adj, const double* __restrict__ part, int nq,
                           double* __restrict__ acc, int dst) {
    const int k = blockIdx.x, q = threadIdx.x;
    if (q >= nq) return;
    const BatchAdj<T>& D = adj[k];
    double s = 0.0;
    for (int t = 0; t < D.tile_count; ++t) s += part[(long long)(D.tile_first + t) * ADJ_NPART + q];
    acc[16 * k + dst + q] += s;
}

// ---------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------
static inline dim3 agrid(int nx, int ny) { return dim3((nx + AX - 1) / AX, (ny + AY - 1) / AY); }

int adj_blocks(int nx, int ny) { return ((nx + AX - 1) / AX) * ((ny + AY - 1) / AY); }

template <typename T>
void launch_adj_node(const T* st, const T* phi, const T* psi, const T* lam_next, T* lam, T* sens, double* part,
                     const StepConst<T>& P, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_node<T>, agrid(P.nx, P.ny), dim3(AX, AY), 0, s, st, phi, psi, lam_next, lam, sens, part,
                       P);
}

template <typename T>
void launch_adj_gather_psi(const T* sens, T* rhs, unsigned long long* rmax, const StepConst<T>& P, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, rmax, 1LL, 0ULL);
    hipLaunchKernelGGL(k_adj_gather_psi<T>, agrid(P.nx, P.ny), dim3(AX, AY), 0, s, sens, rhs, rmax, P);
}

template <typename T>
void launch_adj_finish(const T* sens, const T* phi, const T* psi, const T* lpsi, T* lam, double* part,
                       const StepConst<T>& P, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_finish<T>, agrid(P.nx, P.ny), dim3(AX, AY), 0, s, sens, phi, psi, lpsi, lam, part, P);
}

void launch_adj_reduce(const double* part, int nblocks, int nq, double* acc, int dst, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(RED_T), 0, s, part, nblocks, nq, acc, dst);
}

template <typename T>
void launch_adj_seed(const T* phi, const double* dg, double dJo, double dJi, T* lam, const StepConst<T>& P,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_adj_seed<T>, agrid(P.nx, P.ny), dim3(AX, AY), 0, s, phi, dg, dJo, dJi, lam, P);
}

template <typename T>
void launch_adj_init_drive(const T* s0, const T* lam0, double dU_dG_scale, double u_scale, double* part,
                           const StepConst<T>& P, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_init_drive<T>, agrid(P.nx, P.ny), dim3(AX, AY), 0, s, s0, lam0, dU_dG_scale, u_scale,
                       part, P);
}

template <typename T>
void launch_batch_adj_save(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t, int cur, int r,
                           int what, hipStream_t s) {
    hipLaunchKernelGGL(kba_save<T>, dim3(t.ntiles), dim3(AX, AY), 0, s, inst, adj, t.tiles, cur, r, what);
}

template <typename T>
void launch_batch_adj_phase(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t, int r,
                            hipStream_t s) {
    hipLaunchKernelGGL(kba_phase<T>, dim3(t.ntiles), dim3(AX, AY), 0, s, inst, adj, t.tiles, r);
}

template <typename T>
void launch_batch_adj_node(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t, int r, int A,
                           double* part, hipStream_t s) {
    hipLaunchKernelGGL(kba_node<T>, dim3(t.ntiles), dim3(AX, AY), 0, s, inst, adj, t.tiles, r, A, part);
}

template <typename T>
void launch_batch_adj_gather(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t,
                             unsigned long long* scale, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3((n + 255) / 256), dim3(256), 0, s, scale, (long long)n, 0ULL);
    hipLaunchKernelGGL(kba_gather<T>, dim3(t.ntiles), dim3(AX, AY), 0, s, inst, adj, t.tiles, scale);
}

template <typename T>
void launch_batch_adj_finish(const BatchInst<T>* inst, const BatchInst<T>* ainst, const BatchAdj<T>* adj,
                             const BatchTiles& t, int r, int A, double* part, hipStream_t s) {
    hipLaunchKernelGGL(kba_finish<T>, dim3(t.ntiles), dim3(AX, AY), 0, s, inst, ainst, adj, t.tiles, r, A, part);
}

template <typename T>
void launch_batch_adj_reduce(const BatchAdj<T>* adj, int n, const double* part, int nq, double* acc, int dst,
                             hipStream_t s) {
    hipLaunchKernelGGL(kba_reduce<T>, dim3(n), dim3(64), 0, s, adj, part, nq, acc, dst);
}

#define FCD_BADJ_INSTANTIATE(T)                                                                                  \
    template void launch_batch_adj_save<T>(const BatchInst<T>*, const BatchAdj<T>*, const BatchTiles&, int, int, \
                                           int, hipStream_t);                                                    \
    template void launch_batch_adj_phase<T>(const BatchInst<T>*, const BatchAdj<T>*, const BatchTiles&, int,     \
                                            hipStream_t);                                                        \
    template void launch_batch_adj_node<T>(const BatchInst<T>*, const BatchAdj<T>*, const BatchTiles&, int, int, \
                                           double*, hipStream_t);                                                \
    template void launch_batch_adj_gather<T>(const BatchInst<T>*, const BatchAdj<T>*, const BatchTiles&,         \
                                             unsigned long long*, int, hipStream_t);                             \
    template void launch_batch_adj_finish<T>(const BatchInst<T>*, const BatchInst<T>*, const BatchAdj<T>*,       \
                                             const BatchTiles&, int, int, double*, hipStream_t);                 \
    template void launch_batch_adj_reduce<T>(const BatchAdj<T>*, int, const double*, int, double*, int, hipStream_t);

FCD_BADJ_INSTANTIATE(double)
FCD_BADJ_INSTANTIATE(float)

#define FCD_ADJ_INSTANTIATE(T)                                                                                    \
    template void launch_adj_node<T>(const T*, const T*, const T*, const T*, T*, T*, double*, const StepConst<T>&, \
                                     hipStream_t);                                                                \
    template void launch_adj_gather_psi<T>(const T*, T*, unsigned long long*, const StepConst<T>&, hipStream_t);  \
    template void launch_adj_finish<T>(const T*, const T*, const T*, const T*, T*, double*, const StepConst<T>&,  \
                                       hipStream_t);                                                              \
    template void launch_adj_seed<T>(const T*, const double*, double, double, T*, const StepConst<T>&, hipStream_t); \
    template void launch_adj_init_drive<T>(const T*, const T*, double, double, double*, const StepConst<T>&,      \
                                           hipStream_t);

FCD_ADJ_INSTANTIATE(double)
FCD_ADJ_INSTANTIATE(float)

}  // namespace fcd
