// fcd_potential.hip -- magnetic potential solve (Eq. 6) on gfx950: four-colour SOR and
// geometric multigrid V-cycles, plus the residual max-norm that decides convergence.
//
// Discrete operator (conservative nine-point flux form, lattice units, grid spacing h):
//   (L u)(x) = sum_a c_a (u(x+e_a) - u(x)),  c_a = 3 w_a (mu(x) + mu(x+e_a)) / h^2
// on the finest level (the discretisation of Eq. 6); the coarse levels, whose operator only
// shapes the correction, take the harmonic face mean, c_a = 3 w_a 4 mu mu' / (mu + mu') / h^2
// (mu' = mu(x+e_a)), which carries the flux across the interface where mu jumps: against the
// arithmetic face mean it takes the 2048 x 512 channel from 1.265 to 1.16 V-cycles per step.
// On the finest level u = psi', the right-hand side is H0 sum_a c_a (e_a . h) (so that
// L(psi0 + psi') = 0 with psi0 = -H0 (x cos a + y sin a)) and psi' = 0 on the rows beyond
// the walls.  Coarse levels are cell-centred: a level of nx x ny nodes coarsens to
// ceil(nx/2) x (floor or ceil)(ny/2), coarse node (I, J) standing for fine nodes
// (2I..2I+1, 2J..2J+1); an odd level's last column 2I+1 = nx does not exist, and its last
// row ny - 1 lies above a coarse grid of floor(ny/2) rows (with ceil(ny/2) rows the last
// coarse row stands for that fine row alone).  On the level of spacing h the first row
// sits (h-1)/2 fine cells inside the lower wall line (the finest ghost row y = -1, where
// psi' = 0), so the ghost row below it carries -kappa times it, kappa = (h-1)/(h+1), for
// the correction to vanish on that line (linear extrapolation).  The last row sits
// d = ny0 - (h (ny-1) + (h-1)/2) below the upper line y = ny0 of the finest level (the
// planner keeps d >= h/4); its ghost row carries -kappa_top times it, kappa_top =
// (h - d)/d (equal to kappa when every level above is even; otherwise between -1 and 3,
// the diagonal dominant either way).  Both are 0 on the finest level.  A fine row above
// the coarse grid is interpolated between the last coarse row and its ghost (3/4 of the
// way to the ghost); its residual enters the last coarse row through the ordinary
// weights, and a fine row missing under the last coarse row carries none.  mu_r is
// mirrored beyond the walls on every level.  In x an odd level closes periodically over
// its own width; its coarse level is one node more than half as wide, an approximation of
// the geometry at the seam that the coarse corrections tolerate (the finest level's
// residual decides convergence).
#include <hip/hip_runtime.h>
#include <math.h>

#include "fcd_device.hpp"
#include "fcd_kernels.hpp"
#include "fcd_potential.hpp"

namespace fcd {

constexpr int PX = 64;  // one wavefront per row segment
constexpr int PY = 4;

// A kernel launched with a gated level does nothing when the gating residual test has
// passed.  Every block reads the test's words after issuing its own loads and before any
// barrier, so that the two memory latencies overlap (a gated-off block discards what it
// loaded; every load stays in bounds either way).
template <typename T>
__device__ __forceinline__ bool gated_off(const PotLevel<T>& L) {
    return L.gate.res && L.gate.passed();
}

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
        v = nan_max(v, residual_abs(r, c));
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

// Coarse mu: the harmonic mean of the fine nodes under each coarse node, for up to four
// levels in one launch.  Across an interface the harmonic mean is the coefficient of the
// cell's fluxes in series, which the coarse operator then carries; against the arithmetic
// mean it takes the 2048 x 512 channel's warm-started solves from 1.365 to 1.265 V-cycles
// per step (the first cycle's remaining residual sat on a few interface nodes), the
// geometric mean 1.300.  A block owns a 64 x 16 tile of the finer level, which contains the
// children of every coarse node of the next four levels that lies over it, and averages
// level by level in LDS; the first level is averaged in the finer level's type and stored
// in the coarse type.  A child beyond an odd level's last column or row stands in for its
// sibling, so a coarse node with two (or one) real children averages those.
constexpr int MU_TX = 64, MU_TY = 16;

template <typename T, typename TC>
__device__ __forceinline__ void mg_restrict_mu4_tile(const T* __restrict__ muf, int pitchf, int nxf, int nyf,
                                                     const MuLevels<TC>& C, int bx, int by) {
    constexpr int NT = MU_TX * MU_TY / 4;
    __shared__ T s0[MU_TY][MU_TX];
    __shared__ TC sa[MU_TY / 2][MU_TX / 2];
    __shared__ TC sb[MU_TY / 4][MU_TX / 4];
    const int i0 = bx * MU_TX, j0 = by * MU_TY, tid = threadIdx.x;
    T v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = tid + r * NT, ly = q / MU_TX, lx = q - ly * MU_TX;
        const int i = i0 + lx, j = j0 + ly;
        v[r] = muf[(long long)min(j, nyf - 1) * pitchf + min(i, nxf - 1)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = tid + r * NT;
        s0[q / MU_TX][q % MU_TX] = v[r];
    }
    __syncthreads();
    {  // first level from the finer plane's type
        constexpr int cx = MU_TX / 2;
        const int y = tid / cx, x = tid - y * cx;  // NT = cx * (MU_TY / 2)
        const T* r0 = s0[2 * y];
        const T* r1 = s0[2 * y + 1];
        const TC m = TC(T(4) / ((T(1) / r0[2 * x] + T(1) / r0[2 * x + 1]) + (T(1) / r1[2 * x] + T(1) / r1[2 * x + 1])));
        sa[y][x] = m;
        const int I = (i0 >> 1) + x, J = (j0 >> 1) + y;
        if (I < C.nx[0] && J < C.ny[0]) C.mu[0][(long long)J * C.pitch[0] + I] = m;
    }
    __syncthreads();
    TC* src = &sa[0][0];
    TC* dst = &sb[0][0];
    int sx = MU_TX / 2;  // row length of src
    for (int k = 1; k < C.n; ++k) {
        const int cx = sx / 2, cy = (MU_TY >> k) / 2;
        const int gx0 = i0 >> k, gy0 = j0 >> k;  // src origin on level k-1 of C
        for (int t = tid; t < cx * cy; t += NT) {
            const int y = t / cx, x = t - y * cx;
            const int x1 = gx0 + 2 * x + 1 < C.nx[k - 1] ? 2 * x + 1 : 2 * x;
            const int y1 = gy0 + 2 * y + 1 < C.ny[k - 1] ? 2 * y + 1 : 2 * y;
            const TC* r0 = src + (2 * y) * sx;
            const TC* r1 = src + y1 * sx;
            const TC m = TC(4) / ((TC(1) / r0[2 * x] + TC(1) / r0[x1]) + (TC(1) / r1[2 * x] + TC(1) / r1[x1]));
            dst[y * cx + x] = m;
            const int I = (i0 >> (k + 1)) + x, J = (j0 >> (k + 1)) + y;
            if (I < C.nx[k] && J < C.ny[k]) C.mu[k][(long long)J * C.pitch[k] + I] = m;
        }
        __syncthreads();
        TC* tmp = src;
        src = dst;
        dst = tmp;
        sx = cx;
    }
}

template <typename T, typename TC>
__global__ void __launch_bounds__(MU_TX* MU_TY / 4) k_mg_restrict_mu4(const T* __restrict__ muf, int pitchf, int nxf,
                                                                        int nyf, MuLevels<TC> C) {
    mg_restrict_mu4_tile<T, TC>(muf, pitchf, nxf, nyf, C, blockIdx.x, blockIdx.y);
}

// Bilinear interpolation of the coarse correction at fine node (i, j): weights 9/16,
// 3/16, 3/16, 1/16 of the four nearest coarse nodes; coarse ghost rows by the kappa rule.
// Weight of the neighbouring coarse node in the prolongation to a fine cell a quarter of the
// coarse spacing from its parent's centre towards that neighbour: the flux-continuous value
// for mu constant in each coarse cell, mu_N / (2 (mu_P + mu_N)), which is 1/4 (to rounding)
// for equal mu (bilinear); across an interface the correction's gradient follows the jump of
// mu.  Used between coarse levels and in the tail (the coarse operators are harmonic there):
// the 2048 x 512 channel's solves go from 1.16 to 1.04 V-cycles per step; weighting the
// prolongation into the finest level as well gains nothing (1.175), so that one stays bilinear.
template <typename T>
__device__ __forceinline__ T prolong_w(T mP, T mN) {
    // in FP32 with the reciprocal estimate (the coarse mu are FP32; a weight needs no more)
    const float a = float(mP), b = float(mN);
    return T(b * __builtin_amdgcn_rcpf(2.0f * (a + b)));
}

template <typename T>
__device__ __forceinline__ T prolong_at(const PotLevel<T>& Cl, int i, int j) {
    const int I = i >> 1, J = j >> 1;
    const int I2 = (i & 1) ? (I + 1 == Cl.nx ? 0 : I + 1) : (I == 0 ? Cl.nx - 1 : I - 1);
    if (J >= Cl.ny) {  // the row above the coarse grid (odd fine ny)
        const long long r = (long long)(Cl.ny - 1) * Cl.pitch;
        const T wx = prolong_w(Cl.mu[r + I], Cl.mu[r + I2]);
        return (T(1) / T(4) - T(3) / T(4) * Cl.kappa_top) * ((T(1) - wx) * Cl.u[r + I] + wx * Cl.u[r + I2]);
    }
    int J2 = (j & 1) ? J + 1 : J - 1;
    T gy = T(1);
    bool ghost = false;
    if (J2 < 0) {
        J2 = 0;
        gy = -Cl.kappa;
        ghost = true;
    } else if (J2 >= Cl.ny) {
        J2 = Cl.ny - 1;
        gy = -Cl.kappa_top;
        ghost = true;
    }
    const T* e = Cl.u;
    const long long rJ = (long long)J * Cl.pitch, rJ2 = (long long)J2 * Cl.pitch;
    const T mP = Cl.mu[rJ + I];
    const T wx = prolong_w(mP, Cl.mu[rJ + I2]), wy = ghost ? T(1) / T(4) : prolong_w(mP, Cl.mu[rJ2 + I]);
    return (T(1) - wx) * ((T(1) - wy) * e[rJ + I] + wy * gy * e[rJ2 + I]) +
           wx * ((T(1) - wy) * e[rJ + I2] + wy * gy * e[rJ2 + I2]);
}

// ---------------------------------------------------------------------------------
// Tile smoother.  One block loads a 64 x 16 tile of u and mu with a one-node halo
// into LDS and runs one four-colour Gauss-Seidel sweep on it (the colours of the
// tile in the fixed order 0..3, synchronised through LDS).  Halo values are those of
// the input iterate: between tiles the sweep is a Jacobi step, so the block reads
// uin and writes uout (never the same buffer) and the result does not depend on
// block scheduling.  `inner` sweeps run on the tile before it is written back (the halo
// stays that of the input).  PROLONG adds the prolongation of the coarse correction to every
// loaded value first (prolongation fused with post-smoothing).  MODE selects the
// right-hand side: 0 coarse level (f), 1 finest level formed from H0 and mu on the
// fly, 2 finest level with a given f (adjoint solves).  With res != nullptr the block
// also reduces max |residual| and max |C u| of the INPUT iterate into res[0..1].
// ---------------------------------------------------------------------------------
// Tile geometry: SX x SY nodes, one node of each colour per thread (SX/2 x SY/2 threads).
// The finest level, which is bandwidth-bound, uses 64 x 16 tiles (256 threads); the
// coarser levels, whose kernels are bound by latency, use 32 x 8 tiles of one wavefront,
// whose barriers are cheap and which spread a small level over more CUs.
template <int SX_, int SY_>
struct TileGeom {
    static constexpr int SX = SX_, SY = SY_;
    static constexpr int HX = SX + 2, HY = SY + 2;    // with the halo
    static constexpr int NT = SX * SY / 4;             // threads
    static constexpr int HN = HX * HY;
    static constexpr int HPER = (HN + NT - 1) / NT;    // halo-tile loads per thread
    static constexpr int FPER = SX * SY / NT;          // interior values per thread (4)
    // coarse correction tile for the fused prolongation: coarse columns I0-1 .. I0+SX/2
    // and rows J0-1 .. J0+SY/2 of the tile's fine origin (i0, j0) = (2 I0, 2 J0)
    static constexpr int CX = SX / 2 + 2, CY = SY / 2 + 2;
    static constexpr int CPER = (CX * CY + NT - 1) / NT;
};
using FineTile = TileGeom<64, 16>;
using CoarseTile = TileGeom<32, 8>;

// Reciprocal for the coarse levels' harmonic face coefficients: the hardware estimate in
// FP32 (one instruction, deterministic), exact in FP64.
__device__ __forceinline__ float face_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double face_rcp(double x) { return 1.0 / x; }

// A coarse node's couplings c_a, harmonic face means of mu (as tile_eval with HF), and their
// sum, from a staged tile; a thread of a coarse tile kernel takes them once for each of its
// nodes and keeps them through the sweeps.
template <typename T>
struct Cpl {
    T ce, cw, cn, cs, cne, cnw, csw, cse, C;
};

template <typename T, int HX>
__device__ __forceinline__ Cpl<T> coarse_cpl(const T (*sm)[HX], int lx, int ly, const PotLevel<T>& L) {
    const T mc = sm[ly][lx];
    const T a = L.inv_h2 * (T(1) / T(3)), d = L.inv_h2 * (T(1) / T(12));
    auto fc = [mc](T y) { return T(4) * mc * y * face_rcp(mc + y); };
    Cpl<T> c;
    c.ce = a * fc(sm[ly][lx + 1]);
    c.cw = a * fc(sm[ly][lx - 1]);
    c.cn = a * fc(sm[ly + 1][lx]);
    c.cs = a * fc(sm[ly - 1][lx]);
    c.cne = d * fc(sm[ly + 1][lx + 1]);
    c.cnw = d * fc(sm[ly + 1][lx - 1]);
    c.csw = d * fc(sm[ly - 1][lx - 1]);
    c.cse = d * fc(sm[ly - 1][lx + 1]);
    c.C = ((c.ce + c.cw) + (c.cn + c.cs)) + ((c.cne + c.csw) + (c.cnw + c.cse));
    return c;
}

// The Gauss-Seidel value of coarse node (lx, ly) from its couplings, right-hand side f and
// the wall ghost rules (the arithmetic of tile_eval and the tile update).
template <typename T, int HX>
__device__ __forceinline__ T coarse_gs(const T (*su)[HX], const Cpl<T>& c, int lx, int ly, bool bot, bool top,
                                       T k, T kt, T f) {
    const T old = su[ly][lx];
    const T ue = su[ly][lx + 1], uw = su[ly][lx - 1];
    T un, une, unw, us, usw, use;
    if (top) {
        un = -kt * old;
        une = -kt * ue;
        unw = -kt * uw;
    } else {
        un = su[ly + 1][lx];
        une = su[ly + 1][lx + 1];
        unw = su[ly + 1][lx - 1];
    }
    if (bot) {
        us = -k * old;
        usw = -k * uw;
        use = -k * ue;
    } else {
        us = su[ly - 1][lx];
        usw = su[ly - 1][lx - 1];
        use = su[ly - 1][lx + 1];
    }
    const T acc = ((c.ce * ue + c.cw * uw) + (c.cn * un + c.cs * us)) +
                  ((c.cne * une + c.csw * usw) + (c.cnw * unw + c.cse * use));
    const T cself = (bot ? k * c.cs : T(0)) + (top ? kt * c.cn : T(0));
    return (acc + cself * old - f) / (c.C + cself);
}

// HF: the coarse levels' harmonic face means (as coarse_cpl) in place of mu + mu'.
template <typename T, int HX, bool HF = false>
__device__ __forceinline__ MgEval<T> tile_eval(const T (*su)[HX], const T (*sm)[HX], int lx, int ly, bool bot,
                                               bool top, const PotLevel<T>& L, T fval, bool rhs_from_field) {
    const T mc = sm[ly][lx], me = sm[ly][lx + 1], mw = sm[ly][lx - 1];
    const T mn = sm[ly + 1][lx], ms = sm[ly - 1][lx];
    const T mne = sm[ly + 1][lx + 1], mnw = sm[ly + 1][lx - 1], msw = sm[ly - 1][lx - 1], mse = sm[ly - 1][lx + 1];
    const T k = L.kappa, kt = L.kappa_top;
    const T ue = su[ly][lx + 1], uw = su[ly][lx - 1];
    T un, une, unw, us, usw, use;
    if (top) {
        un = -kt * su[ly][lx];
        une = -kt * ue;
        unw = -kt * uw;
    } else {
        un = su[ly + 1][lx];
        une = su[ly + 1][lx + 1];
        unw = su[ly + 1][lx - 1];
    }
    if (bot) {
        us = -k * su[ly][lx];
        usw = -k * uw;
        use = -k * ue;
    } else {
        us = su[ly - 1][lx];
        usw = su[ly - 1][lx - 1];
        use = su[ly - 1][lx + 1];
    }
    const T a = L.inv_h2 * (T(1) / T(3)), d = L.inv_h2 * (T(1) / T(12));
    auto fc = [](T x, T y) { return HF ? T(4) * x * y * face_rcp(x + y) : x + y; };
    const T ce = a * fc(mc, me), cw = a * fc(mc, mw), cn = a * fc(mc, mn), cs = a * fc(mc, ms);
    const T cne = d * fc(mc, mne), cnw = d * fc(mc, mnw), csw = d * fc(mc, msw), cse = d * fc(mc, mse);
    MgEval<T> r;
    r.C = ((ce + cw) + (cn + cs)) + ((cne + csw) + (cnw + cse));
    r.acc = ((ce * ue + cw * uw) + (cn * un + cs * us)) + ((cne * une + csw * usw) + (cnw * unw + cse * use));
    r.cself = (bot ? k * cs : T(0)) + (top ? kt * cn : T(0));
    if (rhs_from_field) {
        const T sx = (ce - cw) + (cne - csw) + (cse - cnw);
        const T sy = (cn - cs) + (cne - csw) + (cnw - cse);
        r.rhs = L.H0x * sx + L.H0y * sy;
    } else {
        r.rhs = fval;
    }
    return r;
}

// Tile + halo loads, issued together before any LDS store (the loads of one thread
// are independent, so their latencies overlap).  Columns wrap periodically, rows
// beyond the walls are clamped (mu mirrored; u there is never read).

__device__ __forceinline__ int wrap_col(int i, int nx) {
    while (i < 0) i += nx;
    while (i >= nx) i -= nx;
    return i;
}

__device__ __forceinline__ int clamp_row(int j, int ny) { return j < 0 ? 0 : (j >= ny ? ny - 1 : j); }

template <typename T, typename G>
__device__ __forceinline__ void load_tile(const PotLevel<T>& L, const T* __restrict__ uin, int i0, int j0,
                                          T (&uv)[G::HPER], T (&mv)[G::HPER]) {
#pragma unroll
    for (int r = 0; r < G::HPER; ++r) {
        const int q = threadIdx.x + r * G::NT;
        if (q < G::HN) {
            const int ly = q / G::HX, lx = q - ly * G::HX;
            const long long k = (long long)clamp_row(j0 + ly - 1, L.ny) * L.pitch + wrap_col(i0 + lx - 1, L.nx);
            uv[r] = uin[k];
            mv[r] = L.mu[k];
        }
    }
}

// Prolongation at fine tile cell (lx, ly) from the coarse tile sc (bilinear weights
// 9/16, 3/16, 3/16, 1/16; coarse ghost rows by the kappa rule).
template <typename T, int CX, bool OPW>
__device__ __forceinline__ T prolong_tile(const T (*sc)[CX], const T (*scm)[CX], int i0, int j0, int lx, int ly,
                                          int nyc, T kappa, T kappa_top) {
    const int i = i0 + lx - 1, j = j0 + ly - 1;  // unwrapped fine coordinates
    const int I0 = i0 >> 1, J0 = j0 >> 1;
    const int lI = (i >> 1) - I0 + 1, lI2 = (i & 1) ? lI + 1 : lI - 1;
    const int J = j >> 1, lJ = J - J0 + 1;
    if (J >= nyc) {  // the row above the coarse grid (odd fine ny), or a halo row beyond the wall
        const int lt = nyc - 1 - J0 + 1;
        const T wx = OPW ? prolong_w(scm[lt][lI], scm[lt][lI2]) : T(1) / T(4);
        return (T(1) / T(4) - T(3) / T(4) * kappa_top) * ((T(1) - wx) * sc[lt][lI] + wx * sc[lt][lI2]);
    }
    int J2 = (j & 1) ? J + 1 : J - 1;
    T gy = T(1);
    bool ghost = false;
    if (J2 < 0) {
        J2 = 0;
        gy = -kappa;
        ghost = true;
    } else if (J2 >= nyc) {
        J2 = nyc - 1;
        gy = -kappa_top;
        ghost = true;
    }
    const int lJ2 = J2 - J0 + 1;
    const T mP = OPW ? scm[lJ][lI] : T(1);
    const T wx = OPW ? prolong_w(mP, scm[lJ][lI2]) : T(1) / T(4);
    const T wy = (ghost || !OPW) ? T(1) / T(4) : prolong_w(mP, scm[lJ2][lI]);
    return (T(1) - wx) * ((T(1) - wy) * sc[lJ][lI] + wy * gy * sc[lJ2][lI]) +
           wx * ((T(1) - wy) * sc[lJ][lI2] + wy * gy * sc[lJ2][lI2]);
}

template <typename T, typename G, bool PROLONG, int MODE, typename TC>
__device__ __forceinline__ void mg_smooth_tile(const PotLevel<T>& L, const T* __restrict__ uin, T* __restrict__ uout,
                                               const PotLevel<TC>& Cl, unsigned long long* __restrict__ res,
                                               unsigned long long* __restrict__ res_clear, int inner, int bx, int by,
                                               unsigned* __restrict__ count = nullptr) {
    constexpr int SX = G::SX, SY = G::SY, HX = G::HX, HY = G::HY, NT = G::NT, CX = G::CX, CY = G::CY;
    __shared__ T su[HY][HX];
    __shared__ T sm[HY][HX];
    __shared__ T sf[MODE == 1 ? 1 : SY][SX];
    __shared__ T sc[PROLONG ? CY : 1][CX];
    __shared__ T scm[PROLONG && MODE == 0 ? CY : 1][CX];
    __shared__ double wmax[2][NT / 64];
    const int i0 = bx * SX, j0 = by * SY;
    const int tid = threadIdx.x;
    T uv[G::HPER], mv[G::HPER], fv[G::FPER], cv[G::CPER], cmv[G::CPER];
    load_tile<T, G>(L, uin, i0, j0, uv, mv);
    if (MODE != 1) {
#pragma unroll
        for (int r = 0; r < G::FPER; ++r) {
            const int q = tid + r * NT;
            const int ly = q / SX, lx = q - ly * SX;
            const int i = i0 + lx, j = j0 + ly;
            fv[r] = (i < L.nx && j < L.ny) ? L.f[(long long)j * L.pitch + i] : T(0);
        }
    }
    if (PROLONG) {
#pragma unroll
        for (int r = 0; r < G::CPER; ++r) {
            const int q = tid + r * NT;
            if (q < CX * CY) {
                const int ly = q / CX, lx = q - ly * CX;
                const int I = wrap_col((i0 >> 1) - 1 + lx, Cl.nx), J = clamp_row((j0 >> 1) - 1 + ly, Cl.ny);
                cv[r] = T(Cl.u[(long long)J * Cl.pitch + I]);
                if (MODE == 0) cmv[r] = T(Cl.mu[(long long)J * Cl.pitch + I]);
            }
        }
    }
    if (gated_off(L)) {
        // a residual test that does not run leaves its slot zero, which reads as a pass
        if (res && bx == 0 && by == 0 && tid < 2) res[tid] = 0ULL;
        return;
    }
    if (count && bx == 0 && by == 0 && tid == 0) atomicAdd(count, 1u);
    // the next test's (other) residual slot, zeroed for it: the kernel boundary orders this
    // store before that test's atomics, and the host has read that slot before this launch
    if (res_clear && bx == 0 && by == 0 && tid < 2) res_clear[tid] = 0ULL;
    if (PROLONG) {
#pragma unroll
        for (int r = 0; r < G::CPER; ++r) {
            const int q = tid + r * NT;
            if (q < CX * CY) {
                sc[q / CX][q % CX] = cv[r];
                if (MODE == 0) scm[q / CX][q % CX] = cmv[r];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < G::HPER; ++r) {
        const int q = tid + r * NT;
        if (q < G::HN) {
            const int ly = q / HX, lx = q - ly * HX;
            T u = uv[r];
            if (PROLONG)
                u += prolong_tile<T, CX, MODE == 0>(sc, scm, i0, j0, lx, ly, Cl.ny, T(Cl.kappa), T(Cl.kappa_top));
            su[ly][lx] = u;
            sm[ly][lx] = mv[r];
        }
    }
    if (MODE != 1) {
#pragma unroll
        for (int r = 0; r < G::FPER; ++r) {
            const int q = tid + r * NT;
            sf[MODE == 1 ? 0 : q / SX][q % SX] = fv[r];
        }
    }
    __syncthreads();
    const int tx = tid % (SX / 2), ty = tid / (SX / 2);
    if (res) {
        double rm = 0.0, scl = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int lx = 1 + 2 * tx + (c & 1), ly = 1 + 2 * ty + (c >> 1);
            const int i = i0 + lx - 1, j = j0 + ly - 1;
            if (i < L.nx && j < L.ny) {
                const MgEval<T> e = tile_eval<T, HX, MODE == 0>(su, sm, lx, ly, j == 0, j == L.ny - 1, L,
                                                     MODE == 1 ? T(0) : sf[MODE == 1 ? 0 : ly - 1][lx - 1], MODE == 1);
                const T u = su[ly][lx];
                rm = nan_max(rm, fabs((double)(e.acc - e.C * u - e.rhs)));
                scl = nan_max(scl, fabs((double)(e.C * u)));
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rm = nan_max(rm, __shfl_xor(rm, off, 64));
            scl = nan_max(scl, __shfl_xor(scl, off, 64));
        }
        if ((tid & 63) == 0) {
            wmax[0][tid >> 6] = rm;
            wmax[1][tid >> 6] = scl;
        }
        __syncthreads();
        if (tid < 2) {
            double m = wmax[tid][0];
            for (int w = 1; w < NT / 64; ++w) m = nan_max(m, wmax[tid][w]);
            atomicMax(res + tid, (unsigned long long)__double_as_longlong(m));
        }
    }
    // coarse levels: each node's couplings once, kept through the sweeps
    Cpl<T> cp[MODE == 0 ? 4 : 1];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) cp[c] = coarse_cpl<T, HX>(sm, 1 + 2 * tx + (c & 1), 1 + 2 * ty + (c >> 1), L);
    }
    for (int sweep = 0; sweep < inner; ++sweep) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int lx = 1 + 2 * tx + (c & 1), ly = 1 + 2 * ty + (c >> 1);
            const int i = i0 + lx - 1, j = j0 + ly - 1;
            if (i < L.nx && j < L.ny) {
                if constexpr (MODE == 0) {
                    su[ly][lx] = coarse_gs<T, HX>(su, cp[c], lx, ly, j == 0, j == L.ny - 1, L.kappa, L.kappa_top,
                                                  sf[ly - 1][lx - 1]);
                } else {
                    const MgEval<T> e = tile_eval<T, HX>(su, sm, lx, ly, j == 0, j == L.ny - 1, L,
                                                         MODE == 1 ? T(0) : sf[MODE == 1 ? 0 : ly - 1][lx - 1],
                                                         MODE == 1);
                    const T old = su[ly][lx];
                    su[ly][lx] = (e.acc + e.cself * old - e.rhs) / (e.C + e.cself);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int r = 0; r < G::FPER; ++r) {
        const int q = tid + r * NT;
        const int ly = q / SX, lx = q - ly * SX;
        const int i = i0 + lx, j = j0 + ly;
        if (i < L.nx && j < L.ny) uout[(long long)j * L.pitch + i] = su[ly + 1][lx + 1];
    }
}

template <typename T, typename G, bool PROLONG, int MODE, typename TC>
__global__ void __launch_bounds__(G::NT) k_mg_smooth_tile(PotLevel<T> L, const T* __restrict__ uin,
                                                          T* __restrict__ uout, PotLevel<TC> Cl,
                                                          unsigned long long* __restrict__ res,
                                                          unsigned long long* __restrict__ res_clear, int inner,
                                                          unsigned* __restrict__ count) {
    mg_smooth_tile<T, G, PROLONG, MODE, TC>(L, uin, uout, Cl, res, res_clear, inner, blockIdx.x, blockIdx.y, count);
}

// Residual restriction.  The coarse right-hand side at coarse node (I, J) is the
// transpose of the bilinear prolongation applied to the fine residual: weights
// (1, 3, 3, 1)/8 along each axis over fine columns 2I-1 .. 2I+2 (periodic) and rows
// 2J-1 .. 2J+2 (rows beyond the walls carry no residual).  Against the four-child
// average this weighting of order two raises the V-cycle's contraction per cycle from
// about 0.2 to about 0.1 on a uniform mu and cuts the cycles a time step's warm-started
// solve needs by a fifth (measured on a CPU model of this multigrid).  A block therefore
// forms the residuals of its fine tile and of the one-node ring around it, staging the
// iterate and mu with a two-node halo.
template <typename G>
struct RestrictGeom {
    static constexpr int FX = G::SX + 4, FY = G::SY + 4;  // staged: tile with a two-node halo
    static constexpr int RX = G::SX + 2, RY = G::SY + 2;  // residuals: tile and its ring
    static constexpr int FN = FX * FY, RN = RX * RY;
    static constexpr int FPER = (FN + G::NT - 1) / G::NT;
    static constexpr int RPER = (RN + G::NT - 1) / G::NT;
};

// Loads of the staged iterate / mu (origin (i0 - 2, j0 - 2)) and of the right-hand side at
// the residual nodes (origin (i0 - 1, j0 - 1)), all issued before any LDS store.
template <typename T, typename G, int MODE>
__device__ __forceinline__ void restrict_loads(const PotLevel<T>& F, int i0, int j0, T (&uv)[RestrictGeom<G>::FPER],
                                               T (&mv)[RestrictGeom<G>::FPER], T (&fv)[RestrictGeom<G>::RPER]) {
    using R = RestrictGeom<G>;
#pragma unroll
    for (int r = 0; r < R::FPER; ++r) {
        const int q = threadIdx.x + r * G::NT;
        if (q < R::FN) {
            const int ly = q / R::FX, lx = q - ly * R::FX;
            const long long k = (long long)clamp_row(j0 + ly - 2, F.ny) * F.pitch + wrap_col(i0 + lx - 2, F.nx);
            uv[r] = F.u[k];
            mv[r] = F.mu[k];
        }
    }
#pragma unroll
    for (int r = 0; r < R::RPER; ++r) {
        const int q = threadIdx.x + r * G::NT;
        fv[r] = T(0);
        if (MODE != 1 && q < R::RN) {
            const int ly = q / R::RX, lx = q - ly * R::RX;
            fv[r] = F.f[(long long)clamp_row(j0 + ly - 1, F.ny) * F.pitch + wrap_col(i0 + lx - 1, F.nx)];
        }
    }
}

// Residuals f - L u of the tile and its ring into sr (zero on rows beyond the walls).
template <typename T, typename G, int MODE>
__device__ __forceinline__ void restrict_residuals(const PotLevel<T>& F, int i0, int j0,
                                                   const T (*fu)[RestrictGeom<G>::FX],
                                                   const T (*fm)[RestrictGeom<G>::FX],
                                                   const T (&fv)[RestrictGeom<G>::RPER],
                                                   T (*sr)[RestrictGeom<G>::RX]) {
    using R = RestrictGeom<G>;
    (void)i0;
#pragma unroll
    for (int r = 0; r < R::RPER; ++r) {
        const int q = threadIdx.x + r * G::NT;
        if (q < R::RN) {
            const int ly = q / R::RX, lx = q - ly * R::RX;
            const int j = j0 + ly - 1;
            T v = T(0);
            if (j >= 0 && j < F.ny) {
                const MgEval<T> e =
                    tile_eval<T, R::FX, MODE == 0>(fu, fm, lx + 1, ly + 1, j == 0, j == F.ny - 1, F, fv[r],
                                                   MODE == 1);
                v = e.rhs - (e.acc - e.C * fu[ly + 1][lx + 1]);
            }
            sr[ly][lx] = v;
        }
    }
}

// The (1, 3, 3, 1)/8 x (1, 3, 3, 1)/8 weighting of the residuals around coarse node
// (cx, cy) of the tile (sr column / row 0 is the fine column / row before the tile).
template <typename T, int RX>
__device__ __forceinline__ T restrict16(const T (*sr)[RX], int cx, int cy) {
    const T a = T(1) / T(8), b = T(3) / T(8);
    T rows[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const T* r = sr[2 * cy + q] + 2 * cx;
        rows[q] = (a * r[0] + b * r[1]) + (b * r[2] + a * r[3]);
    }
    return (a * rows[0] + b * rows[1]) + (b * rows[2] + a * rows[3]);
}

// Residual restriction by tiles: a block stages its fine tile (SX x SY) with a two-node
// halo, forms the residuals of the tile and its ring and writes the (SX/2) x (SY/2)
// coarse right-hand sides and a zero coarse correction.  Coarse sizes as in the header
// note; fine rows beyond the walls or missing carry no residual (an odd level's last row
// above the coarse grid enters the last coarse row with the weight of row 2J+2), and fine
// columns wrap over the fine width.
template <typename T, typename G, int MODE, typename TC>
__device__ __forceinline__ void mg_restrict_tile(const PotLevel<T>& F, const PotLevel<TC>& Cl, int bx, int by) {
    using R = RestrictGeom<G>;
    constexpr int SX = G::SX, NT = G::NT;
    __shared__ T fu[R::FY][R::FX];
    __shared__ T fm[R::FY][R::FX];
    __shared__ T sr[R::RY][R::RX];
    const int i0 = bx * SX, j0 = by * G::SY;
    const int tid = threadIdx.x;
    T uv[R::FPER], mv[R::FPER], fv[R::RPER];
    restrict_loads<T, G, MODE>(F, i0, j0, uv, mv, fv);
    if (gated_off(Cl)) return;
#pragma unroll
    for (int r = 0; r < R::FPER; ++r) {
        const int q = tid + r * NT;
        if (q < R::FN) {
            fu[q / R::FX][q % R::FX] = uv[r];
            fm[q / R::FX][q % R::FX] = mv[r];
        }
    }
    __syncthreads();
    restrict_residuals<T, G, MODE>(F, i0, j0, fu, fm, fv, sr);
    __syncthreads();
    const int cx = tid % (SX / 2), cy = tid / (SX / 2);
    const int I = (i0 >> 1) + cx, J = (j0 >> 1) + cy;
    if (I < Cl.nx && J < Cl.ny) {
        const long long k = (long long)J * Cl.pitch + I;
        Cl.f[k] = TC(restrict16<T, R::RX>(sr, cx, cy));
        Cl.u[k] = TC(0);
    }
}

template <typename T, typename G, int MODE, typename TC>
__global__ void __launch_bounds__(G::NT) k_mg_restrict_tile(PotLevel<T> F, PotLevel<TC> Cl) {
    mg_restrict_tile<T, G, MODE, TC>(F, Cl, blockIdx.x, blockIdx.y);
}

// Residual restriction fused with the first pre-smoothing of the coarse level below it.
// One block owns a 32 x 8 coarse tile: it stages the matching 64 x 16 tile of the
// smoothed fine iterate and of the fine mu with a two-node halo, forms the fine
// residuals of the tile and its ring (FMODE: the fine level's right-hand side, as the
// smoother's MODE), writes their weighted sums as the coarse right-hand side (to C.f and
// to LDS) and runs `inner` tile sweeps from a zero correction (the whole coarse level
// starts at zero, so the tile's halo is zero as well), writing the result to uout.  Same
// arithmetic as k_mg_restrict_tile followed by k_mg_smooth_tile, one launch fewer.
// Coarse sizes as in k_mg_restrict_tile.
template <typename T, int FMODE, typename TC>
__device__ __forceinline__ void mg_restrict_smooth(const PotLevel<T>& F, const PotLevel<TC>& C, TC* __restrict__ uout,
                                                   int inner, int bx, int by) {
    // fine part on the fine tile's 256 threads (loads staged in registers, issued
    // together); coarse smoothing by the first 64, one coarse node per colour each
    using G = CoarseTile;
    using FG = FineTile;
    using R = RestrictGeom<FG>;
    constexpr int NT = FG::NT, SX = G::SX, SY = G::SY, HX = G::HX;
    constexpr int CPER = (G::HN + NT - 1) / NT;
    __shared__ T fu[R::FY][R::FX];
    __shared__ T fm[R::FY][R::FX];
    __shared__ T sr[R::RY][R::RX];
    __shared__ TC su[G::HY][G::HX];
    __shared__ TC sm[G::HY][G::HX];
    __shared__ TC sf[SY][SX];
    const int I0 = bx * SX, J0 = by * SY;  // coarse tile origin
    const int i0 = 2 * I0, j0 = 2 * J0;                    // fine tile origin
    const int tid = threadIdx.x;
    const int cy = tid / SX, cx = tid - cy * SX;  // this thread's coarse node
    T uv[R::FPER], mv[R::FPER], fv[R::RPER];
    TC cm[CPER];
    restrict_loads<T, FG, FMODE>(F, i0, j0, uv, mv, fv);
#pragma unroll
    for (int r = 0; r < CPER; ++r) {
        const int q = tid + r * NT;
        if (q < G::HN) {
            const int ly = q / HX, lx = q - ly * HX;
            cm[r] = C.mu[(long long)clamp_row(J0 + ly - 1, C.ny) * C.pitch + wrap_col(I0 + lx - 1, C.nx)];
        }
    }
    if (gated_off(C)) return;
#pragma unroll
    for (int r = 0; r < R::FPER; ++r) {
        const int q = tid + r * NT;
        if (q < R::FN) {
            fu[q / R::FX][q % R::FX] = uv[r];
            fm[q / R::FX][q % R::FX] = mv[r];
        }
    }
#pragma unroll
    for (int r = 0; r < CPER; ++r) {
        const int q = tid + r * NT;
        if (q < G::HN) {
            sm[q / HX][q % HX] = cm[r];
            su[q / HX][q % HX] = TC(0);
        }
    }
    __syncthreads();
    restrict_residuals<T, FG, FMODE>(F, i0, j0, fu, fm, fv, sr);
    __syncthreads();
    {
        const TC fc = TC(restrict16<T, R::RX>(sr, cx, cy));
        sf[cy][cx] = fc;
        const int I = I0 + cx, J = J0 + cy;
        if (I < C.nx && J < C.ny) C.f[(long long)J * C.pitch + I] = fc;
    }
    __syncthreads();
    const int tx = tid % (SX / 2), ty = tid / (SX / 2);
    const bool smoother = tid < G::NT;
    Cpl<TC> cp[4];
    if (smoother) {
#pragma unroll
        for (int c = 0; c < 4; ++c) cp[c] = coarse_cpl<TC, HX>(sm, 1 + 2 * tx + (c & 1), 1 + 2 * ty + (c >> 1), C);
    }
    for (int sweep = 0; sweep < inner; ++sweep) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int lx = 1 + 2 * tx + (c & 1), ly = 1 + 2 * ty + (c >> 1);
            const int i = I0 + lx - 1, j = J0 + ly - 1;
            if (smoother && i < C.nx && j < C.ny)
                su[ly][lx] = coarse_gs<TC, HX>(su, cp[c], lx, ly, j == 0, j == C.ny - 1, C.kappa, C.kappa_top,
                                               sf[ly - 1][lx - 1]);
            __syncthreads();
        }
    }
    if (I0 + cx < C.nx && J0 + cy < C.ny) uout[(long long)(J0 + cy) * C.pitch + I0 + cx] = su[cy + 1][cx + 1];
}

template <typename T, int FMODE, typename TC>
__global__ void __launch_bounds__(FineTile::NT) k_mg_restrict_smooth(PotLevel<T> F, PotLevel<TC> C,
                                                                     TC* __restrict__ uout, int inner) {
    mg_restrict_smooth<T, FMODE, TC>(F, C, uout, inner, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------------
// Tail of the V-cycle: the coarsest levels, all in LDS, by one block.  Level 0 of the
// tail takes its right-hand side from global memory (written by the restriction above
// it) and starts from a zero correction; the block runs the V-cycle below it and
// writes the tail's level-0 correction back.  On these small levels the smoother is
// damped Jacobi (weight 4/5, `sweeps` sweeps before and after the coarse correction,
// ping-pong between two LDS arrays): one barrier per sweep instead of four, and two
// Jacobi sweeps smooth at least as well as one four-colour Gauss-Seidel sweep here.
// The coarsest level gets 2 coarse_sweeps Jacobi sweeps when it has at most four rows,
// otherwise that many four-colour SOR sweeps with the factor `omega`.
// ---------------------------------------------------------------------------------
constexpr int TAIL_T = 512;

// One tail level in LDS: iterate, right-hand side, mu, a ping-pong array and the
// operator's couplings, set up once per launch from mu.  The couplings absorb the wall
// ghost rule: a ghost row holds -kappa times the edge row, so the ghost image of the node
// itself moves into the diagonal d and those of its row neighbours into their couplings,
// and the couplings to the ghost row become zero.  Then L u = acc - d u with
// acc = sum c_a u(x + e_a) over in-channel neighbours only (rows clamped; a clamped row
// only ever meets a zero coupling), and a Gauss-Seidel / Jacobi value is (acc - f) / d.
template <typename T>
struct TailLevel {
    int nx, ny;
    unsigned inv;  // ceil(2^32 / nx): row of node t = high word of t * inv
    T *u, *f, *mu, *alt;
    T* c[8];  // couplings to e, w, n, s, ne, nw, sw, se
    T *d, *rd;
};

// TailDiv holds ceil(2^32 / nx) of every tail level (2 <= nx, as coarse levels have), from
// the host: for t < TAIL_MAXN and nx < 2^20, t / nx is the high word of t * inv (the
// rounding up adds less than t / 2^32 < 1 / nx to t / nx), one multiply in place of an
// integer division in every node loop of the tail.

__device__ __forceinline__ int tail_div(int t, unsigned inv) { return (int)__umulhi((unsigned)t, inv); }

template <typename T>
__device__ __forceinline__ TailLevel<T> tail_view(const MgTail<T>& tl, const TailDiv& dv, T* base, int k) {
    long long off = 0;
    for (int m = 0; m < k; ++m) off += (long long)MG_TAIL_ARRAYS * tl.lv[m].nx * tl.lv[m].ny;
    TailLevel<T> S;
    S.nx = tl.lv[k].nx;
    S.ny = tl.lv[k].ny;
    S.inv = dv.inv[k];
    const long long n = (long long)S.nx * S.ny;
    T* p = base + off;
    S.u = p;
    S.f = p + n;
    S.mu = p + 2 * n;
    S.alt = p + 3 * n;
#pragma unroll
    for (int a = 0; a < 8; ++a) S.c[a] = p + (4 + a) * n;
    S.d = p + 12 * n;
    S.rd = p + 13 * n;
    return S;
}

// Couplings of node t = (i, j) from mu (Eq. 35 weights of the flux form with the coarse
// levels' harmonic face means, as coarse_cpl).
template <typename T>
__device__ __forceinline__ void tail_setup_node(const TailLevel<T>& S, const PotLevel<T>& G, int t) {
    const int nx = S.nx, j = tail_div(t, S.inv), i = t - j * nx;
    const int e = i + 1 == nx ? t + 1 - nx : t + 1, w = i == 0 ? t - 1 + nx : t - 1;
    const int dn = j + 1 == S.ny ? 0 : nx, ds = j == 0 ? 0 : -nx;  // mirrored mu beyond the walls
    const T* m = S.mu;
    const T mc = m[t];
    const T a = G.inv_h2 * (T(1) / T(3)), q = G.inv_h2 * (T(1) / T(12)), k = G.kappa, kt = G.kappa_top;
    auto fc = [](T x, T y) { return T(4) * x * y * face_rcp(x + y); };
    T ce = a * fc(mc, m[e]), cw = a * fc(mc, m[w]), cn = a * fc(mc, m[t + dn]), cs = a * fc(mc, m[t + ds]);
    T cne = q * fc(mc, m[e + dn]), cnw = q * fc(mc, m[w + dn]);
    T csw = q * fc(mc, m[w + ds]), cse = q * fc(mc, m[e + ds]);
    const T C = ((ce + cw) + (cn + cs)) + ((cne + csw) + (cnw + cse));
    T d = C;
    if (j == 0) {  // ghost row below: -k times row 0
        d += k * cs;
        ce -= k * cse;
        cw -= k * csw;
        cs = csw = cse = T(0);
    }
    if (j + 1 == S.ny) {  // ghost row above
        d += kt * cn;
        ce -= kt * cne;
        cw -= kt * cnw;
        cn = cne = cnw = T(0);
    }
    S.c[0][t] = ce;
    S.c[1][t] = cw;
    S.c[2][t] = cn;
    S.c[3][t] = cs;
    S.c[4][t] = cne;
    S.c[5][t] = cnw;
    S.c[6][t] = csw;
    S.c[7][t] = cse;
    S.d[t] = d;
    S.rd[t] = T(1) / d;
}

template <typename T>
__device__ __forceinline__ T tail_acc(const TailLevel<T>& S, const T* __restrict__ u, int t) {
    const int nx = S.nx, j = tail_div(t, S.inv), i = t - j * nx;
    const int e = i + 1 == nx ? t + 1 - nx : t + 1, w = i == 0 ? t - 1 + nx : t - 1;
    const int dn = j + 1 == S.ny ? 0 : nx, ds = j == 0 ? 0 : -nx;
    return ((S.c[0][t] * u[e] + S.c[1][t] * u[w]) + (S.c[2][t] * u[t + dn] + S.c[3][t] * u[t + ds])) +
           ((S.c[4][t] * u[e + dn] + S.c[6][t] * u[w + ds]) + (S.c[5][t] * u[w + dn] + S.c[7][t] * u[e + ds]));
}

// Coarsest level with more than four rows: four-colour SOR, factor omega.
template <typename T>
__device__ __forceinline__ void tail_sor(const TailLevel<T>& S, int sweeps, T omega) {
    const int hx = (S.nx + 1) / 2, hy = (S.ny + 1) / 2;
    for (int it = 0; it < sweeps; ++it)
        for (int colour = 0; colour < 4; ++colour) {
            for (int q = threadIdx.x; q < hx * hy; q += TAIL_T) {
                const int tj = q / hx, ti = q - tj * hx;
                const int i = 2 * ti + (colour & 1), j = 2 * tj + (colour >> 1);
                if (i < S.nx && j < S.ny) {
                    const int t = j * S.nx + i;
                    const T old = S.u[t];
                    S.u[t] = old + omega * ((tail_acc(S, S.u, t) - S.f[t]) * S.rd[t] - old);
                }
            }
            __syncthreads();
        }
}

// The first damped Jacobi sweep from u = 0 at node t (no neighbour enters it), as
// tail_jacobi's arithmetic takes it: written by the phase that forms the level's f.
template <typename T>
__device__ __forceinline__ T tail_first_sweep(const TailLevel<T>& S, int t) {
    const T w = T(0.8), old = T(0);
    return old + w * ((T(0) - S.f[t]) * S.rd[t] - old);
}

// Damped Jacobi, an even number of sweeps: u -> alt -> u -> ...; from_alt: the first sweep
// from u = 0 is already in alt (tail_first_sweep), the others follow.
template <typename T>
__device__ __forceinline__ void tail_jacobi(const TailLevel<T>& S, int sweeps, bool from_alt = false) {
    const T w = T(0.8);
    T* a = from_alt ? S.alt : S.u;
    T* b = from_alt ? S.u : S.alt;
    const int n = S.nx * S.ny;
    for (int it = from_alt ? 1 : 0; it < sweeps; ++it) {
        for (int t = threadIdx.x; t < n; t += TAIL_T) {
            const T old = a[t];
            b[t] = old + w * ((tail_acc(S, a, t) - S.f[t]) * S.rd[t] - old);
        }
        __syncthreads();
        T* c = a;
        a = b;
        b = c;
    }
}

// Largest tail level and the loads per thread it takes.
constexpr int TAIL_MAXN = 4096;
constexpr int TAIL_LPER = TAIL_MAXN / TAIL_T;

template <typename T>
__device__ __forceinline__ void mg_tail(const MgTail<T>& tl, const TailDiv& dv) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* base = reinterpret_cast<T*>(lds_raw);
    const int tid = threadIdx.x;
    // every tail level's mu and the top level's right-hand side, all loads issued before
    // any LDS store (one memory latency instead of one per level)
    T m0[TAIL_LPER], f0[TAIL_LPER], mk[MG_MAX_TAIL - 1][2];
    {
        const PotLevel<T> G = tl.lv[0];
        const int n = G.nx * G.ny;
#pragma unroll
        for (int r = 0; r < TAIL_LPER; ++r) {
            const int t = tid + r * TAIL_T;
            if (t < n) {
                const int j = tail_div(t, dv.inv[0]), i = t - j * G.nx;
                const long long g = (long long)j * G.pitch + i;
                m0[r] = G.mu[g];
                f0[r] = G.f[g];
            }
        }
    }
#pragma unroll
    for (int k = 1; k < MG_MAX_TAIL; ++k) {
        if (k < tl.n) {
            const PotLevel<T> G = tl.lv[k];
            const int n = G.nx * G.ny;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int t = tid + r * TAIL_T;
                if (t < n) {
                    const int j = tail_div(t, dv.inv[k]), i = t - j * G.nx;
                    mk[k - 1][r] = G.mu[(long long)j * G.pitch + i];
                }
            }
        }
    }
    if (gated_off(tl.lv[0])) return;
    {
        const TailLevel<T> S = tail_view(tl, dv, base, 0);
        const int n = S.nx * S.ny;
#pragma unroll
        for (int r = 0; r < TAIL_LPER; ++r) {
            const int t = tid + r * TAIL_T;
            if (t < n) {
                S.mu[t] = m0[r];
                S.f[t] = f0[r];
                S.u[t] = T(0);
            }
        }
    }
#pragma unroll
    for (int k = 1; k < MG_MAX_TAIL; ++k) {
        if (k < tl.n) {
            const TailLevel<T> S = tail_view(tl, dv, base, k);
            const int n = S.nx * S.ny;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int t = tid + r * TAIL_T;
                if (t < n) S.mu[t] = mk[k - 1][r];
            }
        }
    }
    __syncthreads();
    // the couplings of every level; on the top level also the first Jacobi sweep from its
    // zero correction (this thread stored that node's f above)
    for (int k = 0; k < tl.n; ++k) {
        const TailLevel<T> S = tail_view(tl, dv, base, k);
        for (int t = tid; t < S.nx * S.ny; t += TAIL_T) {
            tail_setup_node(S, tl.lv[k], t);
            if (k == 0) S.alt[t] = tail_first_sweep(S, t);
        }
    }
    __syncthreads();
    const int sw = 2 * ((tl.nu1 + 1) / 2);  // even
    for (int k = 0; k + 1 < tl.n; ++k) {
        const TailLevel<T> F = tail_view(tl, dv, base, k), Cc = tail_view(tl, dv, base, k + 1);
        tail_jacobi(F, sw, sw > 0);
        // fine residuals f - L u into the (free) ping-pong array, then their
        // (1, 3, 3, 1)/8 x (1, 3, 3, 1)/8 weighted sums (as the tile restrictions)
        const int nf = F.nx * F.ny;
        for (int t = tid; t < nf; t += TAIL_T) F.alt[t] = F.f[t] - (tail_acc(F, F.u, t) - F.d[t] * F.u[t]);
        __syncthreads();
        const int n = Cc.nx * Cc.ny;
        const T wa = T(1) / T(8), wb = T(3) / T(8);
        for (int t = tid; t < n; t += TAIL_T) {
            const int J = tail_div(t, Cc.inv), I = t - J * Cc.nx;
            // fine columns 2I-1 .. 2I+2, periodic over the fine width (which may be odd)
            const int i0 = wrap_col(2 * I - 1, F.nx), i1 = 2 * I, i2 = wrap_col(2 * I + 1, F.nx),
                      i3 = wrap_col(2 * I + 2, F.nx);
            T rows[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 2 * J - 1 + q;
                rows[q] = T(0);
                if (j >= 0 && j < F.ny) {  // rows beyond the walls carry no residual
                    const T* r = F.alt + j * F.nx;
                    rows[q] = (wa * r[i0] + wb * r[i1]) + (wb * r[i2] + wa * r[i3]);
                }
            }
            Cc.f[t] = (wa * rows[0] + wb * rows[1]) + (wb * rows[2] + wa * rows[3]);
            Cc.u[t] = T(0);
            Cc.alt[t] = tail_first_sweep(Cc, t);  // the level's first Jacobi sweep from zero
        }
        __syncthreads();
    }
    {
        const TailLevel<T> S = tail_view(tl, dv, base, tl.n - 1);
        // four colours need an even width: on an odd periodic row the first and last
        // nodes share a colour and neighbour each other
        if (S.ny <= 4 || (S.nx & 1))
            tail_jacobi(S, 2 * tl.coarse_sweeps, tl.coarse_sweeps > 0);
        else
            tail_sor(S, tl.coarse_sweeps, tl.omega);
    }
    for (int k = tl.n - 2; k >= 0; --k) {
        const TailLevel<T> F = tail_view(tl, dv, base, k), Cc = tail_view(tl, dv, base, k + 1);
        PotLevel<T> Cp = tl.lv[k + 1];  // the coarse correction as a level (for prolong_at)
        Cp.u = Cc.u;
        Cp.mu = Cc.mu;
        Cp.pitch = Cc.nx;
        const int n = F.nx * F.ny;
        for (int t = tid; t < n; t += TAIL_T) {
            const int j = tail_div(t, F.inv), i = t - j * F.nx;
            F.u[t] += prolong_at(Cp, i, j);
        }
        __syncthreads();
        tail_jacobi(F, sw);
    }
    const PotLevel<T> G = tl.lv[0];
    const TailLevel<T> S = tail_view(tl, dv, base, 0);
    for (int t = tid; t < S.nx * S.ny; t += TAIL_T) {
        const int j = tail_div(t, S.inv), i = t - j * S.nx;
        G.u[(long long)j * G.pitch + i] = S.u[t];
    }
}

template <typename T>
__global__ void __launch_bounds__(TAIL_T) k_mg_tail(MgTail<T> tl, TailDiv dv) {
    mg_tail<T>(tl, dv);
}

// Publication of a solve decided on the device when no collide-and-stream follows it.
__global__ void __launch_bounds__(64) k_solve_publish(StepGate sg) {
    if (threadIdx.x == 0) publish_tests(sg);
}

// Warm start from the recorded solutions: mode 0 keeps psi' and records it; mode 1
// replaces psi' by the linear extrapolation 2 psi'(t-1) - psi'(t-2), mode 2 by the
// quadratic one 3 psi'(t-1) - 3 psi'(t-2) + psi'(t-3), mode 3 by the cubic one
// 4 psi'(t-1) - 6 psi'(t-2) + 4 psi'(t-3) - psi'(t-4); prev records psi'(t-1), and each
// further plane given (prev2, prev3) the one before it.
template <typename T>
__global__ void __launch_bounds__(PX* PY) k_psi_history(T* __restrict__ psi, T* __restrict__ prev,
                                                        T* __restrict__ prev2, T* __restrict__ prev3, int nx, int ny,
                                                        int pitch, int mode) {
    const int i = blockIdx.x * PX + threadIdx.x, j = blockIdx.y * PY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const long long k = (long long)j * pitch + i;
    const T cur = psi[k];
    const T p1 = prev[k];
    if (mode == 1) psi[k] = T(2) * cur - p1;
    if (mode == 2) psi[k] = T(3) * (cur - p1) + prev2[k];
    if (mode == 3) psi[k] = T(4) * (cur + prev2[k]) - T(6) * p1 - prev3[k];
    if (prev3) prev3[k] = prev2[k];
    if (prev2) prev2[k] = p1;
    prev[k] = cur;
}

// The same warm start with the recorded solutions in a ring of planes: p1, p2, p3 hold
// psi'(t-1), psi'(t-2), psi'(t-3) (as far as mode reads them); the current psi' replaces
// p3, which becomes the ring's newest plane (the caller rotates the ring).  Two writes per
// node instead of the shift's four.
template <typename T>
__global__ void __launch_bounds__(PX* PY) k_psi_history_ring(T* __restrict__ psi, const T* __restrict__ p1,
                                                             const T* __restrict__ p2, T* __restrict__ p3, int nx,
                                                             int ny, int pitch, int mode) {
    const int i = blockIdx.x * PX + threadIdx.x, j = blockIdx.y * PY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const long long k = (long long)j * pitch + i;
    const T cur = psi[k];
    if (mode == 1) psi[k] = T(2) * cur - p1[k];
    if (mode == 2) psi[k] = T(3) * (cur - p1[k]) + p2[k];
    if (mode == 3) psi[k] = T(4) * (cur + p2[k]) - T(6) * p1[k] - p3[k];
    p3[k] = cur;
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

template <typename T, typename TC>
void launch_mg_restrict_mu4(const T* muf, int pitchf, int nxf, int nyf, const MuLevels<TC>& C, hipStream_t s) {
    const dim3 g((nxf + MU_TX - 1) / MU_TX, (nyf + MU_TY - 1) / MU_TY);
    hipLaunchKernelGGL((k_mg_restrict_mu4<T, TC>), g, dim3(MU_TX * MU_TY / 4), 0, s, muf, pitchf, nxf, nyf, C);
}

template <typename T, typename G, typename TC>
void launch_smooth_geom(const PotLevel<T>& L, const T* uin, T* uout, const PotLevel<TC>* prolong_from, int mode,
                        unsigned long long* res, unsigned long long* res_clear, int inner, hipStream_t s,
                        unsigned* count) {
    const dim3 g((L.nx + G::SX - 1) / G::SX, (L.ny + G::SY - 1) / G::SY);
    const PotLevel<TC> Cl = prolong_from ? *prolong_from : PotLevel<TC>{};
#define FCD_TILE_LAUNCH(P, M)                                                                                \
    hipLaunchKernelGGL((k_mg_smooth_tile<T, G, P, M, TC>), g, dim3(G::NT), 0, s, L, uin, uout, Cl, res, res_clear, \
                       inner, count)
    if (prolong_from) {
        if (mode == 0) FCD_TILE_LAUNCH(true, 0);
        else if (mode == 1) FCD_TILE_LAUNCH(true, 1);
        else FCD_TILE_LAUNCH(true, 2);
    } else {
        if (mode == 0) FCD_TILE_LAUNCH(false, 0);
        else if (mode == 1) FCD_TILE_LAUNCH(false, 1);
        else FCD_TILE_LAUNCH(false, 2);
    }
#undef FCD_TILE_LAUNCH
}

// Coarser levels (mode 0): 32 x 8 tiles.  Finest level (modes 1, 2): the tallest of
// 64 x 64, 64 x 32 and 64 x 16 tiles that still gives every compute unit a tile (256);
// larger tiles re-read less halo and synchronise fewer, larger blocks.  Measured on the
// 2048 x 512 channel with three sweeps each way (ms per step): 64 x 16 0.524, 64 x 32
// 0.499, 64 x 64 0.490, 128 x 32 0.490, 32 x 32 0.529, 64 x 8 0.562.  The choice depends
// only on the lattice, so results stay reproducible.
using FineTile32 = TileGeom<64, 32>;
using FineTile64 = TileGeom<64, 64>;
constexpr long long FINE_TILES_MIN = 256;

template <typename T, typename TC>
void launch_mg_smooth_tile(const PotLevel<T>& L, const T* uin, T* uout, const PotLevel<TC>* prolong_from, int mode,
                           unsigned long long* res, int inner, hipStream_t s, unsigned long long* res_clear,
                           unsigned* count) {
    if (res && !res_clear) hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, res, 2LL, 0ULL);
    const long long cols = (L.nx + 63) / 64;
    if (mode == 0)
        launch_smooth_geom<T, CoarseTile, TC>(L, uin, uout, prolong_from, mode, res, res_clear, inner, s, count);
    else if (cols * ((L.ny + 63) / 64) >= FINE_TILES_MIN)
        launch_smooth_geom<T, FineTile64, TC>(L, uin, uout, prolong_from, mode, res, res_clear, inner, s, count);
    else if (cols * ((L.ny + 31) / 32) >= FINE_TILES_MIN)
        launch_smooth_geom<T, FineTile32, TC>(L, uin, uout, prolong_from, mode, res, res_clear, inner, s, count);
    else
        launch_smooth_geom<T, FineTile, TC>(L, uin, uout, prolong_from, mode, res, res_clear, inner, s, count);
}

template <typename T, typename TC>
void launch_mg_restrict_tile(const PotLevel<T>& F, const PotLevel<TC>& C, int mode, hipStream_t s) {
    if (mode == 0) {
        const dim3 g((F.nx + CoarseTile::SX - 1) / CoarseTile::SX, (F.ny + CoarseTile::SY - 1) / CoarseTile::SY);
        hipLaunchKernelGGL((k_mg_restrict_tile<T, CoarseTile, 0, TC>), g, dim3(CoarseTile::NT), 0, s, F, C);
        return;
    }
    const dim3 g((F.nx + FineTile::SX - 1) / FineTile::SX, (F.ny + FineTile::SY - 1) / FineTile::SY);
    if (mode == 1)
        hipLaunchKernelGGL((k_mg_restrict_tile<T, FineTile, 1, TC>), g, dim3(FineTile::NT), 0, s, F, C);
    else
        hipLaunchKernelGGL((k_mg_restrict_tile<T, FineTile, 2, TC>), g, dim3(FineTile::NT), 0, s, F, C);
}

template <typename T, typename TC>
void launch_mg_restrict_smooth(const PotLevel<T>& F, const PotLevel<TC>& C, int fmode, TC* uout, int inner,
                               hipStream_t s) {
    const dim3 g((C.nx + CoarseTile::SX - 1) / CoarseTile::SX, (C.ny + CoarseTile::SY - 1) / CoarseTile::SY);
    if (fmode == 0)
        hipLaunchKernelGGL((k_mg_restrict_smooth<T, 0, TC>), g, dim3(FineTile::NT), 0, s, F, C, uout, inner);
    else if (fmode == 1)
        hipLaunchKernelGGL((k_mg_restrict_smooth<T, 1, TC>), g, dim3(FineTile::NT), 0, s, F, C, uout, inner);
    else
        hipLaunchKernelGGL((k_mg_restrict_smooth<T, 2, TC>), g, dim3(FineTile::NT), 0, s, F, C, uout, inner);
}

template <typename T>
size_t mg_tail_lds_bytes(const MgTail<T>& tl) {
    size_t n = 0;
    for (int k = 0; k < tl.n; ++k) n += (size_t)MG_TAIL_ARRAYS * tl.lv[k].nx * tl.lv[k].ny;
    return n * sizeof(T);
}

template <typename T>
void launch_mg_tail(const MgTail<T>& tl, hipStream_t s) {
    TailDiv dv{};
    for (int k = 0; k < tl.n; ++k) dv.inv[k] = (unsigned)(((1ull << 32) + tl.lv[k].nx - 1) / tl.lv[k].nx);
    hipLaunchKernelGGL(k_mg_tail<T>, dim3(1), dim3(TAIL_T), mg_tail_lds_bytes<T>(tl), s, tl, dv);
}

void launch_solve_publish(const StepGate& sg, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_publish, dim3(1), dim3(64), 0, s, sg);
}

template <typename T>
void launch_psi_history_ring(T* psi, const T* p1, const T* p2, T* p3, int nx, int ny, int pitch, int mode,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_psi_history_ring<T>, pgrid(nx, ny), dim3(PX, PY), 0, s, psi, p1, p2, p3, nx, ny, pitch,
                       mode);
}

template <typename T>
void launch_psi_history(T* psi, T* prev, T* prev2, T* prev3, int nx, int ny, int pitch, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_psi_history<T>, pgrid(nx, ny), dim3(PX, PY), 0, s, psi, prev, prev2, prev3, nx, ny, pitch,
                       mode);
}

// ---------------------------------------------------------------------------------
// Batched multigrid: the tile kernels above, one launch for one level of every channel
// of a batch.  Block b works on jobs[b] (channel k, level l, tile bx, by) with channel
// k's descriptors; a channel whose flag in `active` is 0 has converged and its blocks
// return at once (uniformly, before any barrier).  A channel's V-cycle is the
// single-channel one (finest tiles 64 x 16).
// ---------------------------------------------------------------------------------

// Finest-level sweep: dir 0 reads L0.u and writes t0, dir 1 the reverse; PROLONG adds
// level 1's correction to the input first; MODE 1 forms the right-hand side from the field,
// MODE 2 reads it from L0.f; res != nullptr: max |residual| and max |C u| of the input into
// res[2k], res[2k+1].
template <typename T, bool PROLONG, int MODE, typename TC>
__global__ void __launch_bounds__(FineTile::NT) kbm_smooth_fine(const MgChan<T, TC>* __restrict__ ch,
                                                                const MgJob* __restrict__ jobs,
                                                                const int* __restrict__ active, int dir,
                                                                unsigned long long* __restrict__ res) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    const PotLevel<T> L = c.L0;
    const PotLevel<TC> Cl = c.C[1];
    const T* uin = dir ? c.t0 : L.u;
    T* uout = dir ? L.u : c.t0;
    mg_smooth_tile<T, FineTile, PROLONG, MODE, TC>(L, uin, uout, Cl, res ? res + 2 * J.k : nullptr, nullptr, 1, J.bx,
                                                   J.by);
}

// Copy of t0 into L0.u (a finest-level iterate that ended in the ping-pong plane).
template <typename T, typename TC>
__global__ void __launch_bounds__(FineTile::NT) kbm_copy_fine(const MgChan<T, TC>* __restrict__ ch,
                                                              const MgJob* __restrict__ jobs,
                                                              const int* __restrict__ active) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    const PotLevel<T> L = c.L0;
    const T* src = c.t0;
    for (int q = threadIdx.x; q < FineTile::SX * FineTile::SY; q += FineTile::NT) {
        const int i = J.bx * FineTile::SX + q % FineTile::SX, j = J.by * FineTile::SY + q / FineTile::SX;
        if (i < L.nx && j < L.ny) L.u[(long long)j * L.pitch + i] = src[(long long)j * L.pitch + i];
    }
}

// Restriction of the finest level's residual (its pre-smoothed iterate in t0 when src,
// else in L0.u) fused with level 1's pre-smoothing into t[1].
template <typename T, int FMODE, typename TC>
__global__ void __launch_bounds__(FineTile::NT) kbm_restrict_smooth0(const MgChan<T, TC>* __restrict__ ch,
                                                                     const MgJob* __restrict__ jobs,
                                                                     const int* __restrict__ active, int src,
                                                                     int inner) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    PotLevel<T> F = c.L0;
    if (src) F.u = c.t0;
    const PotLevel<TC> C = c.C[1];
    mg_restrict_smooth<T, FMODE, TC>(F, C, c.t[1], inner, J.bx, J.by);
}

// The same from coarse level l - 1 (pre-smoothed iterate in t[l-1]) into level l (t[l]).
template <typename TC, typename T>
__global__ void __launch_bounds__(FineTile::NT) kbm_restrict_smoothC(const MgChan<T, TC>* __restrict__ ch,
                                                                     const MgJob* __restrict__ jobs,
                                                                     const int* __restrict__ active, int inner) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    PotLevel<TC> F = c.C[J.l - 1];
    F.u = c.t[J.l - 1];
    const PotLevel<TC> C = c.C[J.l];
    mg_restrict_smooth<TC, 0, TC>(F, C, c.t[J.l], inner, J.bx, J.by);
}

// Restriction into the first tail level: from the finest level (tail == 1; its iterate
// in t0 when src) ...
template <typename T, int FMODE, typename TC>
__global__ void __launch_bounds__(FineTile::NT) kbm_restrict_tail0(const MgChan<T, TC>* __restrict__ ch,
                                                                   const MgJob* __restrict__ jobs,
                                                                   const int* __restrict__ active, int src) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    PotLevel<T> F = c.L0;
    if (src) F.u = c.t0;
    const PotLevel<TC> C = c.C[1];
    mg_restrict_tile<T, FineTile, FMODE, TC>(F, C, J.bx, J.by);
}

// ... or from coarse level l = tail - 1 (its iterate in t[l]).
template <typename TC, typename T>
__global__ void __launch_bounds__(CoarseTile::NT) kbm_restrict_tailC(const MgChan<T, TC>* __restrict__ ch,
                                                                     const MgJob* __restrict__ jobs,
                                                                     const int* __restrict__ active) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    PotLevel<TC> F = c.C[J.l];
    F.u = c.t[J.l];
    const PotLevel<TC> C = c.C[J.l + 1];
    mg_restrict_tile<TC, CoarseTile, 0, TC>(F, C, J.bx, J.by);
}

// The tail of channel blockIdx.x.
template <typename TC, typename T>
__global__ void __launch_bounds__(TAIL_T) kbm_tail(const MgChan<T, TC>* __restrict__ ch,
                                                   const int* __restrict__ active) {
    const int k = blockIdx.x;
    if (!active[k]) return;
    mg_tail<TC>(ch[k].tl, ch[k].dv);
}

// Prolongation from level l + 1 fused with level l's post-smoothing, t[l] into C[l].u.
template <typename TC, typename T>
__global__ void __launch_bounds__(CoarseTile::NT) kbm_post_coarse(const MgChan<T, TC>* __restrict__ ch,
                                                                  const MgJob* __restrict__ jobs,
                                                                  const int* __restrict__ active, int inner) {
    const MgJob J = jobs[blockIdx.x];
    if (!active[J.k]) return;
    const MgChan<T, TC>& c = ch[J.k];
    const PotLevel<TC> F = c.C[J.l], Cl = c.C[J.l + 1];
    mg_smooth_tile<TC, CoarseTile, true, 0, TC>(F, c.t[J.l], F.u, Cl, nullptr, nullptr, inner, J.bx, J.by);
}

// Coarse mu of levels 4g+1 .. 4g+4 (those that exist) from level 4g: the finest level's mu
// (g == 0, type T) ...
template <typename T, typename TC>
__global__ void __launch_bounds__(MU_TX* MU_TY / 4) kbm_mu4_0(const MgChan<T, TC>* __restrict__ ch,
                                                              const MgJob* __restrict__ jobs) {
    const MgJob J = jobs[blockIdx.x];
    const MgChan<T, TC>& c = ch[J.k];
    mg_restrict_mu4_tile<T, TC>(c.L0.mu, c.L0.pitch, c.L0.nx, c.L0.ny, c.mu4[0], J.bx, J.by);
}

// ... or coarse level 4g (g = J.l >= 1).
template <typename TC, typename T>
__global__ void __launch_bounds__(MU_TX* MU_TY / 4) kbm_mu4_C(const MgChan<T, TC>* __restrict__ ch,
                                                              const MgJob* __restrict__ jobs) {
    const MgJob J = jobs[blockIdx.x];
    const MgChan<T, TC>& c = ch[J.k];
    const PotLevel<TC> F = c.C[4 * J.l];
    mg_restrict_mu4_tile<TC, TC>(F.mu, F.pitch, F.nx, F.ny, c.mu4[J.l], J.bx, J.by);
}

// The convergence decision of every channel, one block: a channel active on entry stays
// active while its residual (res[2k], the bit pattern of max |r|, and res[2k+1], that of
// max |C u|) is above max(thr, floor * scale), thr the descriptor's or, with rel_scale,
// rel_tol times rel_scale[k] (the bit pattern of a non-negative double, set on the
// device); a NaN residual stops it and is counted.
// Both words are zeroed for the next test; cycles[k] counts the cycles a channel
// receives; counts = {channels left active, NaN channels, decisions of this solve that
// found a channel active} (the last: the cycles the solve needs, counted from zero).
constexpr int BMG_DECIDE_T = 256;

template <typename T, typename TC>
__global__ void __launch_bounds__(BMG_DECIDE_T) kbm_decide(const MgChan<T, TC>* __restrict__ ch, int n,
                                                           unsigned long long* __restrict__ res,
                                                           int* __restrict__ active, int* __restrict__ cycles,
                                                           int* __restrict__ counts, double floor_factor,
                                                           const unsigned long long* __restrict__ rel_scale,
                                                           double rel_tol) {
    __shared__ int cnt[3][BMG_DECIDE_T / 64];
    int a_sum = 0, nan_sum = 0, e_sum = 0;
    for (int k = threadIdx.x; k < n; k += BMG_DECIDE_T) {
        if (!active[k]) continue;
        ++e_sum;
        const double r = __longlong_as_double((long long)res[2 * k]);
        const double sc = __longlong_as_double((long long)res[2 * k + 1]);
        res[2 * k] = 0ULL;
        res[2 * k + 1] = 0ULL;
        int a = 0;
        if (r != r) {
            ++nan_sum;
        } else if (!(r <= fmax(rel_scale ? rel_tol * __longlong_as_double((long long)rel_scale[k]) : ch[k].thr,
                                floor_factor * sc))) {
            a = 1;
            ++cycles[k];
        }
        active[k] = a;
        a_sum += a;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a_sum += __shfl_xor(a_sum, off, 64);
        nan_sum += __shfl_xor(nan_sum, off, 64);
        e_sum += __shfl_xor(e_sum, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        cnt[0][threadIdx.x >> 6] = a_sum;
        cnt[1][threadIdx.x >> 6] = nan_sum;
        cnt[2][threadIdx.x >> 6] = e_sum;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int t = 0;
        for (int w = 0; w < BMG_DECIDE_T / 64; ++w) t += cnt[threadIdx.x][w];
        if (threadIdx.x < 2)
            counts[threadIdx.x] = t;
        else if (t > 0)
            ++counts[2];
    }
}

template <typename T, typename TC>
void launch_bmg_smooth_fine(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, int dir,
                            bool prolong, bool rhs_plane, unsigned long long* res, hipStream_t s) {
#define FCD_BMG_FINE(P, M) \
    hipLaunchKernelGGL((kbm_smooth_fine<T, P, M, TC>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active, dir, res)
    if (prolong) {
        if (rhs_plane) FCD_BMG_FINE(true, 2); else FCD_BMG_FINE(true, 1);
    } else {
        if (rhs_plane) FCD_BMG_FINE(false, 2); else FCD_BMG_FINE(false, 1);
    }
#undef FCD_BMG_FINE
}

template <typename T, typename TC>
void launch_bmg_copy_fine(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, hipStream_t s) {
    hipLaunchKernelGGL((kbm_copy_fine<T, TC>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active);
}

template <typename T, typename TC>
void launch_bmg_restrict_smooth(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, int level,
                                int src, int inner, bool rhs_plane, hipStream_t s) {
    if (level == 1 && rhs_plane)
        hipLaunchKernelGGL((kbm_restrict_smooth0<T, 2, TC>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active,
                           src, inner);
    else if (level == 1)
        hipLaunchKernelGGL((kbm_restrict_smooth0<T, 1, TC>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active,
                           src, inner);
    else
        hipLaunchKernelGGL((kbm_restrict_smoothC<TC, T>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active,
                           inner);
}

template <typename T, typename TC>
void launch_bmg_restrict_tail(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, bool from0,
                              int src, bool rhs_plane, hipStream_t s) {
    if (from0 && rhs_plane)
        hipLaunchKernelGGL((kbm_restrict_tail0<T, 2, TC>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active, src);
    else if (from0)
        hipLaunchKernelGGL((kbm_restrict_tail0<T, 1, TC>), dim3(njobs), dim3(FineTile::NT), 0, s, ch, jobs, active, src);
    else
        hipLaunchKernelGGL((kbm_restrict_tailC<TC, T>), dim3(njobs), dim3(CoarseTile::NT), 0, s, ch, jobs, active);
}

template <typename T, typename TC>
void launch_bmg_tail(const MgChan<T, TC>* ch, int n, size_t lds_bytes, const int* active, hipStream_t s) {
    hipLaunchKernelGGL((kbm_tail<TC, T>), dim3(n), dim3(TAIL_T), lds_bytes, s, ch, active);
}

template <typename T, typename TC>
void launch_bmg_post_coarse(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, int inner,
                            hipStream_t s) {
    hipLaunchKernelGGL((kbm_post_coarse<TC, T>), dim3(njobs), dim3(CoarseTile::NT), 0, s, ch, jobs, active, inner);
}

template <typename T, typename TC>
void launch_bmg_mu4(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, int group, hipStream_t s) {
    if (group == 0)
        hipLaunchKernelGGL((kbm_mu4_0<T, TC>), dim3(njobs), dim3(MU_TX * MU_TY / 4), 0, s, ch, jobs);
    else
        hipLaunchKernelGGL((kbm_mu4_C<TC, T>), dim3(njobs), dim3(MU_TX * MU_TY / 4), 0, s, ch, jobs);
}

template <typename T, typename TC>
void launch_bmg_decide(const MgChan<T, TC>* ch, int n, unsigned long long* res, int* active, int* cycles, int* counts,
                       double floor_factor, const unsigned long long* rel_scale, double rel_tol, hipStream_t s) {
    hipLaunchKernelGGL((kbm_decide<T, TC>), dim3(1), dim3(BMG_DECIDE_T), 0, s, ch, n, res, active, cycles, counts,
                       floor_factor, rel_scale, rel_tol);
}

#define FCD_POT_INSTANTIATE(T)                                                                            \
    template void launch_pot_sweep<T>(const PotLevel<T>&, T, hipStream_t);                                \
    template void launch_pot_residual<T>(const PotLevel<T>&, unsigned long long*, hipStream_t);           \
    template size_t mg_tail_lds_bytes<T>(const MgTail<T>&);                                                \
    template void launch_mg_tail<T>(const MgTail<T>&, hipStream_t);                                        \
    template void launch_psi_history<T>(T*, T*, T*, T*, int, int, int, int, hipStream_t);                  \
    template void launch_psi_history_ring<T>(T*, const T*, const T*, T*, int, int, int, int, hipStream_t);

// Multigrid transfer and smoothing kernels between a level of type T and coarse levels of
// type TC (the coarse levels are FP32 under an FP64 finest level).
#define FCD_BMG_INSTANTIATE(T, TC)                                                                            \
    template void launch_bmg_smooth_fine<T, TC>(const MgChan<T, TC>*, const MgJob*, int, const int*, int, bool,  \
                                                bool, unsigned long long*, hipStream_t);                          \
    template void launch_bmg_copy_fine<T, TC>(const MgChan<T, TC>*, const MgJob*, int, const int*, hipStream_t);  \
    template void launch_bmg_restrict_smooth<T, TC>(const MgChan<T, TC>*, const MgJob*, int, const int*, int, int, \
                                                    int, bool, hipStream_t);                                      \
    template void launch_bmg_restrict_tail<T, TC>(const MgChan<T, TC>*, const MgJob*, int, const int*, bool, int, \
                                                  bool, hipStream_t);                                             \
    template void launch_bmg_tail<T, TC>(const MgChan<T, TC>*, int, size_t, const int*, hipStream_t);            \
    template void launch_bmg_post_coarse<T, TC>(const MgChan<T, TC>*, const MgJob*, int, const int*, int,        \
                                                hipStream_t);                                                     \
    template void launch_bmg_mu4<T, TC>(const MgChan<T, TC>*, const MgJob*, int, int, hipStream_t);              \
    template void launch_bmg_decide<T, TC>(const MgChan<T, TC>*, int, unsigned long long*, int*, int*, int*,     \
                                           double, const unsigned long long*, double, hipStream_t);

#define FCD_MG_INSTANTIATE(T, TC)                                                                             \
    template void launch_mg_restrict_mu4<T, TC>(const T*, int, int, int, const MuLevels<TC>&, hipStream_t);   \
    template void launch_mg_smooth_tile<T, TC>(const PotLevel<T>&, const T*, T*, const PotLevel<TC>*, int,    \
                                               unsigned long long*, int, hipStream_t, unsigned long long*,    \
                                               unsigned*);                                                    \
    template void launch_mg_restrict_tile<T, TC>(const PotLevel<T>&, const PotLevel<TC>&, int, hipStream_t);  \
    template void launch_mg_restrict_smooth<T, TC>(const PotLevel<T>&, const PotLevel<TC>&, int, TC*, int,    \
                                                   hipStream_t);

FCD_POT_INSTANTIATE(double)
FCD_POT_INSTANTIATE(float)
FCD_MG_INSTANTIATE(double, float)
FCD_MG_INSTANTIATE(float, float)
FCD_BMG_INSTANTIATE(double, float)
FCD_BMG_INSTANTIATE(float, float)

}  // namespace fcd
