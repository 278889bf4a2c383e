// fcd_batch.hip -- many independent channels of uneven size stepped together: every
// kernel of the step is launched once for the whole batch over a flattened list of
// 64 x TY-node tiles, each tile mapped to its channel through a table (one table per
// tile shape; the shape is chosen by the batch autotuner).  Per-channel constants live
// in device descriptors.  The potential solve is four-colour SOR; every `check` sweeps a
// residual test and a decision update per-channel activity flags on the device (in fused
// schedules the test rides on a sweep launch and the decision on the next one), so
// converged channels stop relaxing and the result does not depend on how the host
// groups the sweeps into launches or graphs.
#include <hip/hip_runtime.h>

#include "fcd_batch.hpp"
#include "fcd_device.hpp"
#include "fcd_potential.hpp"
#include "fcd_step.hpp"

namespace fcd {

constexpr int TBX = 64;

template <int TY>
constexpr int shape_index() {
    return TY == 1 ? 0 : TY == 2 ? 1 : TY == 4 ? 2 : 3;
}

template <typename T, int TY>
__device__ __forceinline__ void tile_node(const BatchInst<T>& B, int tile, bool colour_grid, int& i, int& j) {
    constexpr int S = shape_index<TY>();
    const int lt = tile - (colour_grid ? B.ctile0[S] : B.tile0[S]);
    const int tx = colour_grid ? B.ctiles_x[S] : B.tiles_x[S];
    const int ty = lt / tx, txi = lt - ty * tx;
    i = txi * TBX + threadIdx.x;
    j = ty * TY + threadIdx.y;
}

template <typename T, int SX>
__device__ __forceinline__ Nb9<T> tile_nb(const T (*t)[SX], int lx, int ly) {
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

template <typename T, int TY>
__global__ void __launch_bounds__(TBX* TY) kb_phase(const BatchInst<T>* __restrict__ inst,
                                                    const int* __restrict__ tile_inst, int cur) {
    const BatchInst<T>& B = inst[tile_inst[blockIdx.x]];
    int i, j;
    tile_node<T, TY>(B, blockIdx.x, false, i, j);
    if (i >= B.P.nx || j >= B.P.ny) return;
    phase_node(static_cast<const T*>(B.dist[cur]), B.phi, B.P, i, j);
}

// Fused collide-and-stream of one tile: the phi1, phi2 and psi' neighbourhoods are staged
// in LDS (the tile plus a one-node ring; columns wrap, rows beyond the walls repeat the
// edge row for phi and are zero for psi', as the global neighbourhood loads give them),
// then each node runs the same per-node update as the single-channel kernel.
template <typename T, int TY>
__global__ void __launch_bounds__(TBX* TY) kb_collide_stream(const BatchInst<T>* __restrict__ inst,
                                                             const int* __restrict__ tile_inst, int cur) {
    constexpr int SX = TBX + 2, SY = TY + 2, S = shape_index<TY>();
    __shared__ T t1[SY][SX], t2[SY][SX], tp[SY][SX];
    const BatchInst<T>& B = inst[tile_inst[blockIdx.x]];
    const int lt = blockIdx.x - B.tile0[S], tx = B.tiles_x[S];
    const int ty = lt / tx, i0 = (lt - ty * tx) * TBX, j0 = ty * TY;
    const int nx = B.P.nx, ny = B.P.ny;
    const long long pitch = B.P.pitch, plane = B.P.plane;
    const T* __restrict__ phi = B.phi;
    const T* __restrict__ psi = B.L0.u;
    for (int q = threadIdx.y * TBX + threadIdx.x; q < SX * SY; q += TBX * TY) {
        const int ly = q / SX, lx = q - ly * SX;
        int i = i0 + lx - 1;
        while (i < 0) i += nx;
        while (i >= nx) i -= nx;
        const int jr = j0 + ly - 1;
        const int j = jr < 0 ? 0 : (jr >= ny ? ny - 1 : jr);
        const long long k = (long long)j * pitch + i;
        t1[ly][lx] = phi[k];
        t2[ly][lx] = phi[plane + k];
        tp[ly][lx] = (jr < 0 || jr >= ny) ? T(0) : psi[k];
    }
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const int lx = threadIdx.x + 1, ly = threadIdx.y + 1;
    collide_stream_nb(static_cast<const T*>(B.dist[cur]), B.dist[1 - cur], tile_nb<T, SX>(t1, lx, ly),
                      tile_nb<T, SX>(t2, lx, ly), tile_nb<T, SX>(tp, lx, ly), B.P, i, j, B.div);
}

template <typename T, int TY>
__global__ void __launch_bounds__(TBX* TY) kb_sor_colour(const BatchInst<T>* __restrict__ inst,
                                                         const int* __restrict__ ctile_inst,
                                                         const int* __restrict__ active, int colour) {
    const int k = ctile_inst[blockIdx.x];
    if (!active[k]) return;
    const BatchInst<T>& B = inst[k];
    int ti, tj;
    tile_node<T, TY>(B, blockIdx.x, true, ti, tj);
    const int i = 2 * ti + (colour & 1), j = 2 * tj + (colour >> 1);
    if (i >= B.P.nx || j >= B.P.ny) return;
    relax_node(B.L0, i, j, B.omega);
}

// Fused sweeps: NS four-colour SOR sweeps of one 64 x 32 tile in one launch.  The tile
// and a halo of H = 4 NS + 1 nodes are staged in LDS (columns wrapped, rows clamped to
// the channel).  Colour phase p = 0 .. 4 NS - 1 (colour p mod 4) updates the nodes of
// its colour that lie within 4 NS - p nodes of the tile, so every value a phase reads
// has already received all earlier phases' updates, and the tile and its first halo ring
// end holding exactly what NS sweeps with one launch per colour produce (same per-node
// arithmetic).  The halo work is repeated by the neighbouring tiles that own it.  Input
// and output are separate planes, since a tile's halo is other tiles' output.  With res
// set, the launch also reduces the tile's residual and |C psi'| max-norms into the
// channel's slots, as the separate residual pass does.
__device__ __forceinline__ int fs_wrap(int i, int nx) {
    while (i < 0) i += nx;
    while (i >= nx) i -= nx;
    return i;
}

// LDS layout of a fused-sweep tile: the even and odd columns of every row are stored in
// two separate planes (node (lx, ly) at plane lx & 1, row ly, element lx >> 1), so the
// same-colour nodes of neighbouring lanes, and each of their neighbours, are consecutive
// elements; an element holds a node's potential and mu_r together (one 2-value LDS read
// per neighbour).  In FP32 the second plane starts half the banks after the first, so a
// row read across both parities is conflict-free as well.
template <int NS>
struct FusedLds {
    static constexpr int H = 4 * NS + 1, HX = FUSED_X + 2 * H, HY = FUSED_Y + 2 * H, HXH = HX / 2;
    static constexpr int PS0 = HY * HXH, PS = PS0 + (24 - PS0 % 16) % 16, N = 2 * PS;
    static_assert(HX % 2 == 0, "even halo row");
    static __device__ __forceinline__ int at(int lx, int ly) { return (lx & 1) * PS + ly * HXH + (lx >> 1); }
};

// A staged node: potential and mu_r.
template <typename T>
struct alignas(2 * sizeof(T)) UM {
    T u, m;
};

// The operator at a staged node: c its element, o the element of its east neighbour (the
// west one is o - 1, in the same plane), row the elements per row; rows beyond the walls
// read the edge row itself, as the clamped global loads do.
template <typename T, bool HF>
__device__ __forceinline__ MgEval<T> fs_eval(const PotLevel<T>& L, const UM<T>* sv, const T* sf, int c,
                                             int o, int row, int j) {
    const int dn = j == L.ny - 1 ? 0 : row, ds = j == 0 ? 0 : -row;
    Nb9<T> m, u;
    const UM<T> vc = sv[c], ve = sv[o], vw = sv[o - 1], vn = sv[c + dn], vs = sv[c + ds];
    const UM<T> vne = sv[o + dn], vnw = sv[o - 1 + dn], vsw = sv[o - 1 + ds], vse = sv[o + ds];
    m.c = vc.m;
    m.e = ve.m;
    m.w = vw.m;
    m.n = vn.m;
    m.s = vs.m;
    m.ne = vne.m;
    m.nw = vnw.m;
    m.sw = vsw.m;
    m.se = vse.m;
    u.c = vc.u;
    u.e = ve.u;
    u.w = vw.u;
    u.n = vn.u;
    u.s = vs.u;
    u.ne = vne.u;
    u.nw = vnw.u;
    u.sw = vsw.u;
    u.se = vse.u;
    return mg_eval_nb(L, m, u, j, HF ? sf[c] : T(0));
}

// Colour phase P of the fused sweeps: colour (cx, cy) of global parity (local column lx
// has the parity of lx + H, since the tile origin is even), nodes with lx in
// [H - R, H + 64 + R), ly likewise, R = 4 NS - P, rows outside the channel left out;
// the phase's nodes are dealt to the block's threads row-major, so few lanes idle.
template <typename T, int NS, bool HF, int P>
__device__ __forceinline__ void fs_phase(const PotLevel<T>& L, UM<T>* sv, const T* sf, int j0, T omega) {
    using F = FusedLds<NS>;
    constexpr int H = F::H, R = 4 * NS - P;
    constexpr int px = ((P & 1) + H) & 1, py = (((P >> 1) & 1) + H) & 1;
    constexpr int a0 = (H - R - px + 1) >> 1, na = ((H + FUSED_X + R - px + 1) >> 1) - a0;
    constexpr int b0 = (H - R - py + 1) >> 1, nb = ((H + FUSED_Y + R - py + 1) >> 1) - b0;
    // only the rows inside the channel: 0 <= j0 - H + ly < ny
    const int lo = max(0, ((H - j0 - py + 1) >> 1) - b0), hi = min(nb, ((L.ny - 1 + H - j0 - py) >> 1) - b0 + 1);
    for (int q = lo * na + threadIdx.x; q < hi * na; q += FUSED_NT) {
        const int bq = q / na, aq = q - bq * na;
        const int ly = 2 * (b0 + bq) + py;
        const int j = j0 - H + ly;
        const int c = px * F::PS + ly * F::HXH + a0 + aq;       // column 2 (a0 + aq) + px
        const int o = (1 - px) * F::PS + ly * F::HXH + a0 + aq + px;  // its east neighbour
        const MgEval<T> r = fs_eval<T, HF>(L, sv, sf, c, o, F::HXH, j);
        sv[c].u = sor_value(r, sv[c].u, omega);
    }
    __syncthreads();
    if constexpr (P + 1 < 4 * NS) fs_phase<T, NS, HF, P + 1>(L, sv, sf, j0, omega);
}

// Whether channel k stays active after a test: its residual is above
// max(thr, floor * |C psi'|) (NaN stays active); thr = rel_tol * scale[k] with scale
// set, else the descriptor's.
template <typename T>
__device__ __forceinline__ int channel_active(const BatchInst<T>* inst, const unsigned long long* res, int k,
                                              const unsigned long long* scale, double rel_tol,
                                              double floor_factor) {
    const double r = __longlong_as_double((long long)res[2 * k]);
    const double sc = __longlong_as_double((long long)res[2 * k + 1]);
    const double thr = scale ? rel_tol * __longlong_as_double((long long)scale[k]) : inst[k].thr;
    return !(r <= fmax(thr, floor_factor * sc));
}

template <typename T>
constexpr double decide_floor() {
    return 16.0 * (sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07);
}

// LATE: the variant for the four-sweep launches late in a solve, when few tiles are
// active: a fixed grid strides over the list of active tiles, and a channel that stops
// on odd parity is copied back to its plane.  The other variants take one list entry
// per block (the grid covers every tile; blocks past the list's end return at once),
// which holds fewer registers than the strided loop, and carry no copy code.
template <typename T, int NS, bool HF, bool LATE>
__global__ void __launch_bounds__(FUSED_NT) kb_sor_fused(const BatchInst<T>* __restrict__ inst,
                                                         const int* __restrict__ stile_inst,
                                                         const int* __restrict__ slist, const int* __restrict__ scount,
                                                         const int* __restrict__ act_in, int* __restrict__ act_out,
                                                         int parity, unsigned long long* __restrict__ res,
                                                         BatchDecide dec) {
    using F = FusedLds<NS>;
    constexpr int H = F::H, HX = F::HX, HN = HX * F::HY, NT = FUSED_NT;
    __shared__ UM<T> sv[F::N];
    __shared__ T sf[HF ? F::N : 1];
    __shared__ double wmax[2][NT / 64];
    // list entries: the tiles of the channels that were active at the last decision
    // kernel (channels stopped since then are skipped tile by tile)
    const int count = *scount;
    for (int b = blockIdx.x; b < count; b = LATE ? b + (int)gridDim.x : count) {
        const int tile = slist[b];
        const int k = stile_inst[tile];
        const BatchInst<T>& B = inst[k];
        // the flags of a deciding launch go to the other buffer, so every block of the
        // channel reads the flag from before the decision
        const int was = act_in[k];
        int act = was;
        if (dec.res) {
            if (act) act = channel_active(inst, dec.res, k, dec.scale, dec.rel_tol, decide_floor<T>());
            if (tile == B.stile0 && threadIdx.x == 0) {
                if (was) dec.sweeps[k] += dec.add;
                act_out[k] = act;
                dec.clear[2 * k] = 0ULL;
                dec.clear[2 * k + 1] = 0ULL;
            }
        }
        const PotLevel<T> L = B.L0;
        const T* __restrict__ uin = parity ? B.alt : L.u;
        T* __restrict__ uout = parity ? L.u : B.alt;
        const int lt = tile - B.stile0, ty = lt / B.stiles_x, tx = lt - ty * B.stiles_x;
        const int i0 = tx * FUSED_X, j0 = ty * FUSED_Y;
        if (!act) {  // uniform over the block
            // a channel stopped by this launch's decision whose last result is in the
            // second plane (odd parity): its tiles move it back to the potential's plane
            if (LATE && dec.res && was && parity)
                for (int q = threadIdx.x; q < FUSED_X * FUSED_Y; q += NT) {
                    const int i = i0 + (q & (FUSED_X - 1)), j = j0 + q / FUSED_X;
                    if (i < L.nx && j < L.ny) uout[(long long)j * L.pitch + i] = uin[(long long)j * L.pitch + i];
                }
            continue;
        }
        // all loads into registers first, then the LDS stores, so that the loads of a
        // thread are in flight together
        constexpr int LPER = (HN + NT - 1) / NT;
        T uv[LPER], mv[LPER], fv[HF ? LPER : 1];
#pragma unroll
        for (int r = 0; r < LPER; ++r) {
            const int q = threadIdx.x + r * NT;
            if (q < HN) {
                const int ly = q / HX, lx = q - ly * HX;
                const int i = fs_wrap(i0 - H + lx, L.nx);
                int j = j0 - H + ly;
                j = j < 0 ? 0 : (j >= L.ny ? L.ny - 1 : j);
                const long long g = (long long)j * L.pitch + i;
                uv[r] = uin[g];
                mv[r] = L.mu[g];
                if (HF) fv[HF ? r : 0] = L.f[g];
            }
        }
#pragma unroll
        for (int r = 0; r < LPER; ++r) {
            const int q = threadIdx.x + r * NT;
            if (q < HN) {
                const int ly = q / HX, lx = q - ly * HX, w = F::at(lx, ly);
                sv[w] = UM<T>{uv[r], mv[r]};
                if (HF) sf[HF ? w : 0] = fv[HF ? r : 0];
            }
        }
        __syncthreads();
        fs_phase<T, NS, HF, 0>(L, sv, sf, j0, B.omega);
        double v = 0.0, sc = 0.0;
        for (int q = threadIdx.x; q < FUSED_X * FUSED_Y; q += NT) {
            const int ly = q / FUSED_X, lx = q - ly * FUSED_X;
            const int i = i0 + lx, j = j0 + ly;
            if (i < L.nx && j < L.ny) {
                const int c = F::at(H + lx, H + ly);
                uout[(long long)j * L.pitch + i] = sv[c].u;
                if (res && B.has_field) {
                    const MgEval<T> r = fs_eval<T, HF>(L, sv, sf, c, F::at(H + lx + 1, H + ly), F::HXH, j);
                    v = nan_max(v, residual_abs(r, sv[c].u));
                    sc = nan_max(sc, fabs((double)(r.C * sv[c].u)));
                }
            }
        }
        if (res) {  // uniform
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
                double mx = wmax[threadIdx.x][0];
                for (int w = 1; w < NT / 64; ++w) mx = nan_max(mx, wmax[threadIdx.x][w]);
                atomicMax(res + 2 * k + threadIdx.x, (unsigned long long)__double_as_longlong(mx));
            }
        }
        __syncthreads();  // the next tile reuses the LDS arrays
    }
}

// Per-channel max-norms of the potential residual (res[2k]) and of C psi' (res[2k+1])
// of the channels still active, over the 64 x 32 fused-sweep tiles (whatever the
// schedule's tile shape): each of the 512 threads takes four nodes, block max, one
// atomicMax per block and quantity (few blocks per channel, so little contention).
template <typename T>
__global__ void __launch_bounds__(FUSED_NT) kb_residual(const BatchInst<T>* __restrict__ inst,
                                                       const int* __restrict__ stile_inst,
                                                       const int* __restrict__ active,
                                                       unsigned long long* __restrict__ res) {
    __shared__ double wmax[2][FUSED_NT / 64];
    const int k = stile_inst[blockIdx.x];
    if (!active[k]) return;  // uniform over the block
    const BatchInst<T>& B = inst[k];
    const int lt = blockIdx.x - B.stile0, ty = lt / B.stiles_x, tx = lt - ty * B.stiles_x;
    double v = 0.0, sc = 0.0;
    if (B.has_field)
        for (int q = threadIdx.x; q < FUSED_X * FUSED_Y; q += FUSED_NT) {
            const int i = tx * FUSED_X + (q & (FUSED_X - 1)), j = ty * FUSED_Y + q / FUSED_X;
            if (i < B.P.nx && j < B.P.ny) {
                const MgEval<T> r = mg_eval(B.L0, i, j);
                const T c = B.L0.u[(long long)j * B.L0.pitch + i];
                v = nan_max(v, residual_abs(r, c));
                sc = nan_max(sc, fabs((double)(r.C * c)));
            }
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
        for (int w = 1; w < FUSED_NT / 64; ++w) m = nan_max(m, wmax[threadIdx.x][w]);
        atomicMax(res + 2 * k + threadIdx.x, (unsigned long long)__double_as_longlong(m));
    }
}

// One block: a channel stays active while its residual is above max(thr, floor * scale)
// (an inactive channel stays inactive for the rest of the solve); the residual slots are
// cleared for the next test, and so are those of also_clear and also_clear2 when set;
// the flags are read from buffer `cur` of the two (active[cur * n + k]) and written to
// both; counts[0] = channels still active, counts[1] = channels whose residual is NaN;
// sweeps[k] grows by `add` (the sweeps since the previous test) for every channel
// active on entry.
constexpr int DECIDE_T = 256;

template <typename T>
__global__ void __launch_bounds__(DECIDE_T) kb_decide(const BatchInst<T>* __restrict__ inst,
                                                      unsigned long long* __restrict__ res,
                                                      unsigned long long* __restrict__ also_clear,
                                                      unsigned long long* __restrict__ also_clear2, int n,
                                                      int* __restrict__ active, int cur, int* __restrict__ counts,
                                                      const unsigned long long* __restrict__ scale, double rel_tol,
                                                      int* __restrict__ sweeps, int add, int* __restrict__ slist,
                                                      int* __restrict__ scount) {
    __shared__ int cnt[2][DECIDE_T / 64];
    __shared__ int scan[DECIDE_T];
    int a_sum = 0, nan_sum = 0;
    for (int k = threadIdx.x; k < n; k += DECIDE_T) {
        if (also_clear) {
            also_clear[2 * k] = 0ULL;
            also_clear[2 * k + 1] = 0ULL;
        }
        if (also_clear2) {
            also_clear2[2 * k] = 0ULL;
            also_clear2[2 * k + 1] = 0ULL;
        }
        int a = 0;
        if (active[cur * n + k]) {
            sweeps[k] += add;
            const double r = __longlong_as_double((long long)res[2 * k]);
            a = channel_active(inst, res, k, scale, rel_tol, decide_floor<T>());
            a_sum += a;
            nan_sum += r != r;
            res[2 * k] = 0ULL;
            res[2 * k + 1] = 0ULL;
        }
        active[k] = a;  // both flag buffers
        active[n + k] = a;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a_sum += __shfl_xor(a_sum, off, 64);
        nan_sum += __shfl_xor(nan_sum, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        cnt[0][threadIdx.x >> 6] = a_sum;
        cnt[1][threadIdx.x >> 6] = nan_sum;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        int s = 0;
        for (int w = 0; w < DECIDE_T / 64; ++w) s += cnt[threadIdx.x][w];
        counts[threadIdx.x] = s;
    }
    // the fused-sweep tiles of the channels still active, in channel order (an exclusive
    // scan of their tile counts, DECIDE_T channels at a time); the barrier makes this
    // block's stores to active visible to all its threads
    __syncthreads();
    int base = 0;
    for (int c0 = 0; c0 < n; c0 += DECIDE_T) {
        const int k = c0 + threadIdx.x;
        int m = 0;
        if (k < n && active[k]) m = inst[k].stiles_x * ((inst[k].P.ny + FUSED_Y - 1) / FUSED_Y);
        scan[threadIdx.x] = m;
        __syncthreads();
        for (int off = 1; off < DECIDE_T; off <<= 1) {  // inclusive scan (Hillis-Steele)
            const int add_in = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
            __syncthreads();
            scan[threadIdx.x] += add_in;
            __syncthreads();
        }
        const int first = base + scan[threadIdx.x] - m;
        for (int q = 0; q < m; ++q) slist[first + q] = inst[k].stile0 + q;
        base += scan[DECIDE_T - 1];
        __syncthreads();  // scan[] is rewritten by the next chunk
    }
    if (threadIdx.x == 0) *scount = base;
}

template <typename T, int TY>
__global__ void __launch_bounds__(TBX* TY) kb_psi_history(const BatchInst<T>* __restrict__ inst,
                                                          const int* __restrict__ tile_inst, int mode) {
    const BatchInst<T>& B = inst[tile_inst[blockIdx.x]];
    int i, j;
    tile_node<T, TY>(B, blockIdx.x, false, i, j);
    if (i >= B.P.nx || j >= B.P.ny || !B.has_field) return;
    const long long q = (long long)j * B.L0.pitch + i;
    const T cur = B.L0.u[q];
    const T p1 = B.prev[q];
    if (mode == 1) B.L0.u[q] = T(2) * cur - p1;
    if (mode == 2) B.L0.u[q] = T(3) * (cur - p1) + B.prev2[q];
    if (mode == 3) B.L0.u[q] = T(4) * (cur + B.prev2[q]) - T(6) * p1 - B.prev3[q];
    if (B.prev3) B.prev3[q] = B.prev2[q];
    if (B.prev2) B.prev2[q] = p1;
    B.prev[q] = cur;
}

template <typename T, int TY>
__global__ void __launch_bounds__(TBX* TY) kb_fill_psi(const BatchInst<T>* __restrict__ inst,
                                                       const int* __restrict__ tile_inst) {
    const BatchInst<T>& B = inst[tile_inst[blockIdx.x]];
    int i, j;
    tile_node<T, TY>(B, blockIdx.x, false, i, j);
    if (i >= B.P.nx || j >= B.P.ny) return;
    B.L0.u[(long long)j * B.L0.pitch + i] = T(0);
}

// ---------------------------------------------------------------------------------
// Launchers: `shape` indexes the tile rows TY = 1, 2, 4, 8.
// ---------------------------------------------------------------------------------
#define FCD_SHAPE_SWITCH(shape, CALL) \
    switch (shape) {                  \
        case 0: CALL(1); break;       \
        case 1: CALL(2); break;       \
        case 2: CALL(4); break;       \
        default: CALL(8); break;      \
    }

template <typename T>
void launch_batch_phase(const BatchInst<T>* inst, const BatchTiles& t, int cur, hipStream_t s) {
#define C_(TY) hipLaunchKernelGGL((kb_phase<T, TY>), dim3(t.ntiles), dim3(TBX, TY), 0, s, inst, t.tiles, cur)
    FCD_SHAPE_SWITCH(t.shape, C_)
#undef C_
}

template <typename T>
void launch_batch_collide(const BatchInst<T>* inst, const BatchTiles& t, int cur, hipStream_t s) {
#define C_(TY) \
    hipLaunchKernelGGL((kb_collide_stream<T, TY>), dim3(t.ntiles), dim3(TBX, TY), 0, s, inst, t.tiles, cur)
    FCD_SHAPE_SWITCH(t.shape, C_)
#undef C_
}

template <typename T>
void launch_batch_sweep(const BatchInst<T>* inst, const BatchTiles& t, const int* active, hipStream_t s) {
    for (int c = 0; c < 4; ++c) {
#define C_(TY) \
    hipLaunchKernelGGL((kb_sor_colour<T, TY>), dim3(t.nctiles), dim3(TBX, TY), 0, s, inst, t.ctiles, active, c)
        FCD_SHAPE_SWITCH(t.shape, C_)
#undef C_
    }
}

template <typename T>
void launch_batch_sweep_fused(const BatchInst<T>* inst, const BatchTiles& t, const int* act_in, int* act_out,
                              int parity, bool rhs_plane, unsigned long long* res, const BatchDecide& dec,
                              hipStream_t s) {
#define C_(NS, HF, LATE)                                                                                    \
    hipLaunchKernelGGL((kb_sor_fused<T, NS, HF, LATE>), dim3(LATE ? t.sgrid : std::max(1, t.nstiles)),          \
                       dim3(FUSED_NT), 0, s, inst, t.stiles, t.slist, t.scount, act_in, act_out, parity, res, dec)
    // a decision meets odd parity (an odd number of launches per test interval) only
    // with four sweeps per launch
    if (t.fused == 1) {
        if (rhs_plane) C_(1, true, false); else C_(1, false, false);
    } else if (t.fused == 2) {
        if (rhs_plane) C_(2, true, false); else C_(2, false, false);
    } else {
        if (rhs_plane) C_(4, true, true); else C_(4, false, true);
    }
#undef C_
}

template <typename T>
void launch_batch_check(const BatchInst<T>* inst, const BatchTiles& t, int n, unsigned long long* res,
                        int* active, int* counts, const unsigned long long* scale, double rel_tol, int* sweeps,
                        int add, hipStream_t s) {
    if (t.nstiles > 0)
        hipLaunchKernelGGL(kb_residual<T>, dim3(t.nstiles), dim3(FUSED_NT), 0, s, inst, t.stiles, active, res);
    launch_batch_decide<T>(inst, t, n, res, nullptr, nullptr, active, 0, counts, scale, rel_tol, sweeps, add, s);
}

template <typename T>
void launch_batch_decide(const BatchInst<T>* inst, const BatchTiles& t, int n, unsigned long long* res,
                         unsigned long long* also_clear, unsigned long long* also_clear2, int* active, int cur,
                         int* counts, const unsigned long long* scale, double rel_tol, int* sweeps, int add,
                         hipStream_t s) {
    hipLaunchKernelGGL(kb_decide<T>, dim3(1), dim3(DECIDE_T), 0, s, inst, res, also_clear, also_clear2, n, active, cur,
                       counts, scale, rel_tol, sweeps, add, t.slist, t.scount);
}

template <typename T>
void launch_batch_psi_history(const BatchInst<T>* inst, const BatchTiles& t, int mode, hipStream_t s) {
#define C_(TY) \
    hipLaunchKernelGGL((kb_psi_history<T, TY>), dim3(t.ntiles), dim3(TBX, TY), 0, s, inst, t.tiles, mode)
    FCD_SHAPE_SWITCH(t.shape, C_)
#undef C_
}

template <typename T>
void launch_batch_fill_psi(const BatchInst<T>* inst, const BatchTiles& t, hipStream_t s) {
#define C_(TY) hipLaunchKernelGGL((kb_fill_psi<T, TY>), dim3(t.ntiles), dim3(TBX, TY), 0, s, inst, t.tiles)
    FCD_SHAPE_SWITCH(t.shape, C_)
#undef C_
}

#define FCD_BATCH_INSTANTIATE(T)                                                                               \
    template void launch_batch_phase<T>(const BatchInst<T>*, const BatchTiles&, int, hipStream_t);           \
    template void launch_batch_collide<T>(const BatchInst<T>*, const BatchTiles&, int, hipStream_t);         \
    template void launch_batch_sweep<T>(const BatchInst<T>*, const BatchTiles&, const int*, hipStream_t);    \
    template void launch_batch_sweep_fused<T>(const BatchInst<T>*, const BatchTiles&, const int*, int*, int, \
                                              bool, unsigned long long*, const BatchDecide&, hipStream_t);   \
    template void launch_batch_decide<T>(const BatchInst<T>*, const BatchTiles&, int, unsigned long long*,   \
                                         unsigned long long*, unsigned long long*, int*, int, int*,          \
                                         const unsigned long long*, double, int*, int, hipStream_t);         \
    template void launch_batch_check<T>(const BatchInst<T>*, const BatchTiles&, int, unsigned long long*,    \
                                        int*, int*, const unsigned long long*, double, int*, int,            \
                                        hipStream_t);                                                        \
    template void launch_batch_psi_history<T>(const BatchInst<T>*, const BatchTiles&, int, hipStream_t);     \
    template void launch_batch_fill_psi<T>(const BatchInst<T>*, const BatchTiles&, hipStream_t);

FCD_BATCH_INSTANTIATE(double)
FCD_BATCH_INSTANTIATE(float)

}  // namespace fcd
