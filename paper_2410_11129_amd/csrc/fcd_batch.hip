// fcd_batch.hip -- many independent channels of uneven size stepped together: every
// kernel of the step is launched once for the whole batch over a flattened list of
// 64x4-node tiles, each tile mapped to its channel through a table.  Per-channel
// constants live in device descriptors; the potential solve is four-colour SOR with a
// per-channel convergence flag so converged channels stop relaxing.
#include <hip/hip_runtime.h>

#include "fcd_batch.hpp"
#include "fcd_device.hpp"
#include "fcd_potential.hpp"
#include "fcd_step.hpp"

namespace fcd {

constexpr int TBX = 64;
constexpr int TBY = 4;

template <typename T>
__device__ __forceinline__ bool tile_node(const BatchInst<T>& B, int lt, int tiles_x, int& i, int& j) {
    const int ty = lt / tiles_x, tx = lt - ty * tiles_x;
    i = tx * TBX + threadIdx.x;
    j = ty * TBY + threadIdx.y;
    return true;
}

template <typename T>
__global__ void __launch_bounds__(TBX* TBY) kb_phase(const BatchInst<T>* __restrict__ inst,
                                                     const int* __restrict__ tile_inst, int cur) {
    const int k = tile_inst[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    tile_node(B, blockIdx.x - B.tile0, B.tiles_x, i, j);
    if (i >= B.P.nx || j >= B.P.ny) return;
    phase_node(static_cast<const T*>(B.dist[cur]), B.phi, B.P, i, j);
}

template <typename T>
__global__ void __launch_bounds__(TBX* TBY) kb_collide_stream(const BatchInst<T>* __restrict__ inst,
                                                              const int* __restrict__ tile_inst, int cur) {
    const int k = tile_inst[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    tile_node(B, blockIdx.x - B.tile0, B.tiles_x, i, j);
    if (i >= B.P.nx || j >= B.P.ny) return;
    collide_stream_node(static_cast<const T*>(B.dist[cur]), B.dist[1 - cur], B.phi, B.L0.u, B.P, i, j);
}

template <typename T>
__global__ void __launch_bounds__(TBX* TBY) kb_sor_colour(const BatchInst<T>* __restrict__ inst,
                                                          const int* __restrict__ ctile_inst,
                                                          const int* __restrict__ active, int colour) {
    const int k = ctile_inst[blockIdx.x];
    if (!active[k]) return;
    const BatchInst<T>& B = inst[k];
    int ti, tj;
    tile_node(B, blockIdx.x - B.ctile0, B.ctiles_x, ti, tj);
    const int i = 2 * ti + (colour & 1), j = 2 * tj + (colour >> 1);
    if (i >= B.P.nx || j >= B.P.ny) return;
    relax_node(B.L0, i, j, B.omega);
}

// Per-channel max-norms of the potential residual (res[2k]) and of C psi' (res[2k+1]):
// block max, one atomicMax per block and quantity into the channel's slots.
template <typename T>
__global__ void __launch_bounds__(TBX* TBY) kb_residual(const BatchInst<T>* __restrict__ inst,
                                                        const int* __restrict__ tile_inst,
                                                        unsigned long long* __restrict__ res) {
    __shared__ double wmax[2][TBY];
    const int k = tile_inst[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    tile_node(B, blockIdx.x - B.tile0, B.tiles_x, i, j);
    double v = 0.0, sc = 0.0;
    if (i < B.P.nx && j < B.P.ny && B.has_field) {
        const MgEval<T> r = mg_eval(B.L0, i, j);
        const T c = B.L0.u[(long long)j * B.L0.pitch + i];
        v = fabs((double)(r.acc - r.C * c - r.rhs));
        sc = fabs((double)(r.C * c));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v = nan_max(v, __shfl_xor(v, off, 64));
        sc = nan_max(sc, __shfl_xor(sc, off, 64));
    }
    if (threadIdx.x == 0) {
        wmax[0][threadIdx.y] = v;
        wmax[1][threadIdx.y] = sc;
    }
    __syncthreads();
    if (threadIdx.y == 0 && threadIdx.x < 2) {
        double m = wmax[threadIdx.x][0];
        for (int w = 1; w < TBY; ++w) m = nan_max(m, wmax[threadIdx.x][w]);
        atomicMax(res + 2 * k + threadIdx.x, (unsigned long long)__double_as_longlong(m));
    }
}

// active[k] = residual above max(thr, floor * scale); counts[0] = channels still
// active, counts[1] = channels whose residual is NaN.  One thread per channel.
template <typename T>
__global__ void kb_decide(const BatchInst<T>* __restrict__ inst, const unsigned long long* __restrict__ res, int n,
                          double floor_factor, int* __restrict__ active, int* __restrict__ counts) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double r = __longlong_as_double((long long)res[2 * k]);
    const double sc = __longlong_as_double((long long)res[2 * k + 1]);
    const double thr = fmax(inst[k].thr, floor_factor * sc);
    const int a = !(r <= thr);
    active[k] = a;
    if (a) atomicAdd(counts, 1);
    if (r != r) atomicAdd(counts + 1, 1);
}

template <typename T>
__global__ void __launch_bounds__(TBX* TBY) kb_psi_history(const BatchInst<T>* __restrict__ inst,
                                                           const int* __restrict__ tile_inst, int mode) {
    const int k = tile_inst[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    tile_node(B, blockIdx.x - B.tile0, B.tiles_x, i, j);
    if (i >= B.P.nx || j >= B.P.ny || !B.has_field) return;
    const long long q = (long long)j * B.L0.pitch + i;
    const T cur = B.L0.u[q];
    if (mode == 1) B.L0.u[q] = T(2) * cur - B.prev[q];
    B.prev[q] = cur;
}

template <typename T>
__global__ void __launch_bounds__(TBX* TBY) kb_fill_psi(const BatchInst<T>* __restrict__ inst,
                                                        const int* __restrict__ tile_inst) {
    const int k = tile_inst[blockIdx.x];
    const BatchInst<T>& B = inst[k];
    int i, j;
    tile_node(B, blockIdx.x - B.tile0, B.tiles_x, i, j);
    if (i >= B.P.nx || j >= B.P.ny) return;
    B.L0.u[(long long)j * B.L0.pitch + i] = T(0);
}

// ---------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------
template <typename T>
void launch_batch_phase(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int cur, hipStream_t s) {
    hipLaunchKernelGGL(kb_phase<T>, dim3(ntiles), dim3(TBX, TBY), 0, s, inst, tile_inst, cur);
}

template <typename T>
void launch_batch_collide(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int cur, hipStream_t s) {
    hipLaunchKernelGGL(kb_collide_stream<T>, dim3(ntiles), dim3(TBX, TBY), 0, s, inst, tile_inst, cur);
}

template <typename T>
void launch_batch_sweep(const BatchInst<T>* inst, const int* ctile_inst, int nctiles, const int* active,
                        hipStream_t s) {
    for (int c = 0; c < 4; ++c)
        hipLaunchKernelGGL(kb_sor_colour<T>, dim3(nctiles), dim3(TBX, TBY), 0, s, inst, ctile_inst, active, c);
}

template <typename T>
void launch_batch_residual(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int n,
                           unsigned long long* res, int* active, int* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3((2 * n + 255) / 256), dim3(256), 0, s, res, 2LL * n, 0ULL);
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, counts, 2LL, 0);
    hipLaunchKernelGGL(kb_residual<T>, dim3(ntiles), dim3(TBX, TBY), 0, s, inst, tile_inst, res);
    const double floor_factor = 16.0 * (sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07);
    hipLaunchKernelGGL(kb_decide<T>, dim3((n + 255) / 256), dim3(256), 0, s, inst, res, n, floor_factor, active,
                       counts);
}

template <typename T>
void launch_batch_psi_history(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int mode, hipStream_t s) {
    hipLaunchKernelGGL(kb_psi_history<T>, dim3(ntiles), dim3(TBX, TBY), 0, s, inst, tile_inst, mode);
}

template <typename T>
void launch_batch_fill_psi(const BatchInst<T>* inst, const int* tile_inst, int ntiles, hipStream_t s) {
    hipLaunchKernelGGL(kb_fill_psi<T>, dim3(ntiles), dim3(TBX, TBY), 0, s, inst, tile_inst);
}

#define FCD_BATCH_INSTANTIATE(T)                                                                                 \
    template void launch_batch_phase<T>(const BatchInst<T>*, const int*, int, int, hipStream_t);               \
    template void launch_batch_collide<T>(const BatchInst<T>*, const int*, int, int, hipStream_t);             \
    template void launch_batch_sweep<T>(const BatchInst<T>*, const int*, int, const int*, hipStream_t);        \
    template void launch_batch_residual<T>(const BatchInst<T>*, const int*, int, int, unsigned long long*, int*, \
                                           int*, hipStream_t);                                                   \
    template void launch_batch_psi_history<T>(const BatchInst<T>*, const int*, int, int, hipStream_t);         \
    template void launch_batch_fill_psi<T>(const BatchInst<T>*, const int*, int, hipStream_t);

FCD_BATCH_INSTANTIATE(double)
FCD_BATCH_INSTANTIATE(float)

}  // namespace fcd
