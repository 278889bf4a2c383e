// fcd_extent.hip -- shape diagnostics of the paper on the device: the extent-based
// deformation index of Eq. 42, and the breakup probe further below.  Eq. 42:
// T = (l_y - l_x) / (l_y + l_x) of the outer droplet (w = phi1 + phi2) and the inner one
// (w = phi1), the interface at w = 1/2.  l_y: over the columns, the largest extent of the
// longest run of rows with w >= 1/2, between the linearly interpolated crossings below and
// above it (a run reaching a wall row ends at the wall, half a node beyond the row); l_x:
// the longest run with w >= 1/2 of the centreline profile (the middle row, or the mean of
// the two middle rows when ny is even), periodic in x, between its interpolated crossings
// (nx when the run closes on itself).  One thread per column for l_y (block max, one
// atomicMax per block on the bit pattern of a non-negative double), one thread per droplet
// for the centreline scan.
#include <hip/hip_runtime.h>

#include "fcd_device.hpp"
#include "fcd_kernels.hpp"

namespace fcd {

namespace {

constexpr int EXT_T = 64;

// w of the outer (d = 0) or inner (d = 1) droplet at plane offset k, in double
template <typename T>
__device__ __forceinline__ double ext_w(const T* __restrict__ phi, long long plane, long long k, int d) {
    return d == 0 ? (double)phi[k] + (double)phi[plane + k] : (double)phi[k];
}

// Fraction of the gap from the node below 1/2 (value a) towards the node at or above
// it (value b) where the linear interpolant crosses 1/2.
__device__ __forceinline__ double ext_cross(double a, double b) { return (0.5 - a) / (b - a); }

template <typename T>
__global__ void __launch_bounds__(EXT_T) k_extent_cols(const T* __restrict__ phi, StepConst<T> P,
                                                       unsigned long long* __restrict__ ly) {
    const int i = blockIdx.x * EXT_T + threadIdx.x;
    double best[2] = {0.0, 0.0};
    if (i < P.nx) {
        for (int d = 0; d < 2; ++d) {
            double prev = -1.0;  // w of the row below (none at the wall)
            double lo = 0.0;
            bool in = false;
            for (int j = 0; j < P.ny; ++j) {
                const double w = ext_w(phi, P.plane, (long long)j * P.pitch + i, d);
                if (w >= 0.5 && !in) {  // a run starts at row j
                    in = true;
                    lo = j == 0 ? -0.5 : (j - 1) + ext_cross(prev, w);
                } else if (w < 0.5 && in) {  // the run ended at row j - 1
                    in = false;
                    const double hi = j - ext_cross(w, prev);
                    best[d] = fmax(best[d], hi - lo);
                }
                prev = w;
            }
            if (in) best[d] = fmax(best[d], (P.ny - 0.5) - lo);
        }
    }
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        double v = best[d];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if (threadIdx.x == 0) atomicMax(ly + d, (unsigned long long)__double_as_longlong(v));
    }
}

template <typename T>
__device__ double centre_value(const T* __restrict__ phi, const StepConst<T>& P, int i, int d) {
    const int jm = P.ny / 2;
    if (P.ny % 2) return ext_w(phi, P.plane, (long long)jm * P.pitch + i, d);
    return 0.5 * (ext_w(phi, P.plane, (long long)(jm - 1) * P.pitch + i, d) +
                  ext_w(phi, P.plane, (long long)jm * P.pitch + i, d));
}

// Threads 0 and 1: the outer and inner droplets' centreline extents.  The scan starts at a
// node below 1/2 and walks once around the period, so no run is cut by the seam.
template <typename T>
__global__ void k_extent_centre(const T* __restrict__ phi, StepConst<T> P, double* __restrict__ lx) {
    const int d = threadIdx.x;
    if (d > 1) return;
    const int nx = P.nx;
    int s = -1;
    for (int i = 0; i < nx && s < 0; ++i)
        if (centre_value(phi, P, i, d) < 0.5) s = i;
    if (s < 0) {
        lx[d] = (double)nx;
        return;
    }
    double best = 0.0, start = 0.0, prev = centre_value(phi, P, s, d);
    bool in = false;
    for (int t = 1; t <= nx; ++t) {
        const int i = s + t < nx ? s + t : s + t - nx;
        const double w = centre_value(phi, P, i, d);
        if (w >= 0.5 && !in) {
            in = true;
            start = (t - 1) + ext_cross(prev, w);  // positions counted from node s
        } else if (w < 0.5 && in) {
            in = false;
            best = fmax(best, t - ext_cross(w, prev) - start);
        }
        prev = w;
    }
    lx[d] = best;  // the walk ends on node s, below 1/2: every run has closed
}

// Breakup probe (Sec. 2.5: breakup is the inner droplet touching the shell's interface):
// a contact node is a core node (phi1 >= 1/2) with a nine-point neighbour in the carrier
// (phi3 >= 1/2; columns periodic, no neighbours beyond the walls).  One block per row
// reduces, in a fixed order, the row's contact count, sum of y, sums of cos and sin of
// 2 pi x / nx over the contact nodes, and the phi1 + phi2 weighted cos and sin sums of the
// outer droplet; a single block then adds the rows in order.
constexpr int BRK_T = 256;

template <typename T>
__global__ void __launch_bounds__(BRK_T) k_breakup_rows(const T* __restrict__ phi, StepConst<T> P,
                                                        double* __restrict__ rows) {
    __shared__ double part[6][BRK_T / 64];
    const int j = blockIdx.x;
    const double two_pi = 6.283185307179586;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < P.nx; i += BRK_T) {
        const long long k = (long long)j * P.pitch + i;
        const double p1 = (double)phi[k], p2 = (double)phi[P.plane + k];
        const double th = two_pi * i / P.nx, c = cos(th), s = sin(th);
        acc[4] += (p1 + p2) * c;
        acc[5] += (p1 + p2) * s;
        if (p1 < 0.5) continue;
        bool touch = false;
        for (int dj = -1; dj <= 1; ++dj) {
            const int jj = j + dj;
            if (jj < 0 || jj >= P.ny) continue;
            for (int di = -1; di <= 1; ++di) {
                if (di == 0 && dj == 0) continue;
                int ii = i + di;
                ii = ii < 0 ? ii + P.nx : (ii >= P.nx ? ii - P.nx : ii);
                const long long kk = (long long)jj * P.pitch + ii;
                touch = touch || (1.0 - (double)phi[kk] - (double)phi[P.plane + kk] >= 0.5);
            }
        }
        if (!touch) continue;
        acc[0] += 1.0;
        acc[1] += j;
        acc[2] += c;
        acc[3] += s;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) part[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0.0;
        for (int w = 0; w < BRK_T / 64; ++w) v += part[threadIdx.x][w];
        rows[(long long)j * 8 + threadIdx.x] = v;
    }
}

__global__ void k_breakup_final(const double* __restrict__ rows, int ny, double* __restrict__ sums) {
    const int q = threadIdx.x;
    if (q >= 6) return;
    double v = 0.0;
    for (int j = 0; j < ny; ++j) v += rows[(long long)j * 8 + q];
    sums[q] = v;
}

}  // namespace

template <typename T>
void launch_breakup_probe(const T* phi, const StepConst<T>& P, double* rows, double* sums, hipStream_t s) {
    hipLaunchKernelGGL(k_breakup_rows<T>, dim3(P.ny), dim3(BRK_T), 0, s, phi, P, rows);
    hipLaunchKernelGGL(k_breakup_final, dim3(1), dim3(64), 0, s, rows, P.ny, sums);
}

template void launch_breakup_probe<double>(const double*, const StepConst<double>&, double*, double*, hipStream_t);
template void launch_breakup_probe<float>(const float*, const StepConst<float>&, double*, double*, hipStream_t);

template <typename T>
void launch_extent(const T* phi, const StepConst<T>& P, unsigned long long* ly, double* lx, hipStream_t s) {
    hipLaunchKernelGGL(k_extent_cols<T>, dim3((P.nx + EXT_T - 1) / EXT_T), dim3(EXT_T), 0, s, phi, P, ly);
    hipLaunchKernelGGL(k_extent_centre<T>, dim3(1), dim3(64), 0, s, phi, P, lx);
}

template void launch_extent<double>(const double*, const StepConst<double>&, unsigned long long*, double*,
                                    hipStream_t);
template void launch_extent<float>(const float*, const StepConst<float>&, unsigned long long*, double*, hipStream_t);

}  // namespace fcd
