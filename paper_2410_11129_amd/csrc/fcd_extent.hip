// fcd_extent.hip -- extent-based deformation index of Eq. 42 on the device:
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

}  // namespace

template <typename T>
void launch_extent(const T* phi, const StepConst<T>& P, unsigned long long* ly, double* lx, hipStream_t s) {
    hipLaunchKernelGGL(k_extent_cols<T>, dim3((P.nx + EXT_T - 1) / EXT_T), dim3(EXT_T), 0, s, phi, P, ly);
    hipLaunchKernelGGL(k_extent_centre<T>, dim3(1), dim3(64), 0, s, phi, P, lx);
}

template void launch_extent<double>(const double*, const StepConst<double>&, unsigned long long*, double*,
                                    hipStream_t);
template void launch_extent<float>(const float*, const StepConst<float>&, unsigned long long*, double*, hipStream_t);

}  // namespace fcd
