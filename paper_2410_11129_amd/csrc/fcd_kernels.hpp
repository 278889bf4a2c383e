// fcd_kernels.hpp -- host-side launchers of the gfx950 kernels (fcd_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "fcd_device.hpp"

namespace fcd {

template <typename T>
void launch_init_fields(T* dist, const double* phi1, const double* phi2, const double* ux, const double* uy,
                        const double* ps, int nx, int ny, int pitch, hipStream_t s);
template <typename T>
void launch_init_droplet(T* dist, int nx, int ny, int pitch, double xc, double yc, double rc, double rs, double xi,
                         double u_scale, hipStream_t s);
template <typename T>
void launch_phase(const T* dist, T* phi, const StepConst<T>& P, hipStream_t s);
template <typename T>
void launch_sor_sweep(T* psi, const T* mur, const StepConst<T>& P, T omega, hipStream_t s);
template <typename T>
void launch_residual(const T* psi, const T* mur, const StepConst<T>& P, unsigned long long* out, hipStream_t s);
template <typename T>
void launch_collide_stream(const T* src, T* dst, const T* phi, const T* psi, const StepConst<T>& P, hipStream_t s);
template <typename T>
void launch_moments(const T* src, const T* phi, const T* psi, const StepConst<T>& P, unsigned mask, double* out,
                    hipStream_t s);
template <typename T>
void launch_to_dense(const T* src, double* out, int nplanes, int nx, int ny, int pitch, hipStream_t s);
template <typename T>
void launch_from_dense(const double* in, T* dst, int nplanes, int nx, int ny, int pitch, hipStream_t s);
template <typename T>
void launch_fill(T* a, long long n, T v, hipStream_t s);
template <typename T>
void launch_diagnostics(const T* phi, const StepConst<T>& P, double* rows, double* cent, double* result,
                        hipStream_t s);

}  // namespace fcd
