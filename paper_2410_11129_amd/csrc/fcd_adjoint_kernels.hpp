// fcd_adjoint_kernels.hpp -- launchers of the reverse coupled step (fcd_adjoint.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "fcd_device.hpp"

namespace fcd {

constexpr int ADJ_NPART = 16;  // parameter partial slots per block

int adj_blocks(int nx, int ny);
template <typename T>
void launch_adj_node(const T* st, const T* phi, const T* psi, const T* lam_next, T* lam, T* sens, double* part,
                     const StepConst<T>& P, hipStream_t s);
template <typename T>
void launch_adj_gather_psi(const T* sens, T* rhs, unsigned long long* rmax, const StepConst<T>& P, hipStream_t s);
template <typename T>
void launch_adj_finish(const T* sens, const T* phi, const T* psi, const T* lpsi, T* lam, double* part,
                       const StepConst<T>& P, hipStream_t s);
void launch_adj_reduce(const double* part, int nblocks, int nq, double* acc, int dst, hipStream_t s);
template <typename T>
void launch_adj_seed(const T* phi, const double* dg, double dJo, double dJi, T* lam, const StepConst<T>& P,
                     hipStream_t s);
template <typename T>
void launch_adj_init_drive(const T* s0, const T* lam0, double dU_dG_scale, double u_scale, double* part,
                           const StepConst<T>& P, hipStream_t s);

}  // namespace fcd
