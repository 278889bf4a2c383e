// fcd_batch.hpp -- per-channel descriptors and launchers of the batched step.
#pragma once

#include <hip/hip_runtime.h>

#include "fcd_device.hpp"

namespace fcd {

// One channel of a batch, as the kernels see it (stored in device memory).
template <typename T>
struct BatchInst {
    StepConst<T> P;   // lattice and physics constants
    PotLevel<T> L0;   // potential level: u = psi', mu = mu_r plane, f = nullptr
    T* dist[2];       // the two state buffers (27 planes each)
    T* phi;           // phi1, phi2, mu_r planes
    T* prev;          // psi' history plane
    T omega;          // SOR factor
    double thr;       // stop when max |residual| <= thr (= tol * H0)
    int tile0, tiles_x;    // first tile in the full-resolution list, tiles per row
    int ctile0, ctiles_x;  // the same for the half-resolution (colour) list
    int has_field;         // H0 != 0
    int pad;
};

template <typename T>
void launch_batch_phase(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int cur, hipStream_t s);
template <typename T>
void launch_batch_collide(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int cur, hipStream_t s);
template <typename T>
void launch_batch_sweep(const BatchInst<T>* inst, const int* ctile_inst, int nctiles, const int* active,
                        hipStream_t s);
template <typename T>
void launch_batch_residual(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int n,
                           unsigned long long* res, int* active, int* counts, hipStream_t s);
template <typename T>
void launch_batch_psi_history(const BatchInst<T>* inst, const int* tile_inst, int ntiles, int mode, hipStream_t s);
template <typename T>
void launch_batch_fill_psi(const BatchInst<T>* inst, const int* tile_inst, int ntiles, hipStream_t s);

}  // namespace fcd
