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
// ev0 / ev1 (nullable): events the launch itself records at the kernel's start and end.
void launch_phase(const T* dist, T* phi, const StepConst<T>& P, hipStream_t s, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr);
// Potential solve (fcd_potential.hip).
template <typename T>
void launch_pot_sweep(const PotLevel<T>& L, T omega, hipStream_t s);
template <typename T>
void launch_pot_residual(const PotLevel<T>& L, unsigned long long* out, hipStream_t s);
// Levels C.mu[0 .. C.n) (n <= 4, each half the previous) from the finer mu plane muf.
template <typename T, typename TC>
void launch_mg_restrict_mu4(const T* muf, int pitchf, int nxf, int nyf, const MuLevels<TC>& C, hipStream_t s);
// One tile-smoother sweep uin -> uout (never the same buffer); prolong_from != nullptr
// adds the prolongation of that coarse level's correction first.  mode 0: coarse level
// (L.f), 1: finest level with the right-hand side from H0, 2: finest level with L.f.
// res != nullptr: max |residual| and max |C u| of uin into res[0..1], which must be zero:
// with res_clear == nullptr a fill launch clears them first; otherwise the kernel itself
// zeroes res_clear[0..1] (the next test's slot) and res must already be zero.
// inner: sweeps on the tile before it is written back.  The coarse correction may be of
// another type (TC) than the level's.  count != nullptr: the launch adds one to *count
// when it runs (it does not when its level's gate has closed it).
template <typename T, typename TC>
void launch_mg_smooth_tile(const PotLevel<T>& L, const T* uin, T* uout, const PotLevel<TC>* prolong_from, int mode,
                           unsigned long long* res, int inner, hipStream_t s, unsigned long long* res_clear = nullptr,
                           unsigned* count = nullptr);
// Residual restriction by tiles from F (u = the smoothed iterate) into C (f, u = 0);
// mode as for the tile smoother.
template <typename T, typename TC>
void launch_mg_restrict_tile(const PotLevel<T>& F, const PotLevel<TC>& C, int mode, hipStream_t s);
// The restriction from F fused with the first `inner`-sweep tile smoothing of the coarse
// level C from a zero correction: C.f is written, the smoothed correction goes to uout
// (C.u is neither read nor written); fmode is F's mode as for the tile smoother.
template <typename T, typename TC>
void launch_mg_restrict_smooth(const PotLevel<T>& F, const PotLevel<TC>& C, int fmode, TC* uout, int inner,
                               hipStream_t s);
// Arrays per node of a multigrid tail level in LDS: iterate, right-hand side, mu, a
// ping-pong array, eight couplings, the diagonal and its reciprocal.
constexpr int MG_TAIL_ARRAYS = 14;
template <typename T>
size_t mg_tail_lds_bytes(const MgTail<T>& tl);
template <typename T>
void launch_mg_tail(const MgTail<T>& tl, hipStream_t s);
template <typename T>
void launch_psi_history(T* psi, T* prev, T* prev2, T* prev3, int nx, int ny, int pitch, int mode, hipStream_t s);
// The same with the recorded solutions in a ring: p1..p3 = psi'(t-1..t-3); psi' replaces p3.
template <typename T>
void launch_psi_history_ring(T* psi, const T* p1, const T* p2, T* p3, int nx, int ny, int pitch, int mode,
                             hipStream_t s);
// Publication of a solve decided on the device that no collide-and-stream ends
// (fcd_potential.hip): one lane, as the collide-and-stream's first.
void launch_solve_publish(const StepGate& sg, hipStream_t s);

// Batched multigrid (fcd_potential.hip): one launch per level for every channel of a
// batch, jobs = (channel, level, tile), channels with active[k] == 0 skipped.
template <typename T, typename TC>
void launch_bmg_smooth_fine(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, int dir,
                            bool prolong, bool rhs_plane, unsigned long long* res, hipStream_t s);
template <typename T, typename TC>
void launch_bmg_copy_fine(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, hipStream_t s);
template <typename T, typename TC>
void launch_bmg_restrict_smooth(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, int level,
                                int src, int inner, bool rhs_plane, hipStream_t s);
template <typename T, typename TC>
void launch_bmg_restrict_tail(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, bool from0,
                              int src, bool rhs_plane, hipStream_t s);
template <typename T, typename TC>
void launch_bmg_tail(const MgChan<T, TC>* ch, int n, size_t lds_bytes, const int* active, hipStream_t s);
template <typename T, typename TC>
void launch_bmg_post_coarse(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, const int* active, int inner,
                            hipStream_t s);
template <typename T, typename TC>
void launch_bmg_mu4(const MgChan<T, TC>* ch, const MgJob* jobs, int njobs, int group, hipStream_t s);
template <typename T, typename TC>
void launch_bmg_decide(const MgChan<T, TC>* ch, int n, unsigned long long* res, int* active, int* cycles, int* counts,
                       double floor_factor, const unsigned long long* rel_scale, double rel_tol, hipStream_t s);
// sg: see StepGate (sg.c == nullptr: ungated).
template <typename T>
void launch_collide_stream(const T* src, T* dst, const T* phi, const T* psi, const StepConst<T>& P,
                           unsigned long long* div, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                           const StepGate& sg = StepGate{});
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
// Eq. 42 extents (fcd_extent.hip): ly[0..1] (bit patterns, zeroed by the caller) and
// lx[0..1] of the outer and inner droplets.
template <typename T>
void launch_extent(const T* phi, const StepConst<T>& P, unsigned long long* ly, double* lx, hipStream_t s);
// Breakup probe (fcd_extent.hip): rows (ny x 8 doubles) of per-row partials, summed in row
// order into sums[0..5] = contact count, sum of y, sum cos, sum sin (contact nodes), outer
// droplet's weighted sum cos, sum sin.
template <typename T>
void launch_breakup_probe(const T* phi, const StepConst<T>& P, double* rows, double* sums, hipStream_t s);
// Open channel (fcd_open.hip): after the periodic collide-and-stream of src into dst, the end
// columns re-collided with zero-gradient phi stencils, then the Eq. 37 inlet and the
// convective outlet (u_in: centreline inflow; U: outlet convective velocity).
// gate: with gate.res set the kernels run only if that residual test passed.
template <typename T>
void launch_open_boundaries(const T* src, T* dst, const T* phi, const T* psi, const StepConst<T>& P, double u_in,
                            double U, hipStream_t s, const ResGate& gate = ResGate{});
// Moments of the two end columns with the open-channel stencils (after launch_moments).
template <typename T>
void launch_open_edge_moments(const T* src, const T* phi, const T* psi, const StepConst<T>& P, unsigned mask,
                              double* out, hipStream_t s);
// Compound-droplet initial state of the open channel (plain distance, Eq. 37 profile).
template <typename T>
void launch_open_init_droplet(T* dist, int nx, int ny, int pitch, double xc, double yc, double rc, double rs,
                              double xi, double u_in, hipStream_t s);

}  // namespace fcd
