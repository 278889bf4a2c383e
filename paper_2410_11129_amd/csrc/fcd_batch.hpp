// fcd_batch.hpp -- per-channel descriptors, tile tables and launchers of the batched step.
#pragma once

#include <hip/hip_runtime.h>

#include "fcd_device.hpp"

namespace fcd {

// Tile shapes 64 x TY, TY = 1, 2, 4, 8 (index 0..3).
constexpr int BATCH_SHAPES = 4;

// One channel of a batch, as the kernels see it (stored in device memory).
template <typename T>
struct BatchInst {
    StepConst<T> P;   // lattice and physics constants
    PotLevel<T> L0;   // potential level: u = psi', mu = mu_r plane, f = nullptr
    T* dist[2];       // the two state buffers (27 planes each)
    T* phi;           // phi1, phi2, mu_r planes
    T* prev;          // psi' history plane: psi'(t-1) ...
    T* prev2;         // ... psi'(t-2) (quadratic start of the multigrid batch; may be null) ...
    T* prev3;         // ... and psi'(t-3) (its cubic start; may be null)
    T* alt;           // second potential plane of the fused sweeps (input and output alternate)
    T omega;          // SOR factor
    double thr;       // stop when max |residual| <= thr (= tol * H0)
    // per tile shape: first tile in the full-resolution and half-resolution (colour)
    // lists, and tiles per row
    int tile0[BATCH_SHAPES], tiles_x[BATCH_SHAPES];
    int ctile0[BATCH_SHAPES], ctiles_x[BATCH_SHAPES];
    int stile0, stiles_x;  // first tile and tiles per row in the fused-sweep (64 x 32) list
    int has_field;         // H0 != 0
    int pad;
    unsigned long long* div;  // the channel's divergence flag word
};

// Per-channel work pointers of the batched adjoint (device descriptors).
template <typename T>
struct BatchAdj {
    T* seg;          // segment records: record r at seg + r * srec (27 state planes, then psi')
    long long srec;  // elements per segment record
    T* lam[2];       // adjoint states (27 planes each)
    T* sens;         // ten stencil sensitivity planes
    T* rhs;          // right-hand side of the adjoint potential equation
    int tile_first, tile_count;  // the channel's tiles in the 64 x 4 list
};

// The tile lists of one shape (device tables: tile -> channel), and the 64 x 32 list of
// the fused sweeps with their sweeps per launch (0: one launch per colour instead).
struct BatchTiles {
    int shape;
    int ntiles, nctiles;
    const int* tiles;
    const int* ctiles;
    int fused;
    int nstiles;
    const int* stiles;
    int* slist;   // device: the fused tiles of the channels active at the last decision
    int* scount;  // kernel (written by it) and their number
    int sgrid;    // blocks of a four-sweep fused launch, which stride over slist
};

// Fused-sweep tile: 64 x 32 nodes plus a halo of 4 nodes per sweep, 512 threads.
constexpr int FUSED_X = 64, FUSED_Y = 32, FUSED_MAX = 4, FUSED_NT = 512;

template <typename T>
void launch_batch_phase(const BatchInst<T>* inst, const BatchTiles& t, int cur, hipStream_t s);
template <typename T>
void launch_batch_collide(const BatchInst<T>* inst, const BatchTiles& t, int cur, hipStream_t s);
// One four-colour SOR sweep of the active channels.
template <typename T>
void launch_batch_sweep(const BatchInst<T>* inst, const BatchTiles& t, const int* active, hipStream_t s);
// The activity decision of a test carried out at the start of the next fused sweep
// launch instead of by a kernel of its own: every block decides its own channel from
// the test's residual slots and the flag before the decision (the blocks of a channel
// all reach the same decision, the one launch_batch_decide takes); the channel's first
// block stores it in the other flag buffer, adds `add` to sweeps[k] if the channel was
// active, and zeroes the channel's slots in `clear` (those of the next test that is not
// this launch's).  A channel stopped by the decision whose result is in the second
// plane (odd parity) is copied back to its own plane by its tiles.  res == nullptr: no
// decision in this launch.
struct BatchDecide {
    const unsigned long long* res;
    unsigned long long* clear;
    const unsigned long long* scale;
    double rel_tol;
    int* sweeps;
    int add;
};
// t.fused (1, 2 or 4) four-colour SOR sweeps of the active channels in one launch,
// bitwise equal to as many launch_batch_sweep calls; parity 0 reads L0.u and writes alt,
// parity 1 the reverse.  rhs_plane: the descriptors' L0.f is set (else the field gives
// the rhs).  Activity flags are read from act_in; a deciding launch writes act_out.
// res != nullptr: also reduce the residual of the result as launch_batch_check does
// (a decision has to follow, folded into the next launch or by launch_batch_decide);
// res, dec.res and dec.clear are three different slot sets.
template <typename T>
void launch_batch_sweep_fused(const BatchInst<T>* inst, const BatchTiles& t, const int* act_in, int* act_out,
                              int parity, bool rhs_plane, unsigned long long* res, const BatchDecide& dec,
                              hipStream_t s);
// The activity decision of launch_batch_check alone, on residual slots already filled;
// also_clear, also_clear2 (may be null): more slot sets to zero, those of earlier tests
// decided by fused launches.  Flags are read from buffer cur of the two at `active`
// (2 n ints) and written to both.  Also lists the fused tiles of the channels left
// active (t.slist, t.scount) for the following fused launches.
template <typename T>
void launch_batch_decide(const BatchInst<T>* inst, const BatchTiles& t, int n, unsigned long long* res,
                         unsigned long long* also_clear, unsigned long long* also_clear2, int* active, int cur,
                         int* counts, const unsigned long long* scale, double rel_tol, int* sweeps, int add,
                         hipStream_t s);
// Residual of the active channels, then the activity decision; res must be zero on entry
// and is left zero; counts[0..1] = active channels, channels with a NaN residual.
// scale != nullptr: channel k's threshold is rel_tol * scale[k] (bit pattern of a
// non-negative double) instead of its descriptor's thr.  sweeps[k] += add for every
// channel active on entry (add: sweeps since the previous test).
template <typename T>
void launch_batch_check(const BatchInst<T>* inst, const BatchTiles& t, int n, unsigned long long* res,
                        int* active, int* counts, const unsigned long long* scale, double rel_tol, int* sweeps,
                        int add, hipStream_t s);
template <typename T>
void launch_batch_psi_history(const BatchInst<T>* inst, const BatchTiles& t, int mode, hipStream_t s);
template <typename T>
void launch_batch_fill_psi(const BatchInst<T>* inst, const BatchTiles& t, hipStream_t s);

// Batched adjoint (fcd_adjoint.hip); all over the 64 x 4 tile list `t` (shape 2).
template <typename T>
void launch_batch_adj_save(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t, int cur, int r,
                           int what, hipStream_t s);
template <typename T>
void launch_batch_adj_phase(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t, int r,
                            hipStream_t s);
template <typename T>
void launch_batch_adj_node(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t, int r, int A,
                           double* part, hipStream_t s);
template <typename T>
void launch_batch_adj_gather(const BatchInst<T>* inst, const BatchAdj<T>* adj, const BatchTiles& t,
                             unsigned long long* scale, int n, hipStream_t s);
template <typename T>
void launch_batch_adj_finish(const BatchInst<T>* inst, const BatchInst<T>* ainst, const BatchAdj<T>* adj,
                             const BatchTiles& t, int r, int A, double* part, hipStream_t s);
template <typename T>
void launch_batch_adj_reduce(const BatchAdj<T>* adj, int n, const double* part, int nq, double* acc, int dst,
                             hipStream_t s);

}  // namespace fcd
