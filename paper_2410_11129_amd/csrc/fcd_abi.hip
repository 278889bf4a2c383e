// fcd_abi.hip -- the C ABI declared in include/fcd.h: argument checks, per-step
// orchestration of the kernels on the caller's stream, potential-solve control.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fcd.h"
#include "fcd_adjoint_kernels.hpp"
#include "fcd_batch.hpp"
#include "fcd_kernels.hpp"

namespace {

thread_local std::string g_err;

fcd_status fail(fcd_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

fcd_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return FCD_OK;
    return fail(FCD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Scratch layout (bytes from the start of the caller's scratch buffer).
// Residual words: bit patterns of max |residual| and max |C psi'|.  The multigrid's tests
// alternate between two slots A and B placed around the divergence flag, so one
// three-word copy brings a test's pair and the flag (A: words 0-2, B: words 2-4); each
// test's kernel zeroes the other slot for the next test.  SOR tests use words 5-6.
constexpr size_t OFF_RES = 0;      // slot A, 2 x uint64
constexpr size_t OFF_DIV = 16;     // uint64: divergence flag (0, or the worst node's max |u| bits / NaN)
constexpr size_t OFF_RES_B = 24;   // slot B, 2 x uint64
constexpr size_t OFF_RES_SOR = 40; // 2 x uint64 (SOR and the explicit residual kernel)
constexpr size_t OFF_SLOTS = 64;   // SOLVE_SLOTS x 2 x uint64: residual tests of solves decided on the device
constexpr size_t OFF_TESTS = OFF_SLOTS + 16 * fcd::SOLVE_SLOTS;  // uint32: such tests run since the last publication
constexpr size_t OFF_CENT = 256;   // 8 doubles: centroids and masses
constexpr size_t OFF_RESULT = 512; // 4 doubles: D_o, D_i, mass1, mass2
constexpr size_t OFF_EXTENT = 768; // Eq. 42 extents: 2 x uint64 (l_y bit patterns), 2 doubles (l_x)
constexpr size_t OFF_BREAKUP = 832; // breakup probe: 6 doubles of sums
constexpr size_t OFF_ROWS = 1024;  // ny * 8 doubles: per-row partial sums
static_assert(OFF_SLOTS >= OFF_RES_SOR + 16 && OFF_TESTS + 8 <= OFF_CENT && (OFF_TESTS + 8) / 8 <= 64,
              "scratch words overlap");

size_t elem_size(int precision) { return precision == FCD_FP64 ? sizeof(double) : sizeof(float); }

// Default SOR factor 2 / (1 + sin(pi / (ny + 1))): the optimum of the five-point
// Laplacian between Dirichlet rows ny + 1 cells apart.  For the nine-point operator the
// asymptotic optimum is larger (2 / (1 + sqrt(1 - rho^2)), rho = 0.4 + 0.6 cos(pi /
// (ny + 1))), but the warm-started solves of a time step are not in the asymptotic
// regime, and which factor needs fewer sweeps there depends on the field direction.
double sor_omega_opt(int ny) { return 2.0 / (1.0 + std::sin(3.14159265358979323846 / (ny + 1))); }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// The periodic channel's drive is the body force whose Poiseuille profile between the
// halfway walls peaks at u_ref: drive_G = 8 rho_3 nu_3 u_ref / ny^2, nu_3 = c_s^2 tau_3
// (the pressure-driven flow of Sec. 2.5 as a body force); d drive_G / d u_ref.
double drive_per_u_ref(const fcd_params& p, int ny) { return 8.0 * p.rho[2] * (p.tau[2] / 3.0) / ((double)ny * ny); }

// Divergence guard settings (0 selects the default).
double u_limit_of(const fcd_params& p) { return p.u_limit > 0.0 ? p.u_limit : 0.5; }
int div_every_of(const fcd_params& p) { return p.div_check_every > 0 ? p.div_check_every : 64; }

// Multigrid hierarchy and scratch layout.  Level 0 is the lattice itself (psi', mu_r
// planes of the caller, in the lattice's precision); a level of nx x ny nodes with
// nx, ny >= 4 has a coarser one of ceil(nx/2) x floor(ny/2) or ceil(ny/2) nodes (odd sizes
// included; the row count by the wall distance below, the geometry in fcd_potential.hip),
// and the coarse levels are FP32 in both precisions: they only compute corrections, each cycle's residual is formed on level 0
// in the lattice's precision, so the solve still reaches that precision's tolerance
// (mixed-precision multigrid), while the latency-bound coarse kernels run FP32 arithmetic
// on half the bytes.  The coarsest levels whose LDS arrays (u, f, mu, a Jacobi ping-pong
// array and the precomputed couplings: MG_TAIL_ARRAYS per node) fit together in
// TAIL_LDS_MAX bytes form the tail, solved in LDS by one block; every level above the tail
// has a second plane for the tile smoother's ping-pong.
using CT = float;  // element type of the coarse levels
constexpr int MAX_LEVELS = 16;
constexpr size_t TAIL_LDS_MAX = 98304;  // of the 160 KB of LDS a gfx950 workgroup may use
// Tile sweeps per smoothing launch on the levels between the finest and the tail.
constexpr int MG_COARSE_INNER = 2;

struct MgPlan {
    int levels;
    int tail;  // first tail level (== levels: no tail)
    int nx[MAX_LEVELS], ny[MAX_LEVELS], pitch[MAX_LEVELS];
    double kappa_top[MAX_LEVELS];  // upper ghost rule of each level (fcd_potential.hip)
    size_t off_mu[MAX_LEVELS], off_u[MAX_LEVELS], off_f[MAX_LEVELS], off_t[MAX_LEVELS];
    // psi' history: a ring of three planes holding psi'(t-1), psi'(t-2) (quadratic
    // extrapolation) and psi'(t-3) (cubic), the newest at fcd_handle::ring
    size_t off_prev;
    size_t off_prev2;
    size_t off_prev3;
    size_t bytes;     // total scratch
};

MgPlan make_plan(const fcd_lattice& l) {
    const size_t esz = elem_size(l.precision);
    MgPlan p{};
    p.levels = 1;
    p.nx[0] = l.nx;
    p.ny[0] = l.ny;
    p.pitch[0] = l.pitch;
    p.kappa_top[0] = 0.0;
    while (p.levels < MAX_LEVELS) {
        const int px = p.nx[p.levels - 1], py = p.ny[p.levels - 1];
        if (px < 4 || py < 4) break;
        const int L = p.levels++;
        p.nx[L] = (px + 1) / 2;
        const int per = (int)(256 / sizeof(CT));
        p.pitch[L] = (p.nx[L] + per - 1) / per * per;
        // rows: floor(py/2), or ceil(py/2) when that puts the last row (spacing h, the first
        // row (h-1)/2 above row 0) nearer the distance (h+1)/2 below the finest level's upper
        // ghost row y = ny that every level of an even hierarchy has, and not closer than
        // h/4; so the distance stays >= h/4 (kappa_top <= 3) and is finite (kappa_top > -1)
        const double h = double(1 << L);
        auto dist = [&](int rows) { return (double)l.ny - (h * (rows - 1) + 0.5 * (h - 1.0)); };
        const int fl = py / 2, ce = (py + 1) / 2;
        const double ideal = 0.5 * (h + 1.0);
        p.ny[L] = (dist(ce) >= 0.25 * h && std::fabs(dist(ce) - ideal) < std::fabs(dist(fl) - ideal)) ? ce : fl;
        const double d = dist(p.ny[L]);
        p.kappa_top[L] = (h - d) / d;
    }
    p.tail = p.levels;
    size_t tail_bytes = 0;
    for (int L = p.levels - 1; L >= 1 && p.levels - L <= fcd::MG_MAX_TAIL; --L) {
        const size_t b = fcd::MG_TAIL_ARRAYS * (size_t)p.nx[L] * p.ny[L] * sizeof(CT);
        if (tail_bytes + b > TAIL_LDS_MAX) break;
        tail_bytes += b;
        p.tail = L;
    }
    // without a tail the coarsest level is solved by launched four-colour sweeps, which
    // need an even width (on an odd periodic row the first and last nodes share a colour)
    while (p.tail == p.levels && p.levels > 1 && (p.nx[p.levels - 1] & 1)) p.tail = --p.levels;
    size_t off = align256(OFF_ROWS + (size_t)l.ny * 8 * sizeof(double));
    p.off_prev = off;
    off += align256((size_t)l.ny * l.pitch * esz);
    p.off_prev2 = off;
    off += align256((size_t)l.ny * l.pitch * esz);
    p.off_prev3 = off;
    off += align256((size_t)l.ny * l.pitch * esz);
    for (int L = 0; L < p.levels; ++L) {
        const size_t plane = align256((size_t)p.ny[L] * p.pitch[L] * (L == 0 ? esz : sizeof(CT)));
        if (L > 0) {
            p.off_mu[L] = off;
            p.off_u[L] = off + plane;
            p.off_f[L] = off + 2 * plane;
            off += 3 * plane;
        }
        if (L < p.tail && p.levels > 1) {
            p.off_t[L] = off;
            off += plane;
        }
    }
    p.bytes = off;
    return p;
}

}  // namespace

// Timed kernel classes: collide-stream, potential iteration (V-cycle or SOR sweep),
// convergence test, phase moments, finest-level pre-smoothing and
// finest-level prolongation + post-smoothing of the multigrid.
enum { TK_COLLIDE = 0, TK_ITER = 1, TK_RESID = 2, TK_PHASE = 3, TK_SMOOTH0 = 4, TK_POST0 = 5, TK_KINDS = 6 };

// Event pairs bracketing launches, resolved into per-class totals after a sync.
struct Timer {
    struct Pair {
        int kind;
        hipEvent_t a, b;
    };
    bool on = false;
    bool collide_only = false;  // only the collide-and-stream's launches are timed
    std::vector<Pair> pending;
    std::vector<hipEvent_t> pool;
    double ms[TK_KINDS] = {};
    double count[TK_KINDS] = {};

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Record the opening event of a bracket; returns false when timing is off.
    bool begin(hipStream_t s, hipEvent_t* a) {
        if (!on) return false;
        *a = take();
        return *a && hipEventRecord(*a, s) == hipSuccess;
    }
    void end(hipStream_t s, int kind, hipEvent_t a) {
        hipEvent_t b = take();
        if (!b || hipEventRecord(b, s) != hipSuccess) return;
        pending.push_back({kind, a, b});
    }
    // Two events for a launch that records them itself (hipExtLaunchKernel): they time the
    // kernel alone, without the host's launch gap that a recorded bracket on an idle stream
    // would include.  Returns false when timing is off.
    bool pair(hipEvent_t* a, hipEvent_t* b) {
        *a = *b = nullptr;
        if (!on) return false;
        *a = take();
        *b = take();
        return *a && *b;
    }
    // The same for a collide-and-stream launch, which is also timed when only it is.
    bool pair_collide(hipEvent_t* a, hipEvent_t* b) {
        *a = *b = nullptr;
        if (!on && !collide_only) return false;
        *a = take();
        *b = take();
        return *a && *b;
    }
    void add(int kind, hipEvent_t a, hipEvent_t b) { pending.push_back({kind, a, b}); }
    // Events of a launch whose time is not wanted (a collision whose gate stayed closed).
    void drop(hipEvent_t a, hipEvent_t b) {
        if (a) pool.push_back(a);
        if (b) pool.push_back(b);
    }
    // Only after the stream has been synchronised.
    void resolve() {
        for (const Pair& p : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
                ms[p.kind] += t;
                count[p.kind] += 1;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    void clear() {
        for (int k = 0; k < TK_KINDS; ++k) ms[k] = count[k] = 0;
    }
    ~Timer() {
        for (const Pair& p : pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};


// Instantiated HIP graphs of recurring launch sequences, keyed by the buffers they
// touch and a kind.  Captured on a private non-blocking stream (default priority) and
// launched on the caller's stream; cleared whenever the parameters baked into the
// kernel arguments change.
struct GraphCache {
    struct Entry {
        const void* k1;
        const void* k2;
        int kind;
        hipGraphExec_t exec;
    };
    std::vector<Entry> entries;
    hipStream_t cap = nullptr;
    bool enabled = true;

    hipGraphExec_t find(const void* k1, const void* k2, int kind) const {
        for (const Entry& e : entries)
            if (e.k1 == k1 && e.k2 == k2 && e.kind == kind) return e.exec;
        return nullptr;
    }
    void clear() {
        for (const Entry& e : entries) (void)hipGraphExecDestroy(e.exec);
        entries.clear();
    }
    ~GraphCache() {
        clear();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

struct fcd_handle {
    fcd_lattice lat;
    fcd_params prm;
    fcd_buffers buf;
    hipStream_t stream;
    int cur;        // index of dist[] holding the current state
    double* host;   // pinned host words: [0] residual bits, [1..4] diagnostics
    long long steps;
    long long sweeps;
    double last_resid;
    int hist;  // completed step solves since the last state change (psi' history validity)
    int qs;    // steps since the last state change (the potential is solved when qs % pot_every == 0)
    int last_iters;  // iterations the previous solve needed (first residual test is deferred)
    int res_slot;    // multigrid residual slot of the next test (0: A, 1: B); that slot is zero
    // time steps whose multigrid solve is decided on the device (step_solve_collide)
    fcd::SolveMirror* mirror;      // pinned, coherent: the tests as published by the GPU
    unsigned long long seq_want;   // publications launched so far (the mirror's seq catches up)
    unsigned long long test_idx;   // index of the next such residual test (slot test_idx % 3)
    fcd::ResGate gate;             // set while launching gated kernels: levels built carry it
    int pipe_last;                 // V-cycles the previous such solve needed
    int ring;  // the psi' history plane (0..2 of off_prev, off_prev2, off_prev3) holding psi'(t-1)
    int init_fresh;  // the state is the compound-droplet initial state (no step since)
    int open_x;      // open channel: Eq. 37 inlet at x = 0, convective outlet at x = nx - 1
    double u_in;     // u_avg of Eq. 37 (centreline value of the inlet profile)
    double u_out;    // convective velocity of the outlet: the section mean of the inlet profile
    // breakup tracking (fcd_breakup_track): the outer droplet's x followed across the periodic
    // boundary since the last state change
    int track_on;
    double track_x_prev, track_x_run;
    long long steps_at_init;  // h->steps when the state was last replaced
    double r_shell;           // shell radius of fcd_init_compound_droplet (0: other initial state)
    // checkpointed adjoint: set by fcd_adjoint_forward, used by fcd_adjoint_backward
    char* adj_work;
    int adj_nsteps, adj_every, adj_from_init;
    // last_iters and hist at each checkpoint (pairs) and at the end, so that a recomputed
    // segment repeats the forward's solves exactly
    std::vector<int> adj_ckpt_iters;
    int adj_final_iters, adj_final_hist;
    GraphCache graphs;
    MgPlan plan;
    Timer timer;
};

namespace {

fcd_status check_params(const fcd_params* p) {
    if (!p) return fail(FCD_ERR_ARG, "params is null");
    for (int k = 0; k < 3; ++k) {
        if (!(p->rho[k] > 0.0)) return fail(FCD_ERR_ARG, "densities must be positive");
        if (!(p->tau[k] > 0.0)) return fail(FCD_ERR_ARG, "relaxation times must be positive");
        if (!(p->chi[k] > -1.0)) return fail(FCD_ERR_ARG, "susceptibilities must exceed -1");
    }
    const double g0 = p->sigma12 + p->sigma13 - p->sigma23, g1 = p->sigma12 + p->sigma23 - p->sigma13,
                 g2 = p->sigma13 + p->sigma23 - p->sigma12;
    if (g0 == 0.0 || g1 == 0.0 || g2 == 0.0) return fail(FCD_ERR_ARG, "a spreading coefficient gamma_i is zero");
    if (1.0 / g0 + 1.0 / g1 + 1.0 / g2 == 0.0) return fail(FCD_ERR_ARG, "gamma_T undefined");
    if (!(p->xi > 0.0) || !(p->mobility > 0.0)) return fail(FCD_ERR_ARG, "xi and mobility must be positive");
    if (!(p->pot_omega == 0.0 || (p->pot_omega > 0.0 && p->pot_omega < 2.0)))
        return fail(FCD_ERR_ARG, "pot_omega must be 0 (automatic) or lie in (0, 2)");
    if (!(p->pot_tol > 0.0)) return fail(FCD_ERR_ARG, "pot_tol must be positive");
    if (p->pot_solver != FCD_SOLVER_SOR && p->pot_solver != FCD_SOLVER_MG)
        return fail(FCD_ERR_ARG, "unknown pot_solver");
    if (p->pot_check_every < 1 || p->pot_max_iters < 0) return fail(FCD_ERR_ARG, "bad potential iteration counts");
    if (p->pot_solver == FCD_SOLVER_MG && (p->pot_smooth < 1 || p->pot_coarse_sweeps == 0))
        return fail(FCD_ERR_ARG, "multigrid needs pot_smooth >= 1 and pot_coarse_sweeps != 0");
    if (p->pot_extrapolate < 0 || p->pot_extrapolate > 3)
        return fail(FCD_ERR_ARG, "pot_extrapolate must be 0, 1, 2 or 3");
    if (p->pot_every < 0) return fail(FCD_ERR_ARG, "pot_every must be >= 0");
    if (!(p->u_limit >= 0.0)) return fail(FCD_ERR_ARG, "u_limit must be >= 0 (0: default)");
    if (p->div_check_every < 0) return fail(FCD_ERR_ARG, "div_check_every must be >= 0 (0: default)");
    return FCD_OK;
}

fcd_status check_lattice(const fcd_lattice* l) {
    if (!l) return fail(FCD_ERR_ARG, "lattice is null");
    if (l->nx < 4 || (l->nx & 1)) return fail(FCD_ERR_ARG, "nx must be even and >= 4");
    if (l->ny < 2) return fail(FCD_ERR_ARG, "ny must be >= 2");
    if (l->pitch < l->nx) return fail(FCD_ERR_ARG, "pitch must be >= nx");
    if (l->precision != FCD_FP64 && l->precision != FCD_FP32) return fail(FCD_ERR_ARG, "unknown precision");
    if ((long long)l->ny * l->pitch * 27 > (1LL << 40)) return fail(FCD_ERR_ARG, "lattice too large");
    return FCD_OK;
}

template <typename T>
fcd::StepConst<T> make_const(const fcd_handle* h) {
    const fcd_params& p = h->prm;
    fcd::StepConst<T> c{};
    c.nx = h->lat.nx;
    c.ny = h->lat.ny;
    c.pitch = h->lat.pitch;
    c.plane = (long long)h->lat.ny * h->lat.pitch;
    c.rho0 = T(p.rho[0]);
    c.rho1 = T(p.rho[1]);
    c.rho2 = T(p.rho[2]);
    c.tau0 = T(p.tau[0]);
    c.tau1 = T(p.tau[1]);
    c.tau2 = T(p.tau[2]);
    c.ic0 = T(1.0 / (1.0 + p.chi[0]));
    c.ic1 = T(1.0 / (1.0 + p.chi[1]));
    c.ic2 = T(1.0 / (1.0 + p.chi[2]));
    const double g0 = p.sigma12 + p.sigma13 - p.sigma23;  // Eq. 27
    const double g1 = p.sigma12 + p.sigma23 - p.sigma13;
    const double g2 = p.sigma13 + p.sigma23 - p.sigma12;
    const double gT = 3.0 / (1.0 / g0 + 1.0 / g1 + 1.0 / g2);  // Eq. 26
    c.gam0 = T(g0);
    c.gam1 = T(g1);
    c.gam2 = T(g2);
    c.igam0 = T(1.0 / g0);
    c.igam1 = T(1.0 / g1);
    c.igam2 = T(1.0 / g2);
    c.s12 = T(p.sigma12);
    c.s13 = T(p.sigma13);
    c.s23 = T(p.sigma23);
    c.eta = T(p.eta);
    c.c_bulk = T(4.0 * gT / p.xi);
    c.c_lap = T(0.75 * p.xi);
    c.four_over_xi = T(4.0 / p.xi);
    c.omega_phi = T(1.0 / (3.0 * p.mobility + 0.5));  // tau_phi = M / c_s^2
    c.H0x = T(p.H0 * std::cos(p.alpha));
    c.H0y = T(p.H0 * std::sin(p.alpha));
    c.half_mu0 = T(0.5 * p.mu0);
    c.drive = T(p.drive_G);
    c.grav_x = T(p.grav_x);
    c.grav_y = T(p.grav_y);
    c.eps2 = T(p.eps_n * p.eps_n);
    c.u_limit = T(u_limit_of(p));
    return c;
}

template <typename T>
T* plane_ptr(void* base, const fcd_handle* h, int q) {
    return static_cast<T*>(base) + (long long)q * h->lat.ny * h->lat.pitch;
}

unsigned long long* res_word(const fcd_handle* h) {
    return reinterpret_cast<unsigned long long*>(static_cast<char*>(h->buf.scratch) + OFF_RES_SOR);
}

unsigned long long* res_slot_ptr(const fcd_handle* h, int slot) {
    return reinterpret_cast<unsigned long long*>(static_cast<char*>(h->buf.scratch) + (slot ? OFF_RES_B : OFF_RES));
}

// The divergence flag sits right after the two residual words, so one three-word copy
// brings a residual test's result and the flag to the host together.
unsigned long long* div_word(const fcd_handle* h) {
    return reinterpret_cast<unsigned long long*>(static_cast<char*>(h->buf.scratch) + OFF_DIV);
}


// FCD_ERR_DIVERGED when a divergence flag word (as the collide kernel raises it) is set.
fcd_status divergence_status(unsigned long long w, double limit, const std::string& who) {
    if (w == 0) return FCD_OK;
    double v;
    std::memcpy(&v, &w, sizeof(v));
    char msg[200];
    if (v != v)
        std::snprintf(msg, sizeof(msg), "%s: the state is not finite (NaN or Inf in p*, phi1 or phi2)", who.c_str());
    else
        std::snprintf(msg, sizeof(msg), "%s: max |u| = %.6g exceeds u_limit = %.6g", who.c_str(), v, limit);
    return fail(FCD_ERR_DIVERGED, msg);
}

// Waits for the stream, then reports the flag.
fcd_status read_divergence(fcd_handle* h) {
    fcd_status st = hip_check(hipMemcpyAsync(h->host + 24, div_word(h), sizeof(unsigned long long),
                                             hipMemcpyDeviceToHost, h->stream), "divergence flag copy");
    if (!st) st = hip_check(hipStreamSynchronize(h->stream), "divergence flag sync");
    if (st) return st;
    unsigned long long w;
    std::memcpy(&w, h->host + 24, sizeof(w));
    return divergence_status(w, u_limit_of(h->prm), "divergence guard");
}

fcd_status clear_divergence(fcd_handle* h) {
    hipLaunchKernelGGL(fcd::k_fill<unsigned long long>, dim3(1), dim3(64), 0, h->stream, div_word(h), 1LL, 0ULL);
    return hip_check(hipGetLastError(), "divergence flag clear");
}

// The psi' history plane holding psi'(t-k), k = 1, 2, 3 (a ring of three planes).
template <typename T>
T* psi_prev(fcd_handle* h, int k = 1) {
    const int q = (h->ring + k - 1) % 3;
    const size_t off = q == 0 ? h->plan.off_prev : q == 1 ? h->plan.off_prev2 : h->plan.off_prev3;
    return reinterpret_cast<T*>(static_cast<char*>(h->buf.scratch) + off);
}

// Level 0 (the lattice's psi' and mu_r planes).
template <typename T>
fcd::PotLevel<T> pot_level(const fcd_handle* h, int l) {
    fcd::PotLevel<T> L{};
    L.nx = h->plan.nx[l];
    L.ny = h->plan.ny[l];
    L.pitch = h->plan.pitch[l];
    L.u = static_cast<T*>(h->buf.psi);
    L.mu = plane_ptr<T>(h->buf.phi, h, 2);
    L.f = nullptr;
    L.gate = h->gate;
    L.inv_h2 = T(1);
    L.kappa = T(0);
    L.kappa_top = T(0);
    L.H0x = T(h->prm.H0 * std::cos(h->prm.alpha));
    L.H0y = T(h->prm.H0 * std::sin(h->prm.alpha));
    return L;
}

// Coarse level l >= 1 (FP32 planes in the scratch).
fcd::PotLevel<CT> coarse_level(const fcd_handle* h, int l) {
    fcd::PotLevel<CT> L{};
    char* s = static_cast<char*>(h->buf.scratch);
    L.nx = h->plan.nx[l];
    L.ny = h->plan.ny[l];
    L.pitch = h->plan.pitch[l];
    {
        const double hh = double(1 << l);
        L.u = reinterpret_cast<CT*>(s + h->plan.off_u[l]);
        L.mu = reinterpret_cast<const CT*>(s + h->plan.off_mu[l]);
        L.f = reinterpret_cast<CT*>(s + h->plan.off_f[l]);
        L.gate = h->gate;
        L.inv_h2 = CT(1.0 / (hh * hh));
        L.kappa = CT((hh - 1.0) / (hh + 1.0));
        L.kappa_top = CT(h->plan.kappa_top[l]);
        L.H0x = L.H0y = CT(0);
    }
    return L;
}

// Rounding floor of the residual test: a residual below 16 machine epsilons of the
// largest diagonal term C psi' cannot be resolved in the working precision.
template <typename T>
constexpr double resid_floor_factor() {
    return 16.0 * (sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07);
}

template <typename T>
fcd_status read_residual(fcd_handle* h, const fcd::PotLevel<T>& L0, double* r, double* scale) {
    hipEvent_t ev = nullptr;
    const bool timed = h->timer.begin(h->stream, &ev);
    fcd::launch_pot_residual<T>(L0, res_word(h), h->stream);
    if (timed) h->timer.end(h->stream, TK_RESID, ev);
    fcd_status st = hip_check(hipGetLastError(), "residual launch");
    if (st) return st;
    // words 2-6: the divergence flag, slot B (skipped) and the SOR words
    st = hip_check(hipMemcpyAsync(h->host, div_word(h), 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                   "residual copy");
    if (st) return st;
    st = hip_check(hipStreamSynchronize(h->stream), "residual sync");
    if (st) return st;
    h->timer.resolve();
    std::memcpy(r, h->host + 3, sizeof(double));
    std::memcpy(scale, h->host + 4, sizeof(double));
    unsigned long long w;
    std::memcpy(&w, h->host, sizeof(w));
    return divergence_status(w, u_limit_of(h->prm), "divergence guard");
}

// Coarse mu on every level, from the current mu_r plane.
template <typename T>
void restrict_mu_all(fcd_handle* h) {
    for (int l = 1; l < h->plan.levels; l += 4) {
        fcd::MuLevels<CT> C{};
        C.n = std::min(4, h->plan.levels - l);
        for (int k = 0; k < C.n; ++k) {
            const fcd::PotLevel<CT> Ck = coarse_level(h, l + k);
            C.mu[k] = const_cast<CT*>(Ck.mu);
            C.nx[k] = Ck.nx;
            C.ny[k] = Ck.ny;
            C.pitch[k] = Ck.pitch;
        }
        if (l == 1) {
            const fcd::PotLevel<T> F = pot_level<T>(h, 0);
            fcd::launch_mg_restrict_mu4<T, CT>(F.mu, F.pitch, F.nx, F.ny, C, h->stream);
        } else {
            const fcd::PotLevel<CT> F = coarse_level(h, l - 1);
            fcd::launch_mg_restrict_mu4<CT, CT>(F.mu, F.pitch, F.nx, F.ny, C, h->stream);
        }
    }
}

// Run the launch sequence `record` (which launches on h->stream) through a cached HIP
// graph, capturing it on first use; eagerly while per-kernel timing is on or graphs
// are disabled.
template <typename F>
fcd_status run_graph_on(GraphCache& G, hipStream_t& stream, bool eager, const void* k1, const void* k2, int kind,
                        F&& record) {
    if (!G.enabled || eager) {
        record();
        return hip_check(hipGetLastError(), "launch");
    }
    hipGraphExec_t exec = G.find(k1, k2, kind);
    if (!exec) {
        fcd_status st = FCD_OK;
        if (!G.cap) st = hip_check(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking), "capture stream");
        if (st) return st;
        hipStream_t saved = stream;
        st = hip_check(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal), "begin capture");
        if (st) return st;
        stream = G.cap;
        record();
        stream = saved;
        hipGraph_t graph = nullptr;
        st = hip_check(hipStreamEndCapture(G.cap, &graph), "end capture");
        if (st) return st;
        st = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
        (void)hipGraphDestroy(graph);
        if (st) return st;
        G.entries.push_back({k1, k2, kind, exec});
    }
    return hip_check(hipGraphLaunch(exec, stream), "graph launch");
}

template <typename F>
fcd_status run_graph(fcd_handle* h, const void* k1, const void* k2, int kind, F&& record) {
    return run_graph_on(h->graphs, h->stream, h->timer.on, k1, k2, kind, record);
}

// SOR sweeps per V-cycle on a coarsest level with ny rows: pot_coarse_sweeps times
// max(1, ny / 2) (a few suffice on the two-row levels of a full hierarchy; a hierarchy
// stopped early gets more on its larger rows), or exactly -pot_coarse_sweeps when negative.
int coarse_sweeps(const fcd_handle* h, int ny) {
    const int c = h->prm.pot_coarse_sweeps;
    return c < 0 ? -c : c * std::max(1, ny / 2);
}

// Solve the coarsest level by launched SOR sweeps (no tail, or no coarse level at all).
template <typename T>
void coarse_solve(fcd_handle* h, const fcd::PotLevel<T>& L, bool finest) {
    const T om = T(finest && h->prm.pot_omega > 0.0 ? h->prm.pot_omega : sor_omega_opt(L.ny));
    for (int s = 0; s < coarse_sweeps(h, L.ny); ++s) fcd::launch_pot_sweep<T>(L, om, h->stream);
}

// Multigrid V-cycle with tile smoothers.  Level l above the tail keeps its iterate in
// the level's u plane and uses a second plane t for the smoother's ping-pong; the
// finest level's mode decides how its right-hand side is formed.
template <typename T>
T* mg_temp(fcd_handle* h, int l) {
    return reinterpret_cast<T*>(static_cast<char*>(h->buf.scratch) + h->plan.off_t[l]);
}

template <typename T>
int fine_mode(const fcd::PotLevel<T>& L0) {
    return L0.f ? 2 : 1;
}

// n pre-smoothing sweeps of the finest level from the buffer a (F.u or the temporary
// plane), alternating between the two; returns the buffer holding the result.
template <typename T>
T* mg_sweeps(fcd_handle* h, const fcd::PotLevel<T>& F, int mode, T* a, int n) {
    T* b = a == F.u ? mg_temp<T>(h, 0) : F.u;
    const fcd::PotLevel<CT>* none = nullptr;
    for (int s = 0; s < n; ++s) {
        hipEvent_t ev = nullptr;
        const bool timed = h->timer.begin(h->stream, &ev);
        fcd::launch_mg_smooth_tile<T, CT>(F, a, b, none, mode, nullptr, 1, h->stream);
        if (timed) h->timer.end(h->stream, TK_SMOOTH0, ev);
        std::swap(a, b);
    }
    return a;
}

// Coarse level l >= 1: the restriction from level l-1 (u = its pre-smoothed iterate
// Fp.u, right-hand side by fmode) fused with the level's pre-smoothing (MG_COARSE_INNER
// tile sweeps from a zero correction, one launch); returns the buffer holding the result.
template <typename TF>
CT* mg_restrict_presmooth(fcd_handle* h, const fcd::PotLevel<TF>& Fp, int fmode, int l) {
    const fcd::PotLevel<CT> F = coarse_level(h, l);
    CT* b = mg_temp<CT>(h, l);
    fcd::launch_mg_restrict_smooth<TF, CT>(Fp, F, fmode, b, MG_COARSE_INNER, h->stream);
    return b;
}

// Prolongation of level l+1's correction fused with the first post-smoothing launch, from
// the pre-smoothed iterate `cur`; the result ends in F.u.  The finest level takes
// pot_smooth launches of one sweep each (each sweep sees its neighbours' latest values,
// which a second sweep inside one tile launch would not), a coarse level one launch of
// MG_COARSE_INNER sweeps: on the latency-bound coarse levels a launch costs more than the
// cycles a second one saves, on the finest level the heavier smoothing pays.
template <typename T>
void mg_postsmooth(fcd_handle* h, const fcd::PotLevel<T>& F, int l, int mode, T* cur, const fcd::PotLevel<CT>& Cl) {
    T* other = cur == F.u ? mg_temp<T>(h, l) : F.u;
    const int nu = l == 0 ? std::max(1, h->prm.pot_smooth) : 1;
    const fcd::PotLevel<CT>* none = nullptr;
    for (int s = 0; s < nu; ++s) {
        hipEvent_t ev = nullptr;
        const bool timed = l == 0 && s == 0 && h->timer.begin(h->stream, &ev);
        fcd::launch_mg_smooth_tile<T, CT>(F, cur, other, s == 0 ? &Cl : none, mode, nullptr,
                                          l == 0 ? 1 : MG_COARSE_INNER, h->stream);
        if (timed) h->timer.end(h->stream, TK_POST0, ev);
        std::swap(cur, other);
    }
    if (cur != F.u)
        (void)hipMemcpy2DAsync(F.u, F.pitch * sizeof(T), cur, F.pitch * sizeof(T), F.nx * sizeof(T), F.ny,
                               hipMemcpyDeviceToDevice, h->stream);
}

// Everything of a V-cycle after the finest level's pre-smoothing, whose result is cur0.
template <typename T>
void vcycle_rest(fcd_handle* h, const fcd::PotLevel<T>& L0, T* cur0) {
    const int L = h->plan.levels;
    const bool tail = h->plan.tail < L;
    const int gend = tail ? h->plan.tail : L - 1;  // levels [0, gend) are smoothed by tiles
    CT* cur[MAX_LEVELS] = {};
    for (int l = 1; l < gend; ++l) {
        if (l == 1) {
            fcd::PotLevel<T> Fp = L0;
            Fp.u = cur0;
            cur[l] = mg_restrict_presmooth<T>(h, Fp, fine_mode(L0), l);
        } else {
            fcd::PotLevel<CT> Fp = coarse_level(h, l - 1);
            Fp.u = cur[l - 1];
            cur[l] = mg_restrict_presmooth<CT>(h, Fp, 0, l);
        }
    }
    if (gend == 1) {
        fcd::PotLevel<T> F = L0;
        F.u = cur0;
        fcd::launch_mg_restrict_tile<T, CT>(F, coarse_level(h, 1), fine_mode(L0), h->stream);
    } else {
        fcd::PotLevel<CT> F = coarse_level(h, gend - 1);
        F.u = cur[gend - 1];
        fcd::launch_mg_restrict_tile<CT, CT>(F, coarse_level(h, gend), 0, h->stream);
    }
    if (tail) {
        fcd::MgTail<CT> tl{};
        tl.n = L - h->plan.tail;
        for (int k = 0; k < tl.n; ++k) tl.lv[k] = coarse_level(h, h->plan.tail + k);
        tl.nu1 = tl.nu2 = 1;  // two damped Jacobi sweeps each way
        tl.coarse_sweeps = coarse_sweeps(h, tl.lv[tl.n - 1].ny);
        tl.omega = CT(sor_omega_opt(tl.lv[tl.n - 1].ny));
        fcd::launch_mg_tail<CT>(tl, h->stream);
    } else {
        coarse_solve<CT>(h, coarse_level(h, L - 1), false);
    }
    for (int l = gend - 1; l >= 1; --l)
        mg_postsmooth<CT>(h, coarse_level(h, l), l, 0, cur[l], coarse_level(h, l + 1));
    mg_postsmooth<T>(h, L0, 0, fine_mode(L0), cur0, coarse_level(h, 1));
}

// One full iteration: a V-cycle, or the coarse sweeps on a single-level hierarchy.
template <typename T>
void vcycle(fcd_handle* h, const fcd::PotLevel<T>& L0) {
    if (h->plan.levels == 1) {
        coarse_solve<T>(h, L0, true);
        return;
    }
    T* cur0 = mg_sweeps<T>(h, L0, fine_mode(L0), L0.u, std::max(1, h->prm.pot_smooth));
    vcycle_rest<T>(h, L0, cur0);
}

// Iterate (SOR sweeps or V-cycles) on the finest-level problem L0 until
// max |residual| <= max(thr0, rounding floor) or max_iters; the coarse mu hierarchy
// must already hold the restriction of L0's mu.  defer_from: iterations of a previous
// comparable solve (the first residual test is deferred past all but one of them).
template <typename T>
fcd_status iterate_level0(fcd_handle* h, const fcd::PotLevel<T>& L0, double thr0, int max_iters, int defer_from,
                          int* iters_out, double* resid_out) {
    const bool mg = h->prm.pot_solver == FCD_SOLVER_MG && h->plan.levels > 1;
    const int every = mg ? 1 : h->prm.pot_check_every;
    const T omega = T(h->prm.pot_omega > 0.0 ? h->prm.pot_omega : sor_omega_opt(L0.ny));
    enum { G_CYCLE = 1, G_REST = 2 };
    auto one = [&]() {
        hipEvent_t ev = nullptr;
        const bool timed = h->timer.begin(h->stream, &ev);
        if (mg)
            (void)run_graph(h, L0.u, L0.f, G_CYCLE, [&]() { vcycle<T>(h, L0); });
        else if (h->prm.pot_solver == FCD_SOLVER_MG)
            vcycle<T>(h, L0);
        else
            fcd::launch_pot_sweep<T>(L0, omega, h->stream);
        if (timed) h->timer.end(h->stream, TK_ITER, ev);
    };
    // SOR: the residual is tested before iterating and then every pot_check_every
    // iterations, except that the first test is deferred past the iterations the
    // previous comparable solve needed minus one: consecutive steps need similar counts,
    // and each test costs a host round trip.  Multigrid: the residual of the iterate
    // entering every V-cycle is tested, reduced by the cycle's first smoothing kernel; the
    // host waits for it before launching the rest of the cycle (the same decisions as a
    // time step's solve decided on the device, step_solve_collide).
    int it = 0;
    const int defer = !mg && defer_from > 1 ? defer_from - 1 : 0;
    if (defer > 0 && defer <= max_iters) {
        for (int s = 0; s < defer; ++s) one();
        it = defer;
    }
    auto thr_of = [&](double sc) { return std::max(thr0, resid_floor_factor<T>() * sc); };
    double r = 0.0, scale = 0.0;
    fcd_status st = FCD_OK;
    if (mg) {
        const int mode = fine_mode(L0);
        T* const t0 = mg_temp<T>(h, 0);
        const fcd::PotLevel<CT>* none = nullptr;
        for (;;) {
            // the test: the first pre-smoothing sweep (F.u into the temporary plane) reduces
            // its input's residual; F.u is the accepted iterate when it passes
            hipEvent_t ev = nullptr;
            bool timed = h->timer.begin(h->stream, &ev);
            const int slot = h->res_slot;
            fcd::launch_mg_smooth_tile<T, CT>(L0, L0.u, t0, none, mode, res_slot_ptr(h, slot), 1, h->stream,
                                              res_slot_ptr(h, 1 - slot));
            h->res_slot = 1 - slot;
            if (timed) h->timer.end(h->stream, TK_RESID, ev);
            // slot A: words 0-2 = (r, scale, flag); slot B: words 2-4 = (flag, r, scale)
            st = hip_check(hipMemcpyAsync(h->host, slot ? div_word(h) : res_slot_ptr(h, 0), 3 * sizeof(double),
                                          hipMemcpyDeviceToHost, h->stream),
                           "residual copy");
            if (!st) st = hip_check(hipStreamSynchronize(h->stream), "residual sync");
            if (st) return st;
            const int o = slot ? 1 : 0;
            std::memcpy(&r, h->host + o, sizeof(double));
            std::memcpy(&scale, h->host + o + 1, sizeof(double));
            {
                unsigned long long w;
                std::memcpy(&w, h->host + (slot ? 0 : 2), sizeof(w));
                st = divergence_status(w, u_limit_of(h->prm), "divergence guard");
                if (st) return st;
            }
            if (r <= thr_of(scale)) break;
            if (r != r) {
                h->last_resid = r;
                return fail(FCD_ERR_DIVERGED, "potential residual is NaN");
            }
            if (it >= max_iters) break;
            timed = h->timer.begin(h->stream, &ev);
            st = run_graph(h, L0.u, L0.f, G_REST, [&]() {
                T* cur0 = mg_sweeps<T>(h, L0, mode, t0, std::max(1, h->prm.pot_smooth) - 1);
                vcycle_rest<T>(h, L0, cur0);
            });
            if (timed) h->timer.end(h->stream, TK_ITER, ev);
            if (st) return st;
            ++it;
        }
    } else {
        st = read_residual<T>(h, L0, &r, &scale);
        if (st) return st;
        while (!(r <= thr_of(scale))) {
            if (r != r) {
                h->last_resid = r;
                return fail(FCD_ERR_DIVERGED, "potential residual is NaN");
            }
            if (it >= max_iters) break;
            const int m = every < max_iters - it ? every : max_iters - it;
            for (int s = 0; s < m; ++s) one();
            st = hip_check(hipGetLastError(), "potential launch");
            if (st) return st;
            it += m;
            st = read_residual<T>(h, L0, &r, &scale);
            if (st) return st;
        }
    }
    h->timer.resolve();
    h->sweeps += it;
    h->last_resid = r;
    if (iters_out) *iters_out = it;
    if (resid_out) *resid_out = r;
    if (!(r <= thr_of(scale))) return fail(FCD_ERR_NOT_CONVERGED, "potential solve reached max_iters");
    return FCD_OK;
}

// Potential solve on the current mu_r plane, warm-started from the stored psi'.

// Wait until the GPU has published the outcome of every collide-and-stream enqueued so far
// (the gated kernel's first lane stores the mirror's seq last); the stream is queried now
// and then so that an asynchronous error ends the wait.
fcd_status wait_decisions(fcd_handle* h) {
    const volatile unsigned long long* seq = &h->mirror->seq;
    for (unsigned it = 1; *seq < h->seq_want; ++it) {
        if ((it & 4095u) == 0) {
            const hipError_t e = hipStreamQuery(h->stream);
            if (e == hipSuccess && *seq < h->seq_want) {
                h->seq_want = *seq;
                return fail(FCD_ERR_HIP, "a potential solve's outcome did not reach the host");
            }
            if (e != hipSuccess && e != hipErrorNotReady) return hip_check(e, "potential solve outcome wait");
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return FCD_OK;
}

// A multigrid solve of the finest-level problem L0 (ungated; its mu hierarchy restricted)
// without the host waiting inside it.  The residual tests (the finest level's first
// pre-smoothing sweep, reducing its input's residual) write rotating slots and count
// themselves; every kernel of a V-cycle, the pre-smoothing sweeps after the test included,
// reads the preceding test's slot and does nothing when that test passed.  The first test
// and `ahead` V-cycles each followed by its test are launched together, then finish(sg),
// which launches what ends the batch: a kernel that publishes sg (the slots, the count of
// tests that ran, the divergence word) with one lane and, for a time step, the
// collide-and-stream gated on the last test.  The host waits for the publication; the last
// test that ran decides, by the same rule as on the device (converged when max |r| <=
// max(thr0, 16 eps max |C psi'|)); when the solve needs more V-cycles the host adds one
// cycle, its test and finish again at a time.  A test that did not run leaves its slot
// zero (a pass): a test that runs zeroes the slot after its own, one that does not zeroes
// its own, and the publication the slot after the last test launched; at most
// SOLVE_SLOTS - 2 cycles are launched at once, so that no slot is reused before its test is
// published.  The decisions are those of the host-decided loop (a test before every
// V-cycle).  Eager launches: the host runs ahead of the GPU here, and a launch after a
// replayed graph waits several microseconds for the graph to retire.  *done: the solve
// converged (a time step's collision has then run); *cycles, *resid: V-cycles run, the
// deciding test's residual.
template <typename T, typename Finish>
fcd_status solve_on_device(fcd_handle* h, const fcd::PotLevel<T>& L0, double thr0, int max_iters, int ahead,
                           Finish&& finish, int* cycles_out, double* resid_out, bool* done_out) {
    char* scr = static_cast<char*>(h->buf.scratch);
    auto slot = [&](unsigned long long k) {
        return reinterpret_cast<unsigned long long*>(scr + OFF_SLOTS) + 2 * (k % fcd::SOLVE_SLOTS);
    };
    unsigned* const tests = reinterpret_cast<unsigned*>(scr + OFF_TESTS);
    const double ff = resid_floor_factor<T>();
    auto passes = [&](double r, double sc) { return r <= std::max(thr0, ff * sc); };
    auto gate_of = [&](unsigned long long k) { return fcd::ResGate{slot(k), thr0, ff}; };
    const int mode = fine_mode(L0);
    T* const t0 = mg_temp<T>(h, 0);
    const int nu1 = std::max(1, h->prm.pot_smooth);
    const fcd::PotLevel<CT>* none = nullptr;
    ahead = std::max(0, std::min({ahead, max_iters, fcd::SOLVE_SLOTS - 2}));
    // test k (gated on test k - 1 unless it is the solve's first) into slot k, zeroing slot k + 1
    auto test = [&](unsigned long long k, const fcd::PotLevel<T>& L) {
        fcd::launch_mg_smooth_tile<T, CT>(L, L.u, t0, none, mode, slot(k), 1, h->stream, slot(k + 1), tests);
    };
    // the V-cycle after test k and test k + 1, both gated on test k
    auto cycle = [&](unsigned long long k) {
        h->gate = gate_of(k);  // the coarse levels built while it is set carry the gate
        fcd::PotLevel<T> L0g = L0;
        L0g.gate = h->gate;
        vcycle_rest<T>(h, L0g, mg_sweeps<T>(h, L0g, mode, t0, nu1 - 1));
        test(k + 1, L0g);
        h->gate = fcd::ResGate{};
        return hip_check(hipGetLastError(), "potential launch");
    };
    // what ends a batch whose last test is k
    auto fin = [&](unsigned long long k) {
        ++h->seq_want;
        return finish(fcd::StepGate{gate_of(k), slot(0), slot(k + 1), tests, h->mirror, div_word(h), h->seq_want});
    };
    const unsigned long long k0 = h->test_idx;
    test(k0, L0);
    fcd_status st = hip_check(hipGetLastError(), "potential launch");
    unsigned long long first = k0, last = k0;  // the tests of the launches awaiting publication
    for (int c = 0; c < ahead && !st; ++c) st = cycle(last++);
    if (!st) st = fin(last);
    if (!st) st = wait_decisions(h);
    long long run = 0;  // tests of this solve that ran
    double r = 0.0;
    bool done = false;
    while (!st) {
        const fcd::SolveMirror m = *h->mirror;
        if (m.tests < 1 || m.tests > last - first + 1) {
            char msg[160];
            std::snprintf(msg, sizeof(msg), "inconsistent count of potential residual tests: %u ran, %llu launched",
                          m.tests, last - first + 1);
            st = fail(FCD_ERR_HIP, msg);
            break;
        }
        // tests first .. first + tests - 1 ran; the last of them decides
        const unsigned long long k = first + m.tests - 1;
        run += m.tests;
        r = m.r[k % fcd::SOLVE_SLOTS];
        done = passes(r, m.scale[k % fcd::SOLVE_SLOTS]);
        st = divergence_status(m.div, u_limit_of(h->prm), "divergence guard");
        if (st || done) break;
        if (r != r) {
            st = fail(FCD_ERR_DIVERGED, "potential residual is NaN");
            break;
        }
        if (run - 1 >= max_iters) {
            st = fail(FCD_ERR_NOT_CONVERGED, "potential solve reached max_iters");
            break;
        }
        first = last + 1;
        st = cycle(last++);
        if (!st) st = fin(last);
        if (!st) st = wait_decisions(h);
    }
    h->test_idx = last + 1;
    *cycles_out = (int)std::max(0LL, run - 1);
    *resid_out = r;
    *done_out = done;
    return st;
}

// Whether solves of this handle run on the device (solve_on_device): multigrid on a
// hierarchy with the LDS tail; per-kernel timing keeps the host-decided loop, whose
// decisions are the same, so the results are bitwise identical either way.
bool solves_on_device(const fcd_handle* h) {
    return h->prm.pot_solver == FCD_SOLVER_MG && h->plan.levels > 1 && h->plan.tail < h->plan.levels &&
           !h->timer.on;
}

// A time step's potential solve and its collide-and-stream (solve_on_device, the
// collision ending each batch): V-cycles launched ahead one fewer than the previous solve
// needed, at least one (none when it needed none).  *collided: the collide-and-stream has
// run (src -> dst).
template <typename T>
fcd_status step_solve_collide(fcd_handle* h, const fcd::StepConst<T>& P, const T* src, T* dst, bool* collided) {
    restrict_mu_all<T>(h);
    T* const psi = static_cast<T*>(h->buf.psi);
    const T* phi = static_cast<const T*>(h->buf.phi);
    // with collide-only timing, the events of the last collision launched (the earlier ones
    // of the step found the solve unconverged and did nothing)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto collide = [&](const fcd::StepGate& sg) {
        h->timer.drop(e0, e1);
        if (!h->timer.pair_collide(&e0, &e1)) e0 = e1 = nullptr;
        fcd::launch_collide_stream<T>(src, dst, phi, psi, P, div_word(h), h->stream, e0, e1, sg);
        if (h->open_x)
            fcd::launch_open_boundaries<T>(src, dst, phi, psi, P, h->u_in, h->u_out, h->stream, sg.gate);
        return hip_check(hipGetLastError(), "collide-stream launch");
    };
    int cycles = 0;
    double r = 0.0;
    const int ahead = h->pipe_last <= 1 ? h->pipe_last : h->pipe_last - 1;
    const fcd_status st = solve_on_device<T>(h, pot_level<T>(h, 0), h->prm.pot_tol * std::fabs(h->prm.H0),
                                             h->prm.pot_max_iters, ahead, collide, &cycles, &r, collided);
    if (e0 && *collided)
        h->timer.add(TK_COLLIDE, e0, e1);
    else
        h->timer.drop(e0, e1);
    h->sweeps += cycles;
    h->last_iters = cycles;
    h->pipe_last = cycles;
    h->last_resid = r;
    return st;
}

template <typename T>
fcd_status solve_impl(fcd_handle* h, double tol, int max_iters, int* iters_out, double* resid_out) {
    T* psi = static_cast<T*>(h->buf.psi);
    if (iters_out) *iters_out = 0;
    if (h->prm.H0 == 0.0) {  // no applied field: psi' = 0 exactly
        fcd::launch_fill<T>(psi, (long long)h->lat.ny * h->lat.pitch, T(0), h->stream);
        if (resid_out) *resid_out = 0.0;
        h->last_resid = 0.0;
        return hip_check(hipGetLastError(), "fill");
    }
    if (h->prm.pot_solver == FCD_SOLVER_MG) restrict_mu_all<T>(h);
    int it = 0;
    fcd_status st = FCD_OK;
    if (solves_on_device(h)) {
        auto publish = [&](const fcd::StepGate& sg) {
            fcd::launch_solve_publish(sg, h->stream);
            return hip_check(hipGetLastError(), "publication launch");
        };
        double r = 0.0;
        bool done = false;
        st = solve_on_device<T>(h, pot_level<T>(h, 0), tol * std::fabs(h->prm.H0), max_iters,
                                h->last_iters <= 1 ? h->last_iters : h->last_iters - 1, publish, &it, &r, &done);
        h->sweeps += it;
        h->last_resid = r;
        if (resid_out) *resid_out = r;
    } else {
        st = iterate_level0<T>(h, pot_level<T>(h, 0), tol * std::fabs(h->prm.H0), max_iters, h->last_iters, &it,
                               resid_out);
    }
    h->last_iters = it;
    if (iters_out) *iters_out = it;
    return st;
}

template <typename T>
fcd_status step_impl(fcd_handle* h, int nsteps) {
    const fcd::StepConst<T> P = make_const<T>(h);
    T* phi = static_cast<T*>(h->buf.phi);
    for (int n = 0; n < nsteps; ++n) {
        const T* src = static_cast<const T*>(h->buf.dist[h->cur]);
        T* dst = static_cast<T*>(h->buf.dist[1 - h->cur]);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool timed = h->timer.pair(&e0, &e1);
        fcd::launch_phase<T>(src, phi, P, h->stream, e0, e1);
        if (timed) h->timer.add(TK_PHASE, e0, e1);
        fcd_status st = hip_check(hipGetLastError(), "phase launch");
        if (st) return st;
        // quasi-static coupling: the potential is solved on the steps qs = 0, K, 2K, ... since
        // the last state change and held in between (K = pot_every; 0 or 1: every step)
        const int K = std::max(1, h->prm.pot_every);
        if (h->qs % K == 0) {
            if (h->prm.pot_extrapolate && h->prm.H0 != 0.0) {
                // the first solve's start (the initial solve) is not extrapolated from; linear
                // from the third solve, quadratic from the fourth, cubic from the fifth (up to
                // the order pot_extrapolate asks for)
                const int ex = h->prm.pot_extrapolate;
                const int mode = h->hist >= 4 && ex == 3 ? 3 : h->hist >= 3 && ex >= 2 ? 2 : h->hist >= 2 ? 1 : 0;
                T* const p3 = psi_prev<T>(h, 3);
                fcd::launch_psi_history_ring<T>(static_cast<T*>(h->buf.psi), psi_prev<T>(h, 1), psi_prev<T>(h, 2), p3,
                                                h->lat.nx, h->lat.ny, h->lat.pitch, mode, h->stream);
                h->ring = (h->ring + 2) % 3;  // psi'(t-3)'s plane now holds the newest solution
            }
            if (h->prm.H0 != 0.0 && solves_on_device(h)) {
                bool collided = false;
                st = step_solve_collide<T>(h, P, src, dst, &collided);
                if (collided) {
                    ++h->hist;
                    ++h->qs;
                    h->cur = 1 - h->cur;
                    ++h->steps;
                }
                if (st) return st;
                if (h->steps % div_every_of(h->prm) == 0) {
                    st = read_divergence(h);
                    if (st) return st;
                }
                continue;
            }
            st = solve_impl<T>(h, h->prm.pot_tol, h->prm.pot_max_iters, nullptr, nullptr);
            if (st) return st;
            ++h->hist;
        }
        ++h->qs;
        timed = h->timer.pair_collide(&e0, &e1);
        fcd::launch_collide_stream<T>(src, dst, phi, static_cast<const T*>(h->buf.psi), P, div_word(h), h->stream,
                                      e0, e1);
        if (timed) h->timer.add(TK_COLLIDE, e0, e1);
        if (h->open_x)
            fcd::launch_open_boundaries<T>(src, dst, phi, static_cast<const T*>(h->buf.psi), P, h->u_in, h->u_out,
                                           h->stream);
        st = hip_check(hipGetLastError(), "collide-stream launch");
        if (st) return st;
        h->cur = 1 - h->cur;
        ++h->steps;
        if (h->steps % div_every_of(h->prm) == 0) {
            st = read_divergence(h);
            if (st) return st;
        }
    }
    return FCD_OK;
}

#define FCD_DISPATCH(h, call) ((h)->lat.precision == FCD_FP64 ? call<double> : call<float>)

template <typename T>
fcd_status refresh_phase(fcd_handle* h) {
    const fcd::StepConst<T> P = make_const<T>(h);
    fcd::launch_phase<T>(static_cast<const T*>(h->buf.dist[h->cur]), static_cast<T*>(h->buf.phi), P, h->stream);
    return hip_check(hipGetLastError(), "phase launch");
}

template <typename T>
fcd_status moments_impl(fcd_handle* h, unsigned mask, double* out) {
    fcd_status st = refresh_phase<T>(h);
    if (st) return st;
    const fcd::StepConst<T> P = make_const<T>(h);
    fcd::launch_moments<T>(static_cast<const T*>(h->buf.dist[h->cur]), static_cast<const T*>(h->buf.phi),
                           static_cast<const T*>(h->buf.psi), P, mask, out, h->stream);
    if (h->open_x)
        fcd::launch_open_edge_moments<T>(static_cast<const T*>(h->buf.dist[h->cur]),
                                         static_cast<const T*>(h->buf.phi), static_cast<const T*>(h->buf.psi), P,
                                         mask, out, h->stream);
    return hip_check(hipGetLastError(), "moments launch");
}

template <typename T>
fcd_status diag_impl(fcd_handle* h, double out[4]) {
    fcd_status st = refresh_phase<T>(h);
    if (st) return st;
    const fcd::StepConst<T> P = make_const<T>(h);
    char* s = static_cast<char*>(h->buf.scratch);
    double* result = reinterpret_cast<double*>(s + OFF_RESULT);
    fcd::launch_diagnostics<T>(static_cast<const T*>(h->buf.phi), P, reinterpret_cast<double*>(s + OFF_ROWS),
                               reinterpret_cast<double*>(s + OFF_CENT), result, h->stream);
    st = hip_check(hipGetLastError(), "diagnostics launch");
    if (st) return st;
    st = hip_check(hipMemcpyAsync(h->host + 1, result, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                   "diagnostics copy");
    if (st) return st;
    st = hip_check(hipStreamSynchronize(h->stream), "diagnostics sync");
    if (st) return st;
    std::memcpy(out, h->host + 1, 4 * sizeof(double));
    return FCD_OK;
}

template <typename T>
fcd_status extent_impl(fcd_handle* h, double out[6]) {
    fcd_status st = refresh_phase<T>(h);
    if (st) return st;
    const fcd::StepConst<T> P = make_const<T>(h);
    char* s = static_cast<char*>(h->buf.scratch);
    unsigned long long* ly = reinterpret_cast<unsigned long long*>(s + OFF_EXTENT);
    fcd::launch_fill<double>(reinterpret_cast<double*>(ly), 2, 0.0, h->stream);  // +0.0 has all bits zero
    fcd::launch_extent<T>(static_cast<const T*>(h->buf.phi), P, ly, reinterpret_cast<double*>(ly + 2), h->stream);
    st = hip_check(hipGetLastError(), "extent launch");
    if (!st)
        st = hip_check(hipMemcpyAsync(h->host + 8, ly, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                       "extent copy");
    if (!st) st = hip_check(hipStreamSynchronize(h->stream), "extent sync");
    if (st) return st;
    for (int d = 0; d < 2; ++d) {
        unsigned long long bits;
        std::memcpy(&bits, h->host + 8 + d, sizeof(bits));
        const double lyd = __builtin_bit_cast(double, bits);
        const double lxd = h->host[10 + d];
        out[2 + 2 * d] = lyd;
        out[3 + 2 * d] = lxd;
        out[d] = lyd + lxd > 0.0 ? (lyd - lxd) / (lyd + lxd) : 0.0;
    }
    return FCD_OK;
}

template <typename T>
fcd_status breakup_impl(fcd_handle* h, double out[4]) {
    fcd_status st = refresh_phase<T>(h);
    if (st) return st;
    const fcd::StepConst<T> P = make_const<T>(h);
    char* s = static_cast<char*>(h->buf.scratch);
    double* sums = reinterpret_cast<double*>(s + OFF_BREAKUP);
    fcd::launch_breakup_probe<T>(static_cast<const T*>(h->buf.phi), P, reinterpret_cast<double*>(s + OFF_ROWS), sums,
                                 h->stream);
    st = hip_check(hipGetLastError(), "breakup probe launch");
    if (!st)
        st = hip_check(hipMemcpyAsync(h->host + 16, sums, 6 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                       "breakup probe copy");
    if (!st) st = hip_check(hipStreamSynchronize(h->stream), "breakup probe sync");
    if (st) return st;
    const double* v = h->host + 16;
    const double two_pi = 6.283185307179586, nx = h->lat.nx;
    auto angle_x = [&](double c, double sn) {
        const double a = std::atan2(sn, c);
        return (a < 0.0 ? a + two_pi : a) * nx / two_pi;
    };
    out[0] = v[0];
    out[1] = v[0] > 0.0 ? v[1] / v[0] : -1.0;
    out[2] = v[0] > 0.0 ? angle_x(v[2], v[3]) : -1.0;
    out[3] = (v[4] != 0.0 || v[5] != 0.0) ? angle_x(v[4], v[5]) : -1.0;
    return FCD_OK;
}

template <typename T>
fcd_status init_fields_impl(fcd_handle* h, const double* phi1, const double* phi2, const double* ux,
                            const double* uy, const double* ps) {
    fcd::launch_init_fields<T>(static_cast<T*>(h->buf.dist[h->cur]), phi1, phi2, ux, uy, ps, h->lat.nx, h->lat.ny,
                               h->lat.pitch, h->stream);
    fcd::launch_fill<T>(static_cast<T*>(h->buf.psi), (long long)h->lat.ny * h->lat.pitch, T(0), h->stream);
    fcd_status st = hip_check(hipGetLastError(), "init launch");
    return st ? st : clear_divergence(h);
}

template <typename T>
fcd_status init_droplet_impl(fcd_handle* h, double xc, double yc, double rc, double rs) {
    const double nu3 = h->prm.tau[2] / 3.0;
    const double u_scale = h->prm.drive_G / (2.0 * h->prm.rho[2] * nu3);
    if (h->open_x)
        fcd::launch_open_init_droplet<T>(static_cast<T*>(h->buf.dist[h->cur]), h->lat.nx, h->lat.ny, h->lat.pitch, xc,
                                         yc, rc, rs, h->prm.xi, h->u_in, h->stream);
    else
        fcd::launch_init_droplet<T>(static_cast<T*>(h->buf.dist[h->cur]), h->lat.nx, h->lat.ny, h->lat.pitch, xc, yc,
                                    rc, rs, h->prm.xi, u_scale, h->stream);
    fcd::launch_fill<T>(static_cast<T*>(h->buf.psi), (long long)h->lat.ny * h->lat.pitch, T(0), h->stream);
    fcd_status st = hip_check(hipGetLastError(), "init launch");
    return st ? st : clear_divergence(h);
}

template <typename T>
fcd_status copy_out_impl(fcd_handle* h, const void* src, int nplanes, double* out) {
    fcd::launch_to_dense<T>(static_cast<const T*>(src), out, nplanes, h->lat.nx, h->lat.ny, h->lat.pitch, h->stream);
    return hip_check(hipGetLastError(), "copy launch");
}

template <typename T>
fcd_status copy_in_impl(fcd_handle* h, void* dst, int nplanes, const double* in) {
    fcd::launch_from_dense<T>(in, static_cast<T*>(dst), nplanes, h->lat.nx, h->lat.ny, h->lat.pitch, h->stream);
    return hip_check(hipGetLastError(), "copy launch");
}


// ---------------------------------------------------------------------------------
// Batches.
// ---------------------------------------------------------------------------------
constexpr int BT_X = 64;  // tile width of the batched kernels; rows 1, 2, 4 or 8 (shape 0..3)
constexpr int BT_ROWS[fcd::BATCH_SHAPES] = {1, 2, 4, 8};
constexpr int BATCH_MAX_CHANNELS = 65536;

struct BatchLayout {
    std::vector<int> pitch;
    std::vector<size_t> off_d0, off_d1, off_phi, off_psi, off_prev, off_prev2, off_prev3, off_alt;  // state / aux
    std::vector<int> tile0[fcd::BATCH_SHAPES], tiles_x[fcd::BATCH_SHAPES];
    std::vector<int> ctile0[fcd::BATCH_SHAPES], ctiles_x[fcd::BATCH_SHAPES];
    std::vector<int> stile0, stiles_x;  // fused-sweep tiles
    int ntiles[fcd::BATCH_SHAPES] = {}, nctiles[fcd::BATCH_SHAPES] = {}, nstiles = 0;
    size_t state_bytes = 0, aux_bytes = 0, scratch_bytes = 0;
    size_t off_inst = 0, off_tiles[fcd::BATCH_SHAPES] = {}, off_ctiles[fcd::BATCH_SHAPES] = {}, off_stiles = 0;
    size_t off_slist = 0;
    size_t off_res = 0, off_active = 0, off_counts = 0, off_sweeps = 0, off_div = 0;
    size_t off_rows = 0, off_cent = 0, off_result = 0;
    // batched multigrid: every channel's hierarchy (as a single channel's), its FP32 coarse
    // planes from off_mgc[k] on, the descriptors, the job lists and one residual slot
    // (two words) per channel; mg_ok: every channel has a coarse level and a tail
    bool mg_ok = false;
    int mg_lmax = 0;
    std::vector<MgPlan> mg;
    std::vector<size_t> off_mgc;
    size_t off_mgchan = 0, off_mgchan_adj = 0, off_jobs = 0, off_mgres = 0, off_mgcycles = 0;
    std::vector<fcd::MgJob> jobs;
    int fine0 = 0, nfine = 0;                                   // level-0 64 x 16 tiles
    int mu0[4] = {}, nmu[4] = {};                              // mu groups 1..3 (group 0: the fine list)
    int rs0[MAX_LEVELS] = {}, nrs[MAX_LEVELS] = {};            // restriction + pre-smoothing into level l
    int rt00 = 0, nrt0 = 0, rtC0 = 0, nrtC = 0;                // restriction into the tail
    int post0[MAX_LEVELS] = {}, npost[MAX_LEVELS] = {};        // prolongation + post-smoothing of level l
};

// Offsets (relative to a channel's multigrid region) of the FP32 planes mu, u, f of its
// levels 1 .. levels-1 and the smoothers' second plane t of the tiled levels; returns
// the region's size.
size_t mg_region(const MgPlan& p, size_t off_mu[], size_t off_u[], size_t off_f[], size_t off_t[]) {
    size_t off = 0;
    for (int l = 1; l < p.levels; ++l) {
        const size_t plane = align256((size_t)p.ny[l] * p.pitch[l] * sizeof(CT));
        off_mu[l] = off;
        off_u[l] = off + plane;
        off_f[l] = off + 2 * plane;
        off += 3 * plane;
        off_t[l] = 0;
        if (l < p.tail) {
            off_t[l] = off;
            off += plane;
        }
    }
    return off;
}

fcd_status batch_layout(int n, const fcd_lattice* lats, BatchLayout* L) {
    if (n < 1 || n > BATCH_MAX_CHANNELS) return fail(FCD_ERR_ARG, "a batch holds 1 to 65536 channels");
    if (!lats) return fail(FCD_ERR_ARG, "lattices are null");
    const int prec = lats[0].precision;
    int max_ny = 0;
    for (int k = 0; k < n; ++k) {
        fcd_status st = check_lattice(&lats[k]);
        if (st) return st;
        if (lats[k].precision != prec) return fail(FCD_ERR_ARG, "all channels of a batch share one precision");
        if (lats[k].ny > max_ny) max_ny = lats[k].ny;
    }
    const size_t esz = elem_size(prec);
    const int per = (int)(256 / esz);
    for (int k = 0; k < n; ++k) {
        const fcd_lattice& l = lats[k];
        const int pitch = (l.nx + per - 1) / per * per;  // batch pitch: 256-byte rows
        const size_t plane = align256((size_t)l.ny * pitch * esz);
        L->pitch.push_back(pitch);
        L->off_d0.push_back(L->state_bytes);
        L->state_bytes += 27 * plane;
        L->off_d1.push_back(L->state_bytes);
        L->state_bytes += 27 * plane;
        L->off_phi.push_back(L->aux_bytes);
        L->aux_bytes += 3 * plane;
        L->off_psi.push_back(L->aux_bytes);
        L->aux_bytes += plane;
        L->off_prev.push_back(L->aux_bytes);
        L->aux_bytes += plane;
        L->off_prev2.push_back(L->aux_bytes);
        L->aux_bytes += plane;
        L->off_prev3.push_back(L->aux_bytes);
        L->aux_bytes += plane;
        L->off_alt.push_back(L->aux_bytes);
        L->aux_bytes += plane;
        {
            const int sx = (l.nx + fcd::FUSED_X - 1) / fcd::FUSED_X, sy = (l.ny + fcd::FUSED_Y - 1) / fcd::FUSED_Y;
            L->stile0.push_back(L->nstiles);
            L->stiles_x.push_back(sx);
            L->nstiles += sx * sy;
        }
        for (int s = 0; s < fcd::BATCH_SHAPES; ++s) {
            const int ty = BT_ROWS[s];
            const int tx = (l.nx + BT_X - 1) / BT_X, tyc = (l.ny + ty - 1) / ty;
            L->tile0[s].push_back(L->ntiles[s]);
            L->tiles_x[s].push_back(tx);
            L->ntiles[s] += tx * tyc;
            const int cx = ((l.nx + 1) / 2 + BT_X - 1) / BT_X, cy = ((l.ny + 1) / 2 + ty - 1) / ty;
            L->ctile0[s].push_back(L->nctiles[s]);
            L->ctiles_x[s].push_back(cx);
            L->nctiles[s] += cx * cy;
        }
    }
    const size_t inst_sz = prec == FCD_FP64 ? sizeof(fcd::BatchInst<double>) : sizeof(fcd::BatchInst<float>);
    size_t off = 0;
    L->off_inst = off;
    off = align256(off + (size_t)n * inst_sz);
    for (int s = 0; s < fcd::BATCH_SHAPES; ++s) {
        L->off_tiles[s] = off;
        off = align256(off + (size_t)L->ntiles[s] * sizeof(int));
        L->off_ctiles[s] = off;
        off = align256(off + (size_t)L->nctiles[s] * sizeof(int));
    }
    L->off_stiles = off;
    off = align256(off + (size_t)L->nstiles * sizeof(int));
    L->off_slist = off;  // active fused tiles, then their count
    off = align256(off + ((size_t)L->nstiles + 1) * sizeof(int));
    L->off_res = off;  // three sets of residual slots (consecutive tests rotate)
    off = align256(off + 6 * (size_t)n * sizeof(unsigned long long));
    L->off_active = off;  // two buffers of activity flags
    off = align256(off + 2 * (size_t)n * sizeof(int));
    L->off_counts = off;
    off = align256(off + 3 * sizeof(int));
    L->off_sweeps = off;
    off = align256(off + (size_t)n * sizeof(int));
    L->off_div = off;  // per-channel divergence flags
    off = align256(off + (size_t)n * sizeof(unsigned long long));
    L->off_rows = off;
    off = align256(off + (size_t)max_ny * 8 * sizeof(double));
    L->off_cent = off;
    off = align256(off + 32 * sizeof(double));
    L->off_result = off;
    off = align256(off + (size_t)n * 4 * sizeof(double));
    // batched multigrid
    L->mg_ok = true;
    for (int k = 0; k < n; ++k) {
        fcd_lattice lk = lats[k];
        lk.pitch = L->pitch[k];
        L->mg.push_back(make_plan(lk));
        const MgPlan& p = L->mg.back();
        if (p.levels < 2 || p.tail >= p.levels) L->mg_ok = false;
        L->mg_lmax = std::max(L->mg_lmax, p.levels);
    }
    if (L->mg_ok) {
        size_t a_mu[MAX_LEVELS], a_u[MAX_LEVELS], a_f[MAX_LEVELS], a_t[MAX_LEVELS];
        for (int k = 0; k < n; ++k) {
            L->off_mgc.push_back(off);
            off = align256(off + mg_region(L->mg[k], a_mu, a_u, a_f, a_t));
        }
        const size_t chan_sz = prec == FCD_FP64 ? sizeof(fcd::MgChan<double, CT>) : sizeof(fcd::MgChan<float, CT>);
        L->off_mgchan = off;
        off = align256(off + (size_t)n * chan_sz);
        L->off_mgchan_adj = off;  // the batched adjoint's potential problems
        off = align256(off + (size_t)n * chan_sz);
        // job lists, in launch order of a V-cycle
        auto tiles = [&](int k, int l, int sx, int sy) {
            const MgPlan& p = L->mg[k];
            const int tx = (p.nx[l] + sx - 1) / sx, ty = (p.ny[l] + sy - 1) / sy;
            for (int by = 0; by < ty; ++by)
                for (int bx = 0; bx < tx; ++bx) L->jobs.push_back({k, l, bx, by});
        };
        L->fine0 = (int)L->jobs.size();
        for (int k = 0; k < n; ++k) tiles(k, 0, 64, 16);
        L->nfine = (int)L->jobs.size() - L->fine0;
        for (int g = 1; g < 4; ++g) {  // mu of levels 4g+1 .. from level 4g (64 x 16 tiles)
            L->mu0[g] = (int)L->jobs.size();
            for (int k = 0; k < n; ++k)
                if (L->mg[k].levels - 1 > 4 * g) {
                    const size_t first = L->jobs.size();
                    tiles(k, 4 * g, 64, 16);
                    for (size_t q = first; q < L->jobs.size(); ++q) L->jobs[q].l = g;
                }
            L->nmu[g] = (int)L->jobs.size() - L->mu0[g];
        }
        for (int l = 1; l < L->mg_lmax; ++l) {  // coarse 32 x 8 tiles of the tiled levels
            L->rs0[l] = (int)L->jobs.size();
            for (int k = 0; k < n; ++k)
                if (l < L->mg[k].tail) tiles(k, l, 32, 8);
            L->nrs[l] = (int)L->jobs.size() - L->rs0[l];
        }
        L->rt00 = (int)L->jobs.size();
        for (int k = 0; k < n; ++k)
            if (L->mg[k].tail == 1) tiles(k, 0, 64, 16);
        L->nrt0 = (int)L->jobs.size() - L->rt00;
        L->rtC0 = (int)L->jobs.size();
        for (int k = 0; k < n; ++k)
            if (L->mg[k].tail >= 2) tiles(k, L->mg[k].tail - 1, 32, 8);
        L->nrtC = (int)L->jobs.size() - L->rtC0;
        for (int l = 1; l < L->mg_lmax; ++l) {
            L->post0[l] = (int)L->jobs.size();
            for (int k = 0; k < n; ++k)
                if (l < L->mg[k].tail) tiles(k, l, 32, 8);
            L->npost[l] = (int)L->jobs.size() - L->post0[l];
        }
        L->off_jobs = off;
        off = align256(off + L->jobs.size() * sizeof(fcd::MgJob));
        L->off_mgres = off;
        off = align256(off + 2 * (size_t)n * sizeof(unsigned long long));
        L->off_mgcycles = off;
        off = align256(off + (size_t)n * sizeof(int));
    }
    L->scratch_bytes = off;
    return FCD_OK;
}

}  // namespace

struct fcd_batch {
    int n;
    int precision;
    hipStream_t stream;
    std::vector<fcd_lattice> lat;
    std::vector<fcd_params> prm;
    BatchLayout L;
    char* state;
    char* aux;
    char* scratch;
    int cur;
    int hist;
    int qs;  // steps since the initial state (the potential is solved when qs % pot_every == 0)
    int last_iters;
    long long steps;
    long long iters;
    double last_resid;
    double* host;  // pinned: [0..1] the solve counts (three ints), [2..] n x 4 diagnostics or n flags
    // launch schedule: tile shape (rows 1, 2, 4, 8), sweeps per graph-launched block and
    // sweeps per fused SOR launch (0: one launch per colour)
    int shape;
    int block_sweeps;
    int fused;
    // tail fusion: blocks that start at or after tail_after sweeps of a solve use
    // tail_fused sweeps per fused launch instead (0: off)
    int tail_fused, tail_after;
    GraphCache graphs;
    // batched adjoint
    int init_fresh;
    char* adj_work;
    int adj_nsteps, adj_every, adj_from_init;
    std::vector<int> adj_ckpt;  // (last_iters, hist) per checkpoint
    int adj_final_iters, adj_final_hist;
    int adj_solve_iters;        // sweeps of the previous adjoint potential solve
    // batched multigrid for the forward potential (channel 0 asks for FCD_SOLVER_MG and
    // every channel has a hierarchy with a tail)
    bool mg;
    size_t mg_lds;       // dynamic LDS of the batched tail launch (largest channel's tail)
    int mg_last_cycles;  // cycles the previous forward solve needed
    int adj_mg_last_cycles;  // ... and the previous adjoint solve
};

namespace {

// Single-channel view of channel k (for the per-channel utility kernels).
template <typename T>
fcd::StepConst<T> batch_const(const fcd_batch* b, int k) {
    fcd_handle h{};
    h.lat = b->lat[k];
    h.lat.pitch = b->L.pitch[k];
    h.prm = b->prm[k];
    return make_const<T>(&h);
}

template <typename T>
T* bptr(char* base, size_t off) {
    return reinterpret_cast<T*>(base + off);
}

// Blocks of a four-sweep fused launch (about four per compute unit); they stride over the
// list of active tiles, so such a launch late in a solve, when few channels are still
// active, dispatches no more blocks than this.
constexpr int FUSED_GRID = 1024;

fcd::BatchTiles btiles(const fcd_batch* b) {
    fcd::BatchTiles t;
    t.shape = b->shape;
    t.ntiles = b->L.ntiles[b->shape];
    t.nctiles = b->L.nctiles[b->shape];
    t.tiles = reinterpret_cast<const int*>(b->scratch + b->L.off_tiles[b->shape]);
    t.ctiles = reinterpret_cast<const int*>(b->scratch + b->L.off_ctiles[b->shape]);
    t.fused = b->fused;
    t.nstiles = b->L.nstiles;
    t.stiles = reinterpret_cast<const int*>(b->scratch + b->L.off_stiles);
    t.slist = reinterpret_cast<int*>(b->scratch + b->L.off_slist);
    t.scount = t.slist + b->L.nstiles;
    t.sgrid = std::max(1, std::min(b->L.nstiles, FUSED_GRID));
    return t;
}

template <typename T>
fcd::BatchInst<T> make_batch_inst(const fcd_batch* b, int k) {
    fcd::BatchInst<T> I{};
    const fcd_lattice& l = b->lat[k];
    const fcd_params& p = b->prm[k];
    I.P = batch_const<T>(b, k);
    I.dist[0] = bptr<T>(b->state, b->L.off_d0[k]);
    I.dist[1] = bptr<T>(b->state, b->L.off_d1[k]);
    I.phi = bptr<T>(b->aux, b->L.off_phi[k]);
    I.prev = bptr<T>(b->aux, b->L.off_prev[k]);
    I.prev2 = bptr<T>(b->aux, b->L.off_prev2[k]);
    I.prev3 = bptr<T>(b->aux, b->L.off_prev3[k]);
    I.alt = bptr<T>(b->aux, b->L.off_alt[k]);
    I.L0.u = bptr<T>(b->aux, b->L.off_psi[k]);
    I.L0.mu = I.phi + 2 * (long long)I.P.plane;
    I.L0.f = nullptr;
    I.L0.nx = l.nx;
    I.L0.ny = l.ny;
    I.L0.pitch = b->L.pitch[k];
    I.L0.inv_h2 = T(1);
    I.L0.kappa = T(0);
    I.L0.kappa_top = T(0);
    I.L0.H0x = T(p.H0 * std::cos(p.alpha));
    I.L0.H0y = T(p.H0 * std::sin(p.alpha));
    I.omega = T(p.pot_omega > 0.0 ? p.pot_omega : sor_omega_opt(l.ny));
    I.thr = p.pot_tol * std::fabs(p.H0);
    I.has_field = p.H0 != 0.0;
    for (int s = 0; s < fcd::BATCH_SHAPES; ++s) {
        I.tile0[s] = b->L.tile0[s][k];
        I.tiles_x[s] = b->L.tiles_x[s][k];
        I.ctile0[s] = b->L.ctile0[s][k];
        I.ctiles_x[s] = b->L.ctiles_x[s][k];
    }
    I.stile0 = b->L.stile0[k];
    I.stiles_x = b->L.stiles_x[k];
    I.div = reinterpret_cast<unsigned long long*>(b->scratch + b->L.off_div) + k;
    return I;
}

// Reads every channel's divergence flag (waits for the stream); FCD_ERR_DIVERGED names the
// first channel whose flag is set.
fcd_status batch_read_divergence(fcd_batch* b) {
    fcd_status st = hip_check(hipMemcpyAsync(b->host + 2, b->scratch + b->L.off_div,
                                             (size_t)b->n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                             b->stream), "divergence flag copy");
    if (!st) st = hip_check(hipStreamSynchronize(b->stream), "divergence flag sync");
    if (st) return st;
    for (int k = 0; k < b->n; ++k) {
        unsigned long long w;
        std::memcpy(&w, b->host + 2 + k, sizeof(w));
        if (w) return divergence_status(w, u_limit_of(b->prm[k]), "divergence guard, channel " + std::to_string(k));
    }
    return FCD_OK;
}

// Channel k's multigrid descriptor: the single-channel hierarchy of its lattice over the
// batch's planes (psi', mu_r and the second potential plane as the finest level's
// ping-pong plane) and its FP32 coarse planes.
template <typename T>
fcd::MgChan<T, CT> make_mgchan(const fcd_batch* b, int k) {
    fcd::MgChan<T, CT> c{};
    const MgPlan& p = b->L.mg[k];
    const fcd_params& prm = b->prm[k];
    const fcd::BatchInst<T> I = make_batch_inst<T>(b, k);
    c.L0 = I.L0;
    c.t0 = I.alt;
    size_t a_mu[MAX_LEVELS], a_u[MAX_LEVELS], a_f[MAX_LEVELS], a_t[MAX_LEVELS];
    mg_region(p, a_mu, a_u, a_f, a_t);
    char* base = b->scratch + b->L.off_mgc[k];
    for (int l = 1; l < p.levels; ++l) {
        const double hh = double(1 << l);
        fcd::PotLevel<CT>& L = c.C[l];
        L.nx = p.nx[l];
        L.ny = p.ny[l];
        L.pitch = p.pitch[l];
        L.mu = reinterpret_cast<const CT*>(base + a_mu[l]);
        L.u = reinterpret_cast<CT*>(base + a_u[l]);
        L.f = reinterpret_cast<CT*>(base + a_f[l]);
        L.inv_h2 = CT(1.0 / (hh * hh));
        L.kappa = CT((hh - 1.0) / (hh + 1.0));
        L.kappa_top = CT(p.kappa_top[l]);
        c.t[l] = l < p.tail ? reinterpret_cast<CT*>(base + a_t[l]) : nullptr;
    }
    c.tl.n = p.levels - p.tail;
    for (int q = 0; q < c.tl.n; ++q) {
        c.tl.lv[q] = c.C[p.tail + q];
        c.dv.inv[q] = (unsigned)(((1ull << 32) + p.nx[p.tail + q] - 1) / p.nx[p.tail + q]);
    }
    c.tl.nu1 = c.tl.nu2 = 1;
    const int nyc = p.ny[p.levels - 1], cs = prm.pot_coarse_sweeps;
    c.tl.coarse_sweeps = cs < 0 ? -cs : cs * std::max(1, nyc / 2);
    c.tl.omega = CT(sor_omega_opt(nyc));
    for (int g = 0; 4 * g + 1 < p.levels && g < 4; ++g) {
        fcd::MuLevels<CT>& M = c.mu4[g];
        M.n = std::min(4, p.levels - 1 - 4 * g);
        for (int q = 0; q < M.n; ++q) {
            const fcd::PotLevel<CT>& Lq = c.C[4 * g + 1 + q];
            M.mu[q] = const_cast<CT*>(Lq.mu);
            M.nx[q] = Lq.nx;
            M.ny[q] = Lq.ny;
            M.pitch[q] = Lq.pitch;
        }
    }
    c.levels = p.levels;
    c.tail = p.tail;
    c.thr = prm.pot_tol * std::fabs(prm.H0);
    return c;
}

template <typename T>
fcd_status batch_upload_mg(fcd_batch* b) {
    if (!b->L.mg_ok) return FCD_OK;
    std::vector<fcd::MgChan<T, CT>> ch(b->n);
    b->mg_lds = 0;
    for (int k = 0; k < b->n; ++k) {
        ch[k] = make_mgchan<T>(b, k);
        b->mg_lds = std::max(b->mg_lds, fcd::mg_tail_lds_bytes<CT>(ch[k].tl));
    }
    return hip_check(hipMemcpy(b->scratch + b->L.off_mgchan, ch.data(), ch.size() * sizeof(ch[0]),
                               hipMemcpyHostToDevice), "multigrid descriptor upload");
}

// Re-uploads the channel descriptors after a parameter change (after the batch's queued
// work, which reads them, has finished).
template <typename T>
fcd_status batch_upload_inst(fcd_batch* b) {
    std::vector<fcd::BatchInst<T>> inst(b->n);
    for (int k = 0; k < b->n; ++k) inst[k] = make_batch_inst<T>(b, k);
    fcd_status st = hip_check(hipStreamSynchronize(b->stream), "batch sync");
    if (!st)
        st = hip_check(hipMemcpy(b->scratch + b->L.off_inst, inst.data(), inst.size() * sizeof(inst[0]),
                                 hipMemcpyHostToDevice), "descriptor upload");
    if (!st) st = batch_upload_mg<T>(b);
    return st;
}

template <typename T>
fcd_status batch_upload(fcd_batch* b) {
    std::vector<fcd::BatchInst<T>> inst(b->n);
    std::vector<int> tiles[fcd::BATCH_SHAPES], ctiles[fcd::BATCH_SHAPES], stiles(b->L.nstiles);
    for (int s = 0; s < fcd::BATCH_SHAPES; ++s) {
        tiles[s].resize(b->L.ntiles[s]);
        ctiles[s].resize(b->L.nctiles[s]);
    }
    for (int k = 0; k < b->n; ++k) {
        fcd::BatchInst<T>& I = inst[k];
        const fcd_lattice& l = b->lat[k];
        I = make_batch_inst<T>(b, k);
        for (int s = 0; s < fcd::BATCH_SHAPES; ++s) {
            const int ty = BT_ROWS[s];
            const int nt = (l.nx + BT_X - 1) / BT_X * ((l.ny + ty - 1) / ty);
            for (int t = 0; t < nt; ++t) tiles[s][I.tile0[s] + t] = k;
            const int nc = ((l.nx + 1) / 2 + BT_X - 1) / BT_X * (((l.ny + 1) / 2 + ty - 1) / ty);
            for (int t = 0; t < nc; ++t) ctiles[s][I.ctile0[s] + t] = k;
        }
        const int ns = I.stiles_x * ((l.ny + fcd::FUSED_Y - 1) / fcd::FUSED_Y);
        for (int t = 0; t < ns; ++t) stiles[I.stile0 + t] = k;
    }
    fcd_status st = hip_check(hipMemcpy(b->scratch + b->L.off_inst, inst.data(), inst.size() * sizeof(inst[0]),
                                        hipMemcpyHostToDevice), "descriptor upload");
    for (int s = 0; s < fcd::BATCH_SHAPES && !st; ++s) {
        st = hip_check(hipMemcpy(b->scratch + b->L.off_tiles[s], tiles[s].data(), tiles[s].size() * sizeof(int),
                                 hipMemcpyHostToDevice), "tile table upload");
        if (!st)
            st = hip_check(hipMemcpy(b->scratch + b->L.off_ctiles[s], ctiles[s].data(),
                                     ctiles[s].size() * sizeof(int), hipMemcpyHostToDevice), "tile table upload");
    }
    if (!st)
        st = hip_check(hipMemcpy(b->scratch + b->L.off_stiles, stiles.data(), stiles.size() * sizeof(int),
                                 hipMemcpyHostToDevice), "tile table upload");
    if (st) return st;
    // an empty list of active fused tiles until the first decision kernel
    st = hip_check(hipMemset(b->scratch + b->L.off_slist, 0, ((size_t)b->L.nstiles + 1) * sizeof(int)),
                   "active tile list");
    if (st) return st;
    // residual slots start (and are always left) at zero
    st = hip_check(hipMemset(b->scratch + b->L.off_res, 0, 6 * (size_t)b->n * sizeof(unsigned long long)),
                   "residual slots");
    if (st || !b->L.mg_ok) return st;
    st = batch_upload_mg<T>(b);
    if (!st)
        st = hip_check(hipMemcpy(b->scratch + b->L.off_jobs, b->L.jobs.data(), b->L.jobs.size() * sizeof(fcd::MgJob),
                                 hipMemcpyHostToDevice), "multigrid job upload");
    if (!st)
        st = hip_check(hipMemset(b->scratch + b->L.off_mgres, 0, 2 * (size_t)b->n * sizeof(unsigned long long)),
                       "multigrid residual slots");
    if (!st)
        st = hip_check(hipMemset(b->scratch + b->L.off_mgcycles, 0, (size_t)b->n * sizeof(int)),
                       "multigrid cycle counts");
    return st;
}

template <typename T>
const fcd::BatchInst<T>* binst(const fcd_batch* b) {
    return reinterpret_cast<const fcd::BatchInst<T>*>(b->scratch + b->L.off_inst);
}

int check_interval(const fcd_batch* b) { return std::max(1, b->prm[0].pot_check_every); }

// Sweeps per fused launch: f = 1 or 2 need a test interval that is a multiple of 2 f (an
// even number of launches per interval, so every test finds the potential in its own
// plane); f = 4 needs a multiple of 4 (its launches copy a channel stopped on odd parity
// back to its plane); f = 0 (one launch per colour) is always allowed.
bool fused_allowed(const fcd_batch* b, int f) {
    const int c = check_interval(b);
    return f == 0 || ((f == 1 || f == 2) && c % (2 * f) == 0) || (f == 4 && c % 4 == 0);
}

// Sweeps per fused launch of the graph block that starts after `done` sweeps of a
// solve: the tail fusion from tail_after sweeps on (when the block size allows it: an
// even number of launches per block), else the schedule's.  Every choice gives the same
// states, so this only trades the repeated halo work of deep fusion, which costs most
// while many channels are active, against launches, which dominate once few are.
int block_fusion(const fcd_batch* b, int done) {
    if (b->fused > 0 && b->tail_fused > 0 && done >= b->tail_after && b->block_sweeps % (2 * b->tail_fused) == 0)
        return b->tail_fused;
    return b->fused;
}

// The problem a batched potential solve works on: the descriptors (u, f, mu, thresholds)
// and, for relative thresholds, per-channel scales on the device.
template <typename T>
struct BatchProblem {
    const fcd::BatchInst<T>* inst;
    const unsigned long long* scale;  // nullptr: absolute thresholds of the descriptors
    double rel_tol;
    int* last_iters;                  // sweeps the previous solve of this problem needed
    bool rhs_plane;                   // the descriptors carry a right-hand-side plane
};

template <typename T>
BatchProblem<T> forward_problem(fcd_batch* b) {
    return {binst<T>(b), nullptr, 0.0, &b->last_iters, false};
}

// A block of `block_sweeps` SOR sweeps with a device-side convergence test after every
// `check` sweeps (block_sweeps is a multiple of check and of twice the sweeps per fused
// launch, so a block has an even number of fused launches and ends with the potential
// in its own plane).  Fused launches alternate the potential between its plane and the
// second plane.  With fused launches a test's decision is taken by the next launch,
// which may itself be a test: consecutive tests rotate over three sets of residual slots
// (the test's, the one being decided, and the one the deciding launch clears for the
// next test that is not its own), and a deciding launch writes the other of the two
// flag buffers.  The block's last test is decided by the decision kernel, which leaves
// every set at zero, both flag buffers equal, and the counts the host reads.
template <typename T>
void batch_block(fcd_batch* b, const BatchProblem<T>& P, int fused) {
    fcd::BatchTiles t = btiles(b);
    t.fused = fused;
    const int n = b->n;
    int* active = bptr<int>(b->scratch, b->L.off_active);
    const int check = check_interval(b);
    unsigned long long* res = bptr<unsigned long long>(b->scratch, b->L.off_res);
    unsigned long long* rset[3] = {res, res + 2 * (size_t)n, res + 4 * (size_t)n};
    int* counts = bptr<int>(b->scratch, b->L.off_counts);
    int* sweeps = bptr<int>(b->scratch, b->L.off_sweeps);
    const int per = t.fused > 0 ? t.fused : 1;
    int parity = 0, tests = 0, cur = 0;
    bool pending = false;  // a test whose decision has not been taken yet
    for (int s = per; s <= b->block_sweeps; s += per) {
        const bool test = s % check == 0;
        if (t.fused > 0) {
            fcd::BatchDecide dec{};
            if (pending)
                dec = {rset[(tests - 1) % 3], rset[(test ? tests + 1 : tests) % 3], P.scale, P.rel_tol, sweeps, check};
            fcd::launch_batch_sweep_fused<T>(P.inst, t, active + cur * n, active + (1 - cur) * n, parity,
                                             P.rhs_plane, test ? rset[tests % 3] : nullptr, dec, b->stream);
            if (pending) cur = 1 - cur;
            parity ^= 1;
            pending = test;
            tests += test;
        } else {
            fcd::launch_batch_sweep<T>(P.inst, t, active, b->stream);
            if (test)
                fcd::launch_batch_check<T>(P.inst, t, n, res, active, counts, P.scale, P.rel_tol, sweeps, check,
                                           b->stream);
        }
    }
    if (pending)
        fcd::launch_batch_decide<T>(P.inst, t, n, rset[(tests - 1) % 3], rset[tests % 3], rset[(tests + 1) % 3], active,
                                    cur, counts, P.scale, P.rel_tol, sweeps, check, b->stream);
}

template <typename T>
fcd_status batch_read_counts(fcd_batch* b, int* active_count, int* needed = nullptr) {
    int* counts = bptr<int>(b->scratch, b->L.off_counts);
    fcd_status st = hip_check(hipMemcpyAsync(b->host, counts, 3 * sizeof(int), hipMemcpyDeviceToHost, b->stream),
                              "batch count copy");
    if (!st) st = hip_check(hipStreamSynchronize(b->stream), "batch count sync");
    if (st) return st;
    int c[3];
    std::memcpy(c, b->host, sizeof(c));
    if (c[1] > 0) return fail(FCD_ERR_DIVERGED, "a channel's potential residual is NaN");
    *active_count = c[0];
    if (needed) *needed = c[2];
    return FCD_OK;
}

// Potential solves of every channel: all channels start active; the first test runs
// before any sweep; blocks of sweeps (HIP graphs) follow until no channel is active.
// The host reads the active count after each block, except that it launches the blocks
// the previous solve needed minus one without reading.  Which sweeps a channel receives
// is decided on the device, so the result does not depend on the block size.
template <typename T>
fcd_status batch_solve(fcd_batch* b, const BatchProblem<T>& P, int max_iters) {
    const fcd::BatchTiles t = btiles(b);
    int* active = bptr<int>(b->scratch, b->L.off_active);
    fcd::launch_fill<int>(active, 2 * b->n, 1, b->stream);
    fcd::launch_batch_check<T>(P.inst, t, b->n, bptr<unsigned long long>(b->scratch, b->L.off_res), active,
                               bptr<int>(b->scratch, b->L.off_counts), P.scale, P.rel_tol,
                               bptr<int>(b->scratch, b->L.off_sweeps), 0, b->stream);
    fcd_status st = hip_check(hipGetLastError(), "batch check launch");
    if (st) return st;
    int left = 1, it = 0;
    const int G = b->block_sweeps;
    // blocks launched without a read: as many as the previous solve took, less one; when the
    // first read after them finds every channel converged, the solve may have needed fewer,
    // so the next solve is given one block fewer (else the count could only ever grow)
    const int blind0 = *P.last_iters > G ? (*P.last_iters + G - 1) / G - 1 : 0;
    int blind = blind0;
    bool first_read = true, overshoot = false;
    if (blind == 0) {
        st = batch_read_counts<T>(b, &left);
        if (st) return st;
        first_read = false;
    }
    while (left > 0) {
        if (it >= max_iters) break;
        const int f = block_fusion(b, it);
        st = run_graph_on(b->graphs, b->stream, false, P.inst, nullptr, ((f * 8 + b->shape) << 24) + G,
                          [&]() { batch_block<T>(b, P, f); });
        if (st) return st;
        it += G;
        if (blind > 0) {
            --blind;
            continue;
        }
        st = batch_read_counts<T>(b, &left);
        if (st) return st;
        if (first_read) overshoot = blind0 > 0 && left == 0;
        first_read = false;
    }
    b->iters += it;
    *P.last_iters = overshoot ? it - G : it;
    b->last_resid = 0.0;
    if (left > 0) return fail(FCD_ERR_NOT_CONVERGED, "a channel's potential solve reached pot_max_iters");
    return FCD_OK;
}

// Batched multigrid.  One V-cycle of every active channel (the single-channel cycle:
// pot_smooth finest sweeps, of which the first also reduces its input's residual into
// the channel's slot, restriction with pre-smoothing down the tiled levels, the tail,
// prolongation with post-smoothing back up, pot_smooth finest sweeps), with the
// convergence decision taken on the device after the first sweep: a channel whose input
// already meets its threshold stops there (its psi' plane untouched, the sweep's output
// in the second plane discarded), so every channel receives exactly the cycles its own
// single-channel solve would, whatever the batch.
constexpr int BMG_INNER = 2;            // tile sweeps per launch on the tiled coarse levels
constexpr int BMG_BLOCK_CYCLES = 2;     // V-cycles per graph launch

// A batched potential problem: the descriptors (finest level's iterate, right-hand side from
// the field or from a plane), the thresholds (the descriptors' absolute ones, or rel_tol times
// per-channel scales on the device) and the cycle count of its previous solve.
template <typename T>
struct BmgProblem {
    const fcd::MgChan<T, CT>* ch;
    bool rhs_plane;
    const unsigned long long* scale;
    double rel_tol;
    int* last_cycles;
};

template <typename T>
BmgProblem<T> bmg_forward(fcd_batch* b) {
    return {reinterpret_cast<const fcd::MgChan<T, CT>*>(b->scratch + b->L.off_mgchan), false, nullptr, 0.0,
            &b->mg_last_cycles};
}

template <typename T>
void bmg_cycle(fcd_batch* b, const BmgProblem<T>& P) {
    const BatchLayout& L = b->L;
    const fcd::MgChan<T, CT>* ch = P.ch;
    const bool rp = P.rhs_plane;
    const auto* jobs = reinterpret_cast<const fcd::MgJob*>(b->scratch + L.off_jobs);
    int* active = bptr<int>(b->scratch, b->L.off_active);
    unsigned long long* res = bptr<unsigned long long>(b->scratch, L.off_mgres);
    int* cycles = bptr<int>(b->scratch, L.off_mgcycles);
    int* counts = bptr<int>(b->scratch, L.off_counts);
    hipStream_t st = b->stream;
    const int nu = std::max(1, b->prm[0].pot_smooth);
    const fcd::MgJob* fine = jobs + L.fine0;
    // pre-smoothing: sweep q reads the plane the previous one wrote (q even: psi' -> second)
    int cur = 0;  // plane holding the current finest iterate: 0 psi', 1 the second plane
    for (int q = 0; q < nu; ++q) {
        fcd::launch_bmg_smooth_fine<T, CT>(ch, fine, L.nfine, active, cur, false, rp, q == 0 ? res : nullptr, st);
        cur = 1 - cur;
        if (q == 0)
            fcd::launch_bmg_decide<T, CT>(ch, b->n, res, active, cycles, counts, resid_floor_factor<T>(), P.scale,
                                          P.rel_tol, st);
    }
    for (int l = 1; l < L.mg_lmax; ++l)
        if (L.nrs[l])
            fcd::launch_bmg_restrict_smooth<T, CT>(ch, jobs + L.rs0[l], L.nrs[l], active, l, cur, BMG_INNER, rp, st);
    if (L.nrt0) fcd::launch_bmg_restrict_tail<T, CT>(ch, jobs + L.rt00, L.nrt0, active, true, cur, rp, st);
    if (L.nrtC) fcd::launch_bmg_restrict_tail<T, CT>(ch, jobs + L.rtC0, L.nrtC, active, false, cur, rp, st);
    fcd::launch_bmg_tail<T, CT>(ch, b->n, b->mg_lds, active, st);
    for (int l = L.mg_lmax - 1; l >= 1; --l)
        if (L.npost[l]) fcd::launch_bmg_post_coarse<T, CT>(ch, jobs + L.post0[l], L.npost[l], active, BMG_INNER, st);
    for (int q = 0; q < nu; ++q) {
        fcd::launch_bmg_smooth_fine<T, CT>(ch, fine, L.nfine, active, cur, q == 0, rp, nullptr, st);
        cur = 1 - cur;
    }
    if (cur) fcd::launch_bmg_copy_fine<T, CT>(ch, fine, L.nfine, active, st);
}

// Potential solves of every channel by batched V-cycles: the coarse mu of every level,
// then graph launches of BMG_BLOCK_CYCLES cycles until no channel is active; the host
// reads the active count after each launch, except for the launches the previous solve
// needed minus one.
template <typename T>
fcd_status batch_solve_mg(fcd_batch* b, const BmgProblem<T>& P, int max_iters) {
    const BatchLayout& L = b->L;
    const fcd::MgChan<T, CT>* ch = P.ch;
    const auto* jobs = reinterpret_cast<const fcd::MgJob*>(b->scratch + L.off_jobs);
    fcd::launch_bmg_mu4<T, CT>(ch, jobs + L.fine0, L.nfine, 0, b->stream);
    for (int g = 1; g < 4; ++g)
        if (L.nmu[g]) fcd::launch_bmg_mu4<T, CT>(ch, jobs + L.mu0[g], L.nmu[g], g, b->stream);
    int* counts = bptr<int>(b->scratch, L.off_counts);
    fcd::launch_fill<int>(bptr<int>(b->scratch, L.off_active), b->n, 1, b->stream);
    fcd::launch_fill<int>(counts + 2, 1, 0, b->stream);
    fcd_status st = hip_check(hipGetLastError(), "batch multigrid launch");
    if (st) return st;
    // graph launches without a read: as many as the previous solve's cycles need, less one
    // (the decision kernel counts the cycles a solve needs, however many were launched)
    const int G = BMG_BLOCK_CYCLES;
    int blind = *P.last_cycles > G ? (*P.last_cycles + G - 1) / G - 1 : 0;
    int left = 1, it = 0, needed = 0;
    while (left > 0) {
        if (it >= max_iters) break;
        st = run_graph_on(b->graphs, b->stream, false, ch, jobs, (7 << 24) + std::max(1, b->prm[0].pot_smooth),
                          [&]() {
                              for (int c = 0; c < G; ++c) bmg_cycle<T>(b, P);
                          });
        if (st) return st;
        it += G;
        if (blind > 0) {
            --blind;
            continue;
        }
        st = batch_read_counts<T>(b, &left, &needed);
        if (st) return st;
    }
    b->iters += it;
    *P.last_cycles = needed;
    b->last_resid = 0.0;
    if (left > 0) return fail(FCD_ERR_NOT_CONVERGED, "a channel's potential solve reached pot_max_iters");
    return FCD_OK;
}

template <typename T>
fcd_status batch_step_impl(fcd_batch* b, int nsteps) {
    const fcd_params& p0 = b->prm[0];
    for (int n = 0; n < nsteps; ++n) {
        const fcd::BatchTiles t = btiles(b);
        fcd::launch_batch_phase<T>(binst<T>(b), t, b->cur, b->stream);
        fcd_status st = hip_check(hipGetLastError(), "batch phase launch");
        if (st) return st;
        if (b->qs % std::max(1, p0.pot_every) == 0) {  // quasi-static coupling, as fcd_step
            if (p0.pot_extrapolate) {
                // linear from the third solve; with the multigrid quadratic from the fourth and
                // cubic from the fifth, up to pot_extrapolate (in SOR batches the higher orders'
                // coefficients amplify the FP32 solve's rounding, so they start linearly)
                const int ex = b->mg ? p0.pot_extrapolate : 1;
                const int mode = ex >= 3 && b->hist >= 4 ? 3 : ex >= 2 && b->hist >= 3 ? 2 : b->hist >= 2 ? 1 : 0;
                fcd::launch_batch_psi_history<T>(binst<T>(b), t, mode, b->stream);
            }
            st = b->mg ? batch_solve_mg<T>(b, bmg_forward<T>(b), p0.pot_max_iters)
                       : batch_solve<T>(b, forward_problem<T>(b), p0.pot_max_iters);
            if (st) return st;
            ++b->hist;
        }
        ++b->qs;
        fcd::launch_batch_collide<T>(binst<T>(b), t, b->cur, b->stream);
        st = hip_check(hipGetLastError(), "batch collide launch");
        if (st) return st;
        b->cur = 1 - b->cur;
        ++b->steps;
        if (b->steps % div_every_of(p0) == 0) {
            st = batch_read_divergence(b);
            if (st) return st;
        }
    }
    return FCD_OK;
}

// Autotuner: every (fusion, tile shape, block size) candidate advances the batch by one
// untimed step (which captures its graphs) and `steps` real steps timed with HIP events
// on the batch stream; the fastest is kept.  Then, where four sweeps per launch are
// allowed, the tail fusion is chosen the same way among off and four sweeps per launch
// after 8, 16 or 32 tests (one untimed step each first).  The candidates differ only in
// launch geometry and in how sweeps are grouped into launches and graph launches, so
// the states they produce are bitwise the same as an untuned run's.
template <typename T>
fcd_status batch_autotune_impl(fcd_batch* b, int steps, int* choice) {
    const int check = check_interval(b);
    const int blocks[3] = {2 * check, 8 * check, 32 * check};
    double best = 1e300;
    int best_shape = b->shape, best_block = b->block_sweeps, best_fused = b->fused;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    fcd_status st = hip_check(hipEventCreate(&e0), "event");
    if (!st) st = hip_check(hipEventCreate(&e1), "event");
    auto timed = [&](float* ms) {
        if (!st) st = hip_check(hipEventRecord(e0, b->stream), "event");
        if (!st) st = batch_step_impl<T>(b, steps);
        if (!st) st = hip_check(hipEventRecord(e1, b->stream), "event");
        if (!st) st = hip_check(hipEventSynchronize(e1), "event");
        if (!st) st = hip_check(hipEventElapsedTime(ms, e0, e1), "event");
    };
    for (int f = 0; f <= fcd::FUSED_MAX && !st; ++f) {
      if (!fused_allowed(b, f)) continue;
      for (int s = 0; s < fcd::BATCH_SHAPES && !st; ++s) {
        for (int g = 0; g < 3 && !st; ++g) {
            b->fused = f;
            b->shape = s;
            b->block_sweeps = blocks[g];
            st = batch_step_impl<T>(b, 1);  // captures the candidate's graphs outside the timing
            float ms = 0.f;
            timed(&ms);
            if (!st && ms < best) {
                best = ms;
                best_shape = s;
                best_block = blocks[g];
                best_fused = f;
            }
        }
      }
    }
    b->shape = best_shape;
    b->block_sweeps = best_block;
    b->fused = best_fused;
    if (fused_allowed(b, 4)) {
        const int tails[4][2] = {{0, 0}, {4, 8 * check}, {4, 16 * check}, {4, 32 * check}};
        double tbest = 1e300;
        int bt = b->tail_fused, ba = b->tail_after;
        for (int c = 0; c < 4 && !st; ++c) {
            b->tail_fused = tails[c][0];
            b->tail_after = tails[c][1];
            st = batch_step_impl<T>(b, 1);
            float ms = 0.f;
            timed(&ms);
            if (!st && ms < tbest) {
                tbest = ms;
                bt = tails[c][0];
                ba = tails[c][1];
            }
        }
        b->tail_fused = bt;
        b->tail_after = ba;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    choice[0] = BT_ROWS[b->shape];
    choice[1] = b->block_sweeps;
    choice[2] = b->fused;
    choice[3] = b->tail_fused;
    choice[4] = b->tail_after;
    return st;
}

// SOR factor tuner: for each candidate scale s, every channel relaxes with
// 2 / (1 + s sin(pi / (ny + 1))) for `steps` real steps while the decision kernel counts
// the sweeps each channel receives; each channel keeps the factor of its smallest
// count (the first candidate on ties).  The counts depend on the channels' states only,
// so the choice is reproducible.
template <typename T>
fcd_status batch_tune_omega_impl(fcd_batch* b, int steps, int ncand, const double* scale, double* omega_out) {
    std::vector<long long> best(b->n, -1);
    std::vector<double> pick(b->n, 0.0);
    std::vector<int> cnt(b->n);
    int* sweeps = bptr<int>(b->scratch, b->L.off_sweeps);
    fcd_status st = FCD_OK;
    for (int c = 0; c < ncand && !st; ++c) {
        for (int k = 0; k < b->n; ++k)
            b->prm[k].pot_omega = 2.0 / (1.0 + scale[c] * std::sin(3.14159265358979323846 / (b->lat[k].ny + 1)));
        st = batch_upload_inst<T>(b);
        if (!st) st = hip_check(hipMemsetAsync(sweeps, 0, (size_t)b->n * sizeof(int), b->stream), "sweep counters");
        if (!st) st = batch_step_impl<T>(b, steps);
        if (!st)
            st = hip_check(hipMemcpyAsync(cnt.data(), sweeps, (size_t)b->n * sizeof(int), hipMemcpyDeviceToHost,
                                          b->stream), "sweep counters");
        if (!st) st = hip_check(hipStreamSynchronize(b->stream), "sweep counters");
        for (int k = 0; k < b->n && !st; ++k)
            if (best[k] < 0 || cnt[k] < best[k]) {
                best[k] = cnt[k];
                pick[k] = b->prm[k].pot_omega;
            }
    }
    if (st) return st;
    for (int k = 0; k < b->n; ++k) {
        b->prm[k].pot_omega = pick[k];
        omega_out[k] = pick[k];
    }
    return batch_upload_inst<T>(b);
}

template <typename T>
fcd_status batch_init_impl(fcd_batch* b, const double* geom) {
    for (int k = 0; k < b->n; ++k) {
        const fcd_params& p = b->prm[k];
        const fcd_lattice& l = b->lat[k];
        const double u_scale = p.drive_G / (2.0 * p.rho[2] * p.tau[2] / 3.0);
        fcd::launch_init_droplet<T>(bptr<T>(b->state, b->L.off_d0[k]), l.nx, l.ny, b->L.pitch[k], geom[4 * k],
                                    geom[4 * k + 1], geom[4 * k + 2], geom[4 * k + 3], p.xi, u_scale, b->stream);
    }
    fcd::launch_batch_fill_psi<T>(binst<T>(b), btiles(b), b->stream);
    hipLaunchKernelGGL(fcd::k_fill<unsigned long long>, dim3((b->n + 255) / 256), dim3(256), 0, b->stream,
                       reinterpret_cast<unsigned long long*>(b->scratch + b->L.off_div), (long long)b->n, 0ULL);
    b->cur = 0;
    b->hist = 0;
    b->qs = 0;
    b->last_iters = 0;
    b->init_fresh = 1;
    return hip_check(hipGetLastError(), "batch init launch");
}

template <typename T>
void batch_refresh_phase(fcd_batch* b, int k) {
    const fcd::StepConst<T> P = batch_const<T>(b, k);
    const size_t off = b->cur == 0 ? b->L.off_d0[k] : b->L.off_d1[k];
    fcd::launch_phase<T>(bptr<T>(b->state, off), bptr<T>(b->aux, b->L.off_phi[k]), P, b->stream);
}

template <typename T>
fcd_status batch_diag_impl(fcd_batch* b, double* out) {
    double* results = bptr<double>(b->scratch, b->L.off_result);
    for (int k = 0; k < b->n; ++k) {
        batch_refresh_phase<T>(b, k);
        const fcd::StepConst<T> P = batch_const<T>(b, k);
        fcd::launch_diagnostics<T>(bptr<T>(b->aux, b->L.off_phi[k]), P, bptr<double>(b->scratch, b->L.off_rows),
                                   bptr<double>(b->scratch, b->L.off_cent), results + 4 * k, b->stream);
    }
    fcd_status st = hip_check(hipGetLastError(), "batch diagnostics launch");
    if (st) return st;
    st = hip_check(hipMemcpyAsync(b->host + 2, results, (size_t)b->n * 4 * sizeof(double), hipMemcpyDeviceToHost,
                                  b->stream), "batch diagnostics copy");
    if (st) return st;
    st = hip_check(hipStreamSynchronize(b->stream), "batch diagnostics sync");
    if (st) return st;
    std::memcpy(out, b->host + 2, (size_t)b->n * 4 * sizeof(double));
    return batch_read_divergence(b);
}

template <typename T>
fcd_status batch_state_impl(fcd_batch* b, int k, double* out) {
    const fcd_lattice& l = b->lat[k];
    const size_t off = b->cur == 0 ? b->L.off_d0[k] : b->L.off_d1[k];
    fcd::launch_to_dense<T>(bptr<T>(b->state, off), out, 27, l.nx, l.ny, b->L.pitch[k], b->stream);
    return hip_check(hipGetLastError(), "batch copy launch");
}

template <typename T>
fcd_status batch_moments_impl(fcd_batch* b, int k, unsigned mask, double* out) {
    batch_refresh_phase<T>(b, k);
    const size_t off = b->cur == 0 ? b->L.off_d0[k] : b->L.off_d1[k];
    fcd::launch_moments<T>(bptr<T>(b->state, off), bptr<T>(b->aux, b->L.off_phi[k]),
                           bptr<T>(b->aux, b->L.off_psi[k]), batch_const<T>(b, k), mask, out, b->stream);
    return hip_check(hipGetLastError(), "batch moments launch");
}

// ---------------------------------------------------------------------------------
// Checkpointed adjoint.
// ---------------------------------------------------------------------------------
struct AdjLayout {
    size_t plane, state;
    size_t crec;  // checkpoint record: state, psi' and the three psi' history planes (warm start)
    size_t srec;  // segment record: state and the step's psi'
    int nseg, nblocks;
    size_t off_ckpt, off_final, off_seg, off_lam, off_sens, off_rhs, off_lpsi, off_lprev, off_lprev2, off_part, off_acc,
        off_rmax, bytes;
};

AdjLayout adj_layout(const fcd_lattice& l, int nsteps, int every) {
    AdjLayout L{};
    L.plane = (size_t)l.ny * l.pitch * elem_size(l.precision);
    L.state = 27 * L.plane;
    L.crec = align256(L.state + 4 * L.plane);
    L.srec = align256(L.state + L.plane);
    L.nseg = (nsteps + every - 1) / every;
    L.nblocks = fcd::adj_blocks(l.nx, l.ny);
    size_t off = 0;
    L.off_ckpt = off;
    off += (size_t)L.nseg * L.crec;
    L.off_final = off;
    off += L.crec;
    L.off_seg = off;
    off += (size_t)every * L.srec;
    L.off_lam = off;
    off += 2 * align256(L.state);
    L.off_sens = off;
    off += align256(10 * L.plane);
    L.off_rhs = off;
    off += align256(L.plane);
    L.off_lpsi = off;
    off += align256(L.plane);
    L.off_lprev = off;
    off += align256(L.plane);
    L.off_lprev2 = off;
    off += align256(L.plane);
    L.off_part = off;
    off += align256(3 * (size_t)L.nblocks * fcd::ADJ_NPART * sizeof(double));
    L.off_acc = off;
    off += 256;
    L.off_rmax = off;
    off += 256;
    L.bytes = off;
    return L;
}

fcd_status dcopy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    return hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "device copy");
}

// Checkpoint records hold everything a step reads: the state, psi' (the solver's warm
// start) and the psi' history planes (in the order psi'(t-1), psi'(t-2), psi'(t-3)); the
// history count and the previous solve's iteration count are kept on the host beside them.

template <typename T>
fcd_status save_record(fcd_handle* h, char* rec, const AdjLayout& L) {
    fcd_status st = dcopy(rec, h->buf.dist[h->cur], L.state, h->stream);
    if (!st) st = dcopy(rec + L.state, h->buf.psi, L.plane, h->stream);
    if (!st) st = dcopy(rec + L.state + L.plane, psi_prev<T>(h), L.plane, h->stream);
    if (!st) st = dcopy(rec + L.state + 2 * L.plane, psi_prev<T>(h, 2), L.plane, h->stream);
    if (!st) st = dcopy(rec + L.state + 3 * L.plane, psi_prev<T>(h, 3), L.plane, h->stream);
    return st;
}

template <typename T>
fcd_status load_record(fcd_handle* h, const char* rec, const AdjLayout& L) {
    fcd_status st = dcopy(h->buf.dist[h->cur], rec, L.state, h->stream);
    if (!st) st = dcopy(h->buf.psi, rec + L.state, L.plane, h->stream);
    if (!st) st = dcopy(psi_prev<T>(h), rec + L.state + L.plane, L.plane, h->stream);
    if (!st) st = dcopy(psi_prev<T>(h, 2), rec + L.state + 2 * L.plane, L.plane, h->stream);
    if (!st) st = dcopy(psi_prev<T>(h, 3), rec + L.state + 3 * L.plane, L.plane, h->stream);
    return st;
}

template <typename T>
fcd_status adj_forward_impl(fcd_handle* h, int nsteps, int every, char* work, double D_out[2]) {
    const AdjLayout L = adj_layout(h->lat, nsteps, every);
    h->adj_work = work;
    h->adj_nsteps = nsteps;
    h->adj_every = every;
    h->adj_from_init = h->init_fresh;
    h->adj_ckpt_iters.assign(2 * (size_t)L.nseg, 0);
    fcd_status st = FCD_OK;
    for (int t = 0; t < nsteps && !st; ++t) {
        if (t % every == 0) {
            st = save_record<T>(h, work + L.off_ckpt + (size_t)(t / every) * L.crec, L);
            h->adj_ckpt_iters[2 * (t / every)] = h->last_iters;
            h->adj_ckpt_iters[2 * (t / every) + 1] = h->hist;
        }
        if (!st) st = step_impl<T>(h, 1);
    }
    if (st) return st;
    st = save_record<T>(h, work + L.off_final, L);
    if (st) return st;
    h->adj_final_iters = h->last_iters;
    h->adj_final_hist = h->hist;
    double d[4];
    st = diag_impl<T>(h, d);
    if (st) return st;
    D_out[0] = d[0];
    D_out[1] = d[1];
    return FCD_OK;
}

template <typename T>
fcd_status adj_backward_impl(fcd_handle* h, const double dJ[2], double grad[6]) {
    if (!h->adj_work || h->adj_every < 1) return fail(FCD_ERR_ARG, "fcd_adjoint_forward has not run");
    const int nsteps = h->adj_nsteps, every = h->adj_every;
    const AdjLayout L = adj_layout(h->lat, nsteps, every);
    char* w = h->adj_work;
    const fcd::StepConst<T> P = make_const<T>(h);
    const long long pl = P.plane;
    T* lam[2] = {reinterpret_cast<T*>(w + L.off_lam), reinterpret_cast<T*>(w + L.off_lam + align256(L.state))};
    T* sens = reinterpret_cast<T*>(w + L.off_sens);
    T* rhs = reinterpret_cast<T*>(w + L.off_rhs);
    T* lpsi = reinterpret_cast<T*>(w + L.off_lpsi);
    double* partA = reinterpret_cast<double*>(w + L.off_part);
    double* partB = partA + (size_t)L.nblocks * fcd::ADJ_NPART;
    double* partC = partB + (size_t)L.nblocks * fcd::ADJ_NPART;
    double* acc = reinterpret_cast<double*>(w + L.off_acc);
    unsigned long long* rmax = reinterpret_cast<unsigned long long*>(w + L.off_rmax);
    T* phi = static_cast<T*>(h->buf.phi);
    char* scr = static_cast<char*>(h->buf.scratch);
    T* lprev = reinterpret_cast<T*>(w + L.off_lprev);
    T* lprev2 = reinterpret_cast<T*>(w + L.off_lprev2);
    fcd::launch_fill<double>(acc, 16, 0.0, h->stream);
    fcd::launch_fill<T>(lpsi, pl, T(0), h->stream);
    int lhist = 0;  // adjoint potential solves so far (warm-start extrapolation validity)
    // seed: adjoint of the final state from J = dJ[0] D_o + dJ[1] D_i
    fcd_status st = load_record<T>(h, w + L.off_final, L);
    if (st) return st;
    double d[4];
    st = diag_impl<T>(h, d);  // phase planes and the deformation moments of the final state
    if (st) return st;
    fcd::launch_adj_seed<T>(phi, reinterpret_cast<const double*>(scr + OFF_CENT) + 8, dJ[0], dJ[1], lam[0], P,
                            h->stream);
    int A = 0, adj_iters = 0;
    const bool field = h->prm.H0 != 0.0;
    for (int seg = L.nseg - 1; seg >= 0 && !st; --seg) {
        const int t0 = seg * every, t1 = std::min(nsteps, t0 + every);
        st = load_record<T>(h, w + L.off_ckpt + (size_t)seg * L.crec, L);
        if (st) break;
        h->last_iters = h->adj_ckpt_iters[2 * seg];
        h->hist = h->adj_ckpt_iters[2 * seg + 1];
        for (int t = t0; t < t1 && !st; ++t) {
            char* rec = w + L.off_seg + (size_t)(t - t0) * L.srec;
            st = dcopy(rec, h->buf.dist[h->cur], L.state, h->stream);
            if (!st) st = step_impl<T>(h, 1);
            if (!st) st = dcopy(rec + L.state, h->buf.psi, L.plane, h->stream);
        }
        for (int t = t1 - 1; t >= t0 && !st; --t) {
            const char* rec = w + L.off_seg + (size_t)(t - t0) * L.srec;
            const T* s_t = reinterpret_cast<const T*>(rec);
            const T* psi_t = reinterpret_cast<const T*>(rec + L.state);
            fcd::launch_phase<T>(s_t, phi, P, h->stream);
            fcd::launch_adj_node<T>(s_t, phi, psi_t, lam[A], lam[1 - A], sens, partA, P, h->stream);
            fcd::launch_adj_reduce(partA, L.nblocks, 13, acc, 0, h->stream);
            st = hip_check(hipGetLastError(), "adjoint node launch");
            if (st) break;
            if (field) {
                fcd::launch_adj_gather_psi<T>(sens, rhs, rmax, P, h->stream);
                if (h->prm.pot_solver == FCD_SOLVER_MG) restrict_mu_all<T>(h);
                st = hip_check(hipMemcpyAsync(h->host, rmax, sizeof(double), hipMemcpyDeviceToHost, h->stream),
                               "adjoint rhs copy");
                if (!st) st = hip_check(hipStreamSynchronize(h->stream), "adjoint rhs sync");
                if (st) break;
                double rm;
                std::memcpy(&rm, h->host, sizeof(double));
                if (rm > 0.0) {
                    // warm start: linear extrapolation of the last two adjoint solutions
                    if (h->prm.pot_extrapolate) {
                        // the adjoint potentials of successive (reversed) steps, extrapolated
                        // as in the forward, at most quadratically
                        const int mode = lhist >= 3 && h->prm.pot_extrapolate >= 2 ? 2 : lhist >= 2 ? 1 : 0;
                        fcd::launch_psi_history<T>(lpsi, lprev, lprev2, static_cast<T*>(nullptr), h->lat.nx,
                                                   h->lat.ny, h->lat.pitch, mode, h->stream);
                    }
                    ++lhist;
                    fcd::PotLevel<T> La = pot_level<T>(h, 0);
                    La.u = lpsi;
                    La.f = rhs;
                    La.H0x = La.H0y = T(0);
                    int it = 0;
                    if (solves_on_device(h)) {
                        auto publish = [&](const fcd::StepGate& sg) {
                            fcd::launch_solve_publish(sg, h->stream);
                            return hip_check(hipGetLastError(), "publication launch");
                        };
                        double r = 0.0;
                        bool done = false;
                        st = solve_on_device<T>(h, La, h->prm.pot_tol * rm, h->prm.pot_max_iters,
                                                adj_iters <= 1 ? adj_iters : adj_iters - 1, publish, &it, &r, &done);
                        h->sweeps += it;
                        h->last_resid = r;
                    } else {
                        st = iterate_level0<T>(h, La, h->prm.pot_tol * rm, h->prm.pot_max_iters, adj_iters, &it,
                                               nullptr);
                    }
                    adj_iters = it;
                    if (st) break;
                } else {
                    fcd::launch_fill<T>(lpsi, pl, T(0), h->stream);
                    lhist = 0;
                }
                fcd::launch_adj_finish<T>(sens, phi, psi_t, lpsi, lam[1 - A], partB, P, h->stream);
                fcd::launch_adj_reduce(partB, L.nblocks, 2, acc, 13, h->stream);
            } else {
                fcd::launch_fill<T>(lpsi, pl, T(0), h->stream);
                fcd::launch_adj_finish<T>(sens, phi, psi_t, lpsi, lam[1 - A], partB, P, h->stream);
            }
            st = hip_check(hipGetLastError(), "adjoint finish launch");
            A = 1 - A;
        }
    }
    if (st) return st;
    if (h->adj_from_init) {
        const double nu3 = h->prm.tau[2] / 3.0;
        const double dUdG = 1.0 / (2.0 * h->prm.rho[2] * nu3);
        fcd::launch_adj_init_drive<T>(reinterpret_cast<const T*>(w + L.off_ckpt), lam[A], dUdG,
                                      h->prm.drive_G * dUdG, partC, P, h->stream);
        fcd::launch_adj_reduce(partC, L.nblocks, 1, acc, 15, h->stream);
    }
    st = hip_check(hipMemcpyAsync(h->host, acc, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                   "adjoint result copy");
    if (!st) st = hip_check(hipStreamSynchronize(h->stream), "adjoint result sync");
    if (st) return st;
    double a[16];
    std::memcpy(a, h->host, sizeof(a));
    const fcd_params& p = h->prm;
    const double ca = std::cos(p.alpha), sa = std::sin(p.alpha);
    const double hx = a[0] + a[13], hy = a[1] + a[14];
    grad[0] = hx * ca + hy * sa;
    grad[1] = p.H0 * (-hx * sa + hy * ca);
    grad[2] = (a[2] + a[15]) * drive_per_u_ref(p, h->lat.ny);
    const double g[3] = {p.sigma12 + p.sigma13 - p.sigma23, p.sigma12 + p.sigma23 - p.sigma13,
                         p.sigma13 + p.sigma23 - p.sigma12};
    const double gT = 3.0 / (1.0 / g[0] + 1.0 / g[1] + 1.0 / g[2]);
    double gb[3];
    for (int k = 0; k < 3; ++k)
        gb[k] = a[6 + k] - a[9 + k] / (g[k] * g[k]) + a[12] * (4.0 / p.xi) * gT * gT / (3.0 * g[k] * g[k]);
    grad[3] = a[3] + gb[0] + gb[1] - gb[2];
    grad[4] = a[4] + gb[0] - gb[1] + gb[2];
    grad[5] = a[5] - gb[0] + gb[1] + gb[2];
    // leave the handle on the forward's final state
    h->last_iters = h->adj_final_iters;
    h->hist = h->adj_final_hist;
    return load_record<T>(h, w + L.off_final, L);
}

// ---------------------------------------------------------------------------------
// Batched checkpointed adjoint.  Per channel the work buffer holds the checkpoint
// records (state, psi', psi' history), the final record, the segment records (state,
// psi'), two adjoint states, the ten sensitivity planes and the adjoint potential's
// right-hand side, solution and history; shared: the adjoint-potential descriptors,
// the per-channel adjoint descriptors, per-tile partials, per-channel accumulators
// and scales.
// ---------------------------------------------------------------------------------
struct BatchAdjLayout {
    int nseg = 0;
    std::vector<size_t> plane, crec, srec, off_ckpt, off_final, off_seg, off_lam0, off_lam1, off_sens, off_rhs,
        off_lpsi, off_lprev;
    size_t off_ainst = 0, off_adj = 0, off_part = 0, off_partC = 0, off_acc = 0, off_scale = 0, bytes = 0;
};

BatchAdjLayout batch_adj_layout(const fcd_batch* b, int nsteps, int every) {
    BatchAdjLayout A;
    A.nseg = (nsteps + every - 1) / every;
    const size_t esz = elem_size(b->precision);
    size_t off = 0;
    int max_blocks = 0;
    for (int k = 0; k < b->n; ++k) {
        const size_t pl = align256((size_t)b->lat[k].ny * b->L.pitch[k] * esz);
        A.plane.push_back(pl);
        A.crec.push_back(31 * pl);
        A.srec.push_back(28 * pl);
        A.off_ckpt.push_back(off);
        off += (size_t)A.nseg * 31 * pl;
        A.off_final.push_back(off);
        off += 31 * pl;
        A.off_seg.push_back(off);
        off += (size_t)every * 28 * pl;
        A.off_lam0.push_back(off);
        off += 27 * pl;
        A.off_lam1.push_back(off);
        off += 27 * pl;
        A.off_sens.push_back(off);
        off += 10 * pl;
        A.off_rhs.push_back(off);
        off += pl;
        A.off_lpsi.push_back(off);
        off += pl;
        A.off_lprev.push_back(off);
        off += pl;
        max_blocks = std::max(max_blocks, fcd::adj_blocks(b->lat[k].nx, b->lat[k].ny));
    }
    const size_t inst_sz = b->precision == FCD_FP64 ? sizeof(fcd::BatchInst<double>) : sizeof(fcd::BatchInst<float>);
    const size_t adj_sz = b->precision == FCD_FP64 ? sizeof(fcd::BatchAdj<double>) : sizeof(fcd::BatchAdj<float>);
    A.off_ainst = off;
    off = align256(off + (size_t)b->n * inst_sz);
    A.off_adj = off;
    off = align256(off + (size_t)b->n * adj_sz);
    A.off_part = off;
    off = align256(off + (size_t)b->L.ntiles[2] * fcd::ADJ_NPART * sizeof(double));
    A.off_partC = off;
    off = align256(off + (size_t)max_blocks * fcd::ADJ_NPART * sizeof(double));
    A.off_acc = off;
    off = align256(off + (size_t)b->n * 16 * sizeof(double));
    A.off_scale = off;
    off = align256(off + (size_t)b->n * sizeof(unsigned long long));
    A.bytes = off;
    return A;
}

char* bstate(fcd_batch* b, int k) { return b->state + (b->cur == 0 ? b->L.off_d0[k] : b->L.off_d1[k]); }

// Whole-batch records: the current state, psi' and psi' history of every channel.
fcd_status batch_save_records(fcd_batch* b, const BatchAdjLayout& A, const std::vector<size_t>& off, int idx) {
    fcd_status st = FCD_OK;
    for (int k = 0; k < b->n && !st; ++k) {
        char* rec = b->adj_work + off[k] + (size_t)idx * A.crec[k];
        const size_t pl = A.plane[k];
        st = dcopy(rec, bstate(b, k), 27 * pl, b->stream);
        if (!st) st = dcopy(rec + 27 * pl, b->aux + b->L.off_psi[k], pl, b->stream);
        if (!st) st = dcopy(rec + 28 * pl, b->aux + b->L.off_prev[k], pl, b->stream);
        if (!st) st = dcopy(rec + 29 * pl, b->aux + b->L.off_prev2[k], pl, b->stream);
        if (!st) st = dcopy(rec + 30 * pl, b->aux + b->L.off_prev3[k], pl, b->stream);
    }
    return st;
}

fcd_status batch_load_records(fcd_batch* b, const BatchAdjLayout& A, const std::vector<size_t>& off, int idx) {
    fcd_status st = FCD_OK;
    for (int k = 0; k < b->n && !st; ++k) {
        const char* rec = b->adj_work + off[k] + (size_t)idx * A.crec[k];
        const size_t pl = A.plane[k];
        st = dcopy(bstate(b, k), rec, 27 * pl, b->stream);
        if (!st) st = dcopy(b->aux + b->L.off_psi[k], rec + 27 * pl, pl, b->stream);
        if (!st) st = dcopy(b->aux + b->L.off_prev[k], rec + 28 * pl, pl, b->stream);
        if (!st) st = dcopy(b->aux + b->L.off_prev2[k], rec + 29 * pl, pl, b->stream);
        if (!st) st = dcopy(b->aux + b->L.off_prev3[k], rec + 30 * pl, pl, b->stream);
    }
    return st;
}

template <typename T>
fcd_status batch_adj_forward_impl(fcd_batch* b, int nsteps, int every, char* work, double* D_out) {
    const BatchAdjLayout A = batch_adj_layout(b, nsteps, every);
    // descriptors of the adjoint potential problems and of the per-channel work planes
    std::vector<fcd::BatchInst<T>> ainst(b->n);
    std::vector<fcd::BatchAdj<T>> adj(b->n);
    for (int k = 0; k < b->n; ++k) {
        fcd::BatchInst<T>& I = ainst[k];
        I = make_batch_inst<T>(b, k);
        I.L0.u = reinterpret_cast<T*>(work + A.off_lpsi[k]);
        I.L0.f = reinterpret_cast<T*>(work + A.off_rhs[k]);
        I.L0.H0x = I.L0.H0y = T(0);
        I.prev = reinterpret_cast<T*>(work + A.off_lprev[k]);
        I.prev2 = nullptr;  // the adjoint solves start linearly
        I.prev3 = nullptr;
        fcd::BatchAdj<T>& D = adj[k];
        D.seg = reinterpret_cast<T*>(work + A.off_seg[k]);
        D.srec = (long long)(A.srec[k] / sizeof(T));
        D.lam[0] = reinterpret_cast<T*>(work + A.off_lam0[k]);
        D.lam[1] = reinterpret_cast<T*>(work + A.off_lam1[k]);
        D.sens = reinterpret_cast<T*>(work + A.off_sens[k]);
        D.rhs = reinterpret_cast<T*>(work + A.off_rhs[k]);
        D.tile_first = b->L.tile0[2][k];
        D.tile_count = b->L.tiles_x[2][k] * ((b->lat[k].ny + BT_ROWS[2] - 1) / BT_ROWS[2]);
    }
    fcd_status st = hip_check(hipMemcpy(work + A.off_ainst, ainst.data(), ainst.size() * sizeof(ainst[0]),
                                        hipMemcpyHostToDevice), "adjoint descriptor upload");
    if (!st && b->mg) {
        // the adjoint potential problems for the batched multigrid: each channel's hierarchy
        // with the adjoint potential plane and its right-hand side on the finest level
        std::vector<fcd::MgChan<T, CT>> mch(b->n);
        for (int k = 0; k < b->n; ++k) {
            mch[k] = make_mgchan<T>(b, k);
            mch[k].L0 = ainst[k].L0;
        }
        st = hip_check(hipMemcpy(b->scratch + b->L.off_mgchan_adj, mch.data(), mch.size() * sizeof(mch[0]),
                                 hipMemcpyHostToDevice), "adjoint multigrid descriptor upload");
    }
    if (!st) st = hip_check(hipMemcpy(work + A.off_adj, adj.data(), adj.size() * sizeof(adj[0]),
                                      hipMemcpyHostToDevice), "adjoint descriptor upload");
    if (st) return st;
    b->adj_work = work;
    b->adj_nsteps = nsteps;
    b->adj_every = every;
    b->adj_from_init = b->init_fresh;
    b->adj_ckpt.assign(2 * (size_t)A.nseg, 0);
    for (int t = 0; t < nsteps && !st; ++t) {
        if (t % every == 0) {
            st = batch_save_records(b, A, A.off_ckpt, t / every);
            b->adj_ckpt[2 * (t / every)] = b->last_iters;
            b->adj_ckpt[2 * (t / every) + 1] = b->hist;
        }
        if (!st) st = batch_step_impl<T>(b, 1);
    }
    if (!st) st = batch_save_records(b, A, A.off_final, 0);
    if (st) return st;
    b->init_fresh = 0;
    b->adj_final_iters = b->last_iters;
    b->adj_final_hist = b->hist;
    std::vector<double> d(4 * (size_t)b->n);
    st = batch_diag_impl<T>(b, d.data());
    if (st) return st;
    for (int k = 0; k < b->n; ++k) {
        D_out[2 * k] = d[4 * k];
        D_out[2 * k + 1] = d[4 * k + 1];
    }
    return FCD_OK;
}

template <typename T>
fcd_status batch_adj_backward_impl(fcd_batch* b, const double* dJ, double* grad) {
    if (!b->adj_work || b->adj_every < 1) return fail(FCD_ERR_ARG, "fcd_batch_adjoint_forward has not run");
    const int nsteps = b->adj_nsteps, every = b->adj_every;
    const BatchAdjLayout A = batch_adj_layout(b, nsteps, every);
    char* w = b->adj_work;
    const fcd::BatchInst<T>* inst = binst<T>(b);
    const fcd::BatchInst<T>* ainst = reinterpret_cast<const fcd::BatchInst<T>*>(w + A.off_ainst);
    const fcd::BatchAdj<T>* adj = reinterpret_cast<const fcd::BatchAdj<T>*>(w + A.off_adj);
    double* part = reinterpret_cast<double*>(w + A.off_part);
    double* partC = reinterpret_cast<double*>(w + A.off_partC);
    double* acc = reinterpret_cast<double*>(w + A.off_acc);
    unsigned long long* scale = reinterpret_cast<unsigned long long*>(w + A.off_scale);
    fcd::BatchTiles t2;
    t2.shape = 2;
    t2.ntiles = b->L.ntiles[2];
    t2.nctiles = b->L.nctiles[2];
    t2.tiles = reinterpret_cast<const int*>(b->scratch + b->L.off_tiles[2]);
    t2.ctiles = reinterpret_cast<const int*>(b->scratch + b->L.off_ctiles[2]);
    fcd::launch_fill<double>(acc, 16LL * b->n, 0.0, b->stream);
    fcd::launch_batch_fill_psi<T>(ainst, btiles(b), b->stream);  // adjoint potentials start at zero
    fcd_status st = batch_load_records(b, A, A.off_final, 0);
    if (st) return st;
    // seed: adjoint of every channel's final state from J_k = dJ[2k] D_o + dJ[2k+1] D_i
    double* cent = bptr<double>(b->scratch, b->L.off_cent);
    double* results = bptr<double>(b->scratch, b->L.off_result);
    for (int k = 0; k < b->n; ++k) {
        batch_refresh_phase<T>(b, k);
        const fcd::StepConst<T> P = batch_const<T>(b, k);
        T* phi = bptr<T>(b->aux, b->L.off_phi[k]);
        fcd::launch_diagnostics<T>(phi, P, bptr<double>(b->scratch, b->L.off_rows), cent, results + 4 * k, b->stream);
        fcd::launch_adj_seed<T>(phi, cent + 8, dJ[2 * k], dJ[2 * k + 1], reinterpret_cast<T*>(w + A.off_lam0[k]), P,
                                b->stream);
    }
    st = hip_check(hipGetLastError(), "batch adjoint seed");
    if (st) return st;
    int Aidx = 0, lhist = 0;
    b->adj_solve_iters = 0;
    const fcd_params& p0 = b->prm[0];
    const BatchProblem<T> adjP{ainst, scale, p0.pot_tol, &b->adj_solve_iters, true};
    b->adj_mg_last_cycles = 0;
    const BmgProblem<T> adjM{reinterpret_cast<const fcd::MgChan<T, CT>*>(b->scratch + b->L.off_mgchan_adj), true, scale,
                             p0.pot_tol, &b->adj_mg_last_cycles};
    for (int seg = A.nseg - 1; seg >= 0 && !st; --seg) {
        const int t0 = seg * every, t1 = std::min(nsteps, t0 + every);
        st = batch_load_records(b, A, A.off_ckpt, seg);
        if (st) break;
        b->last_iters = b->adj_ckpt[2 * seg];
        b->hist = b->adj_ckpt[2 * seg + 1];
        for (int t = t0; t < t1 && !st; ++t) {
            fcd::launch_batch_adj_save<T>(inst, adj, t2, b->cur, t - t0, 0, b->stream);
            st = batch_step_impl<T>(b, 1);
            fcd::launch_batch_adj_save<T>(inst, adj, t2, b->cur, t - t0, 1, b->stream);
        }
        for (int t = t1 - 1; t >= t0 && !st; --t) {
            const int r = t - t0;
            fcd::launch_batch_adj_phase<T>(inst, adj, t2, r, b->stream);
            fcd::launch_batch_adj_node<T>(inst, adj, t2, r, Aidx, part, b->stream);
            fcd::launch_batch_adj_reduce<T>(adj, b->n, part, 13, acc, 0, b->stream);
            fcd::launch_batch_adj_gather<T>(inst, adj, t2, scale, b->n, b->stream);
            // warm start: linear extrapolation of the last two adjoint solutions
            if (p0.pot_extrapolate) fcd::launch_batch_psi_history<T>(ainst, btiles(b), lhist >= 2 ? 1 : 0, b->stream);
            ++lhist;
            st = hip_check(hipGetLastError(), "batch adjoint launch");
            if (!st) st = b->mg ? batch_solve_mg<T>(b, adjM, p0.pot_max_iters) : batch_solve<T>(b, adjP, p0.pot_max_iters);
            if (st) break;
            fcd::launch_batch_adj_finish<T>(inst, ainst, adj, t2, r, Aidx, part, b->stream);
            fcd::launch_batch_adj_reduce<T>(adj, b->n, part, 2, acc, 13, b->stream);
            st = hip_check(hipGetLastError(), "batch adjoint launch");
            Aidx = 1 - Aidx;
        }
    }
    if (st) return st;
    if (b->adj_from_init) {
        for (int k = 0; k < b->n; ++k) {
            const fcd_params& p = b->prm[k];
            const fcd::StepConst<T> P = batch_const<T>(b, k);
            const double dUdG = 1.0 / (2.0 * p.rho[2] * p.tau[2] / 3.0);
            const T* s0 = reinterpret_cast<const T*>(w + A.off_ckpt[k]);
            const T* lam0 = reinterpret_cast<const T*>(w + (Aidx == 0 ? A.off_lam0[k] : A.off_lam1[k]));
            fcd::launch_adj_init_drive<T>(s0, lam0, dUdG, p.drive_G * dUdG, partC, P, b->stream);
            fcd::launch_adj_reduce(partC, fcd::adj_blocks(b->lat[k].nx, b->lat[k].ny), 1, acc + 16 * k, 15, b->stream);
        }
    }
    std::vector<double> a(16 * (size_t)b->n);
    st = hip_check(hipStreamSynchronize(b->stream), "batch adjoint sync");
    if (!st) st = hip_check(hipMemcpy(a.data(), acc, a.size() * sizeof(double), hipMemcpyDeviceToHost), "copy");
    if (st) return st;
    for (int k = 0; k < b->n; ++k) {
        const double* ak = a.data() + 16 * k;
        const fcd_params& p = b->prm[k];
        double* g = grad + 6 * k;
        const double ca = std::cos(p.alpha), sa = std::sin(p.alpha);
        const double hx = ak[0] + ak[13], hy = ak[1] + ak[14];
        g[0] = hx * ca + hy * sa;
        g[1] = p.H0 * (-hx * sa + hy * ca);
        g[2] = (ak[2] + ak[15]) * drive_per_u_ref(p, b->lat[k].ny);
        const double gm[3] = {p.sigma12 + p.sigma13 - p.sigma23, p.sigma12 + p.sigma23 - p.sigma13,
                              p.sigma13 + p.sigma23 - p.sigma12};
        const double gT = 3.0 / (1.0 / gm[0] + 1.0 / gm[1] + 1.0 / gm[2]);
        double gb[3];
        for (int q = 0; q < 3; ++q)
            gb[q] = ak[6 + q] - ak[9 + q] / (gm[q] * gm[q]) + ak[12] * (4.0 / p.xi) * gT * gT / (3.0 * gm[q] * gm[q]);
        g[3] = ak[3] + gb[0] + gb[1] - gb[2];
        g[4] = ak[4] + gb[0] - gb[1] + gb[2];
        g[5] = ak[5] - gb[0] + gb[1] + gb[2];
    }
    b->last_iters = b->adj_final_iters;
    b->hist = b->adj_final_hist;
    return batch_load_records(b, A, A.off_final, 0);
}


#define FCD_BDISPATCH(b, call) ((b)->precision == FCD_FP64 ? call<double> : call<float>)

}  // namespace

extern "C" {

size_t fcd_scratch_bytes(const fcd_lattice* lat) {
    if (check_lattice(lat) != FCD_OK) return 0;
    return make_plan(*lat).bytes;
}

fcd_status fcd_create(const fcd_lattice* lat, const fcd_params* prm, const fcd_buffers* buf, void* hip_stream,
                      fcd_handle** out) {
    if (!out) return fail(FCD_ERR_ARG, "out is null");
    *out = nullptr;
    fcd_status st = check_lattice(lat);
    if (st) return st;
    st = check_params(prm);
    if (st) return st;
    if (!buf || !buf->dist[0] || !buf->dist[1] || !buf->phi || !buf->psi || !buf->scratch)
        return fail(FCD_ERR_ARG, "a device buffer is null");
    if (buf->dist[0] == buf->dist[1]) return fail(FCD_ERR_ARG, "the two state buffers must differ");
    const size_t align = elem_size(lat->precision);
    const void* ptrs[5] = {buf->dist[0], buf->dist[1], buf->phi, buf->psi, buf->scratch};
    for (const void* p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) % align) return fail(FCD_ERR_ARG, "misaligned device buffer");
    if (reinterpret_cast<uintptr_t>(buf->scratch) % 256) return fail(FCD_ERR_ARG, "scratch must be 256-byte aligned");
    fcd_handle* h = new (std::nothrow) fcd_handle();
    if (!h) return fail(FCD_ERR_OOM, "handle allocation failed");
    h->lat = *lat;
    h->prm = *prm;
    h->buf = *buf;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->cur = 0;
    h->steps = h->sweeps = 0;
    h->last_resid = 0.0;
    h->hist = 0;
    h->qs = 0;
    h->last_iters = 0;
    h->init_fresh = 0;
    h->open_x = 0;
    h->u_in = h->u_out = 0.0;
    h->track_on = 0;
    h->track_x_prev = h->track_x_run = 0.0;
    h->steps_at_init = 0;
    h->r_shell = 0.0;
    h->adj_work = nullptr;
    h->adj_nsteps = h->adj_every = h->adj_from_init = 0;
    h->adj_final_iters = h->adj_final_hist = 0;
    h->plan = make_plan(*lat);
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host), 32 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return fail(FCD_ERR_OOM, "pinned host allocation failed");
    }
    // written by the GPU while the host polls it: coherent (fine-grained) host memory
    if (hipHostMalloc(reinterpret_cast<void**>(&h->mirror), sizeof(fcd::SolveMirror), hipHostMallocCoherent) !=
        hipSuccess) {
        (void)hipHostFree(h->host);
        delete h;
        return fail(FCD_ERR_OOM, "pinned host allocation failed");
    }
    std::memset(h->mirror, 0, sizeof(fcd::SolveMirror));
    h->seq_want = 0;
    h->test_idx = 0;
    h->gate = fcd::ResGate{};
    h->pipe_last = 1;
    h->ring = 0;
    // the scratch arrives with the caller's contents: zero both residual slots, the flag,
    // the SOR words and the device-decided solve's words
    h->res_slot = 0;
    hipLaunchKernelGGL(fcd::k_fill<unsigned long long>, dim3(1), dim3(64), 0, h->stream, res_slot_ptr(h, 0),
                       (long long)((OFF_TESTS + 8) / sizeof(unsigned long long)), 0ULL);
    st = hip_check(hipGetLastError(), "residual slot clear");
    if (st) {
        (void)hipHostFree(h->mirror);
        (void)hipHostFree(h->host);
        delete h;
        return st;
    }
    *out = h;
    return FCD_OK;
}

fcd_status fcd_set_params(fcd_handle* h, const fcd_params* prm) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = check_params(prm);
    if (st) return st;
    h->prm = *prm;
    h->graphs.clear();
    return FCD_OK;
}

fcd_status fcd_use_graphs(fcd_handle* h, int32_t enable) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    h->graphs.clear();
    h->graphs.enabled = enable != 0;
    return st;
}

fcd_status fcd_set_open_channel(fcd_handle* h, double u_avg) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (!(u_avg >= 0.0) || !(u_avg < 1.0)) return fail(FCD_ERR_ARG, "need 0 <= u_avg < 1");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    h->open_x = 1;
    h->u_in = u_avg;
    double U = 0.0;
    for (int j = 0; j < h->lat.ny; ++j) {
        const double s = (j + 0.5) / h->lat.ny;
        U += 4.0 * u_avg * s * (1.0 - s);
    }
    h->u_out = U / h->lat.ny;
    h->graphs.clear();
    return st;
}

fcd_status fcd_init_compound_droplet(fcd_handle* h, double xc, double yc, double r_core, double r_shell) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    h->hist = 0;
    h->qs = 0;
    h->last_iters = 0;
    h->init_fresh = 1;
    h->track_on = 0;
    h->steps_at_init = h->steps;
    h->r_shell = r_shell;
    if (!(r_core >= 0.0) || !(r_shell >= r_core)) return fail(FCD_ERR_ARG, "need 0 <= r_core <= r_shell");
    return FCD_DISPATCH(h, init_droplet_impl)(h, xc, yc, r_core, r_shell);
}

fcd_status fcd_init_fields(fcd_handle* h, const double* phi1, const double* phi2, const double* ux,
                           const double* uy, const double* pstar) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    h->init_fresh = 0;
    h->hist = 0;
    h->qs = 0;
    h->last_iters = 0;
    h->track_on = 0;
    h->steps_at_init = h->steps;
    h->r_shell = 0.0;
    if (!phi1 || !phi2 || !ux || !uy) return fail(FCD_ERR_ARG, "a field pointer is null");
    return FCD_DISPATCH(h, init_fields_impl)(h, phi1, phi2, ux, uy, pstar);
}

fcd_status fcd_solve_potential(fcd_handle* h, double tol, int32_t max_iters, int32_t* iters_out,
                               double* resid_out) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (!(tol > 0.0) || max_iters < 0) return fail(FCD_ERR_ARG, "bad tolerance or iteration limit");
    fcd_status st = FCD_DISPATCH(h, refresh_phase)(h);
    if (st) return st;
    int it = 0;
    st = FCD_DISPATCH(h, solve_impl)(h, tol, max_iters, &it, resid_out);
    if (iters_out) *iters_out = it;
    // an explicit solve (typically from a cold start) says nothing about how many cycles
    // the next time step's warm-started solve needs: its first residual test is not deferred
    h->last_iters = 0;
    return st;
}

fcd_status fcd_step(fcd_handle* h, int32_t nsteps) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (nsteps < 0) return fail(FCD_ERR_ARG, "nsteps must be >= 0");
    if (nsteps > 0) h->init_fresh = 0;
    return FCD_DISPATCH(h, step_impl)(h, nsteps);
}

fcd_status fcd_read_moments(fcd_handle* h, uint32_t mask, double* out) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (!out || mask == 0 || (mask & ~uint32_t(FCD_M_ALL))) return fail(FCD_ERR_ARG, "bad mask or null output");
    return FCD_DISPATCH(h, moments_impl)(h, mask, out);
}

fcd_status fcd_read_state(fcd_handle* h, double* out) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    return FCD_DISPATCH(h, copy_out_impl)(h, h->buf.dist[h->cur], 27, out);
}

fcd_status fcd_write_state(fcd_handle* h, const double* in) {
    if (!h || !in) return fail(FCD_ERR_ARG, "null argument");
    h->init_fresh = 0;
    h->hist = 0;
    h->qs = 0;
    h->last_iters = 0;
    h->track_on = 0;
    h->steps_at_init = h->steps;
    fcd_status st = FCD_DISPATCH(h, copy_in_impl)(h, h->buf.dist[h->cur], 27, in);
    return st ? st : clear_divergence(h);
}

fcd_status fcd_read_psi(fcd_handle* h, double* out) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    return FCD_DISPATCH(h, copy_out_impl)(h, h->buf.psi, 1, out);
}

fcd_status fcd_write_psi(fcd_handle* h, const double* in) {
    if (!h || !in) return fail(FCD_ERR_ARG, "null argument");
    h->hist = 0;
    h->qs = 0;
    h->last_iters = 0;
    return FCD_DISPATCH(h, copy_in_impl)(h, h->buf.psi, 1, in);
}

fcd_status fcd_deformation(fcd_handle* h, double out[4]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    fcd_status st = FCD_DISPATCH(h, diag_impl)(h, out);
    return st ? st : read_divergence(h);
}

fcd_status fcd_extent_deformation(fcd_handle* h, double out[6]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    fcd_status st = FCD_DISPATCH(h, extent_impl)(h, out);
    return st ? st : read_divergence(h);
}

fcd_status fcd_breakup_probe(fcd_handle* h, double out[4]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    fcd_status st = FCD_DISPATCH(h, breakup_impl)(h, out);
    return st ? st : read_divergence(h);
}

fcd_status fcd_breakup_track(fcd_handle* h, double out[6]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    double v[4];
    fcd_status st = FCD_DISPATCH(h, breakup_impl)(h, v);
    if (!st) st = read_divergence(h);
    if (st) return st;
    const double nx = h->lat.nx, ny = h->lat.ny;
    // shortest signed displacement along the periodic channel
    auto wrapped = [&](double d) { return d - nx * std::floor(d / nx + 0.5); };
    const double xo = v[3];
    if (!h->track_on) {
        h->track_on = 1;
        h->track_x_prev = h->track_x_run = xo;
    } else if (!h->open_x) {
        h->track_x_run += wrapped(xo - h->track_x_prev);
        h->track_x_prev = xo;
    }
    out[0] = v[0];
    for (int k = 1; k < 6; ++k) out[k] = -1.0;
    if (v[0] > 0.0) {
        // the contact point, unwrapped through the outer droplet's position (periodic), or
        // the distance from the inlet (open channel: no seam is crossed)
        const double x_b = h->open_x ? v[2] : h->track_x_run + wrapped(v[2] - xo);
        // Eq. 38 with u_avg the velocity scale of the flow: the centreline inflow of Eq. 37
        // (open channel), or the Poiseuille peak the drive sustains (periodic channel)
        const double u_scale =
            h->open_x ? h->u_in : h->prm.drive_G / drive_per_u_ref(h->prm, h->lat.ny);
        const double t_b = (double)(h->steps - h->steps_at_init);
        out[1] = h->r_shell > 0.0 ? t_b * u_scale / (2.0 * h->r_shell) : -1.0;
        out[2] = x_b / ny;
        out[3] = std::fabs(v[1] - (ny - 1) / 2.0) / ny;
        out[4] = x_b;
        out[5] = v[1];
    }
    return FCD_OK;
}

fcd_status fcd_stats(fcd_handle* h, double out[3]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    out[0] = (double)h->steps;
    out[1] = (double)h->sweeps;
    out[2] = h->last_resid;
    return FCD_OK;
}

fcd_status fcd_timing(fcd_handle* h, int32_t enable) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    if (st) return st;
    h->timer.resolve();
    h->timer.clear();
    h->timer.on = enable == 1;
    h->timer.collide_only = enable == 2;
    return FCD_OK;
}

fcd_status fcd_timing_read(fcd_handle* h, double out[12]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    if (st) return st;
    h->timer.resolve();
    for (int k = 0; k < TK_KINDS; ++k) {
        out[2 * k] = h->timer.ms[k];
        out[2 * k + 1] = h->timer.count[k];
    }
    return FCD_OK;
}

fcd_status fcd_sync(fcd_handle* h) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    if (st) return st;
    st = hip_check(hipGetLastError(), "async error");
    return st ? st : read_divergence(h);
}

fcd_status fcd_destroy(fcd_handle* h) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    (void)hipHostFree(h->mirror);
    (void)hipHostFree(h->host);
    delete h;
    return st;
}

const char* fcd_last_error(void) { return g_err.c_str(); }

size_t fcd_adjoint_bytes(const fcd_lattice* lat, int32_t nsteps, int32_t ckpt_every) {
    if (check_lattice(lat) != FCD_OK || nsteps < 1 || ckpt_every < 1) return 0;
    return adj_layout(*lat, nsteps, ckpt_every).bytes;
}

fcd_status fcd_adjoint_forward(fcd_handle* h, int32_t nsteps, int32_t ckpt_every, void* work, double D_out[2]) {
    if (!h || !work || !D_out) return fail(FCD_ERR_ARG, "null argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(FCD_ERR_ARG, "need nsteps >= 1 and ckpt_every >= 1");
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(FCD_ERR_ARG, "work must be 256-byte aligned");
    if (h->prm.pot_every > 1) return fail(FCD_ERR_ARG, "the adjoint needs a potential solve every step (pot_every <= 1)");
    if (h->open_x) return fail(FCD_ERR_ARG, "the adjoint covers the periodic channel only");
    return FCD_DISPATCH(h, adj_forward_impl)(h, nsteps, ckpt_every, static_cast<char*>(work), D_out);
}

fcd_status fcd_adjoint_backward(fcd_handle* h, const double dJ_dD[2], double grad[6]) {
    if (!h || !dJ_dD || !grad) return fail(FCD_ERR_ARG, "null argument");
    return FCD_DISPATCH(h, adj_backward_impl)(h, dJ_dD, grad);
}

fcd_status fcd_batch_sizes(int32_t n, const fcd_lattice* lats, size_t bytes_out[3]) {
    if (!bytes_out) return fail(FCD_ERR_ARG, "bytes_out is null");
    BatchLayout L;
    fcd_status st = batch_layout(n, lats, &L);
    if (st) return st;
    bytes_out[0] = L.state_bytes;
    bytes_out[1] = L.aux_bytes;
    bytes_out[2] = L.scratch_bytes;
    return FCD_OK;
}

fcd_status fcd_batch_create(int32_t n, const fcd_lattice* lats, const fcd_params* prms, void* state, void* aux,
                            void* scratch, void* hip_stream, fcd_batch** out) {
    if (!out) return fail(FCD_ERR_ARG, "out is null");
    *out = nullptr;
    BatchLayout L;
    fcd_status st = batch_layout(n, lats, &L);
    if (st) return st;
    if (!prms) return fail(FCD_ERR_ARG, "params are null");
    for (int k = 0; k < n; ++k) {
        st = check_params(&prms[k]);
        if (st) return st;
    }
    if (!state || !aux || !scratch) return fail(FCD_ERR_ARG, "a device buffer is null");
    for (const void* p : {state, aux, scratch})
        if (reinterpret_cast<uintptr_t>(p) % 256) return fail(FCD_ERR_ARG, "batch buffers must be 256-byte aligned");
    fcd_batch* b = new (std::nothrow) fcd_batch();
    if (!b) return fail(FCD_ERR_OOM, "batch allocation failed");
    b->n = n;
    b->precision = lats[0].precision;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->lat.assign(lats, lats + n);
    b->prm.assign(prms, prms + n);
    b->L = L;
    b->state = static_cast<char*>(state);
    b->aux = static_cast<char*>(aux);
    b->scratch = static_cast<char*>(scratch);
    b->cur = b->hist = b->qs = b->last_iters = 0;
    b->steps = b->iters = 0;
    b->last_resid = 0.0;
    b->shape = 2;  // 64 x 4 tiles
    b->init_fresh = 0;
    b->mg = prms[0].pot_solver == FCD_SOLVER_MG && L.mg_ok;
    b->mg_lds = 0;
    b->mg_last_cycles = b->adj_mg_last_cycles = 0;
    b->adj_work = nullptr;
    b->adj_nsteps = b->adj_every = b->adj_from_init = 0;
    b->adj_final_iters = b->adj_final_hist = b->adj_solve_iters = 0;
    b->block_sweeps = 8 * std::max(1, prms[0].pot_check_every);
    b->fused = 0;  // default: the deepest fusion allowed up to two sweeps per launch
    for (int f = 2; f >= 1 && b->fused == 0; --f)
        if (fused_allowed(b, f)) b->fused = f;
    // and four sweeps per launch after 16 tests
    b->tail_fused = fused_allowed(b, 4) ? 4 : 0;
    b->tail_after = 16 * check_interval(b);
    if (hipHostMalloc(reinterpret_cast<void**>(&b->host), (2 + 4 * (size_t)n) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        delete b;
        return fail(FCD_ERR_OOM, "pinned host allocation failed");
    }
    st = FCD_BDISPATCH(b, batch_upload)(b);
    if (st) {
        (void)hipHostFree(b->host);
        delete b;
        return st;
    }
    *out = b;
    return FCD_OK;
}

fcd_status fcd_batch_init_compound_droplet(fcd_batch* b, const double* geom) {
    if (!b || !geom) return fail(FCD_ERR_ARG, "null argument");
    for (int k = 0; k < b->n; ++k)
        if (!(geom[4 * k + 2] >= 0.0) || !(geom[4 * k + 3] >= geom[4 * k + 2]))
            return fail(FCD_ERR_ARG, "need 0 <= r_core <= r_shell");
    return FCD_BDISPATCH(b, batch_init_impl)(b, geom);
}

fcd_status fcd_batch_step(fcd_batch* b, int32_t nsteps) {
    if (!b) return fail(FCD_ERR_ARG, "batch is null");
    if (nsteps < 0) return fail(FCD_ERR_ARG, "nsteps must be >= 0");
    if (nsteps > 0) b->init_fresh = 0;
    return FCD_BDISPATCH(b, batch_step_impl)(b, nsteps);
}

fcd_status fcd_batch_deformation(fcd_batch* b, double* out) {
    if (!b || !out) return fail(FCD_ERR_ARG, "null argument");
    return FCD_BDISPATCH(b, batch_diag_impl)(b, out);
}

fcd_status fcd_batch_read_state(fcd_batch* b, int32_t k, double* out) {
    if (!b || !out || k < 0 || k >= b->n) return fail(FCD_ERR_ARG, "bad batch channel or null output");
    return FCD_BDISPATCH(b, batch_state_impl)(b, k, out);
}

fcd_status fcd_batch_read_moments(fcd_batch* b, int32_t k, uint32_t mask, double* out) {
    if (!b || !out || k < 0 || k >= b->n) return fail(FCD_ERR_ARG, "bad batch channel or null output");
    if (mask == 0 || (mask & ~uint32_t(FCD_M_ALL))) return fail(FCD_ERR_ARG, "bad mask");
    return FCD_BDISPATCH(b, batch_moments_impl)(b, k, mask, out);
}

fcd_status fcd_batch_autotune(fcd_batch* b, int32_t steps_per_candidate, int32_t choice[5]) {
    if (!b || !choice) return fail(FCD_ERR_ARG, "null argument");
    if (steps_per_candidate < 1) return fail(FCD_ERR_ARG, "steps_per_candidate must be >= 1");
    return FCD_BDISPATCH(b, batch_autotune_impl)(b, steps_per_candidate, choice);
}

fcd_status fcd_batch_tune_omega(fcd_batch* b, int32_t steps, int32_t ncand, const double* scale, double* omega_out) {
    if (!b || !scale || !omega_out) return fail(FCD_ERR_ARG, "null argument");
    if (steps < 1 || ncand < 1 || ncand > 16) return fail(FCD_ERR_ARG, "need steps >= 1 and 1 <= ncand <= 16");
    for (int c = 0; c < ncand; ++c)
        if (!(scale[c] > 0.0 && scale[c] < 10.0)) return fail(FCD_ERR_ARG, "candidate scales must lie in (0, 10)");
    return FCD_BDISPATCH(b, batch_tune_omega_impl)(b, steps, ncand, scale, omega_out);
}

fcd_status fcd_batch_set_schedule(fcd_batch* b, int32_t tile_rows, int32_t block_sweeps, int32_t fused_sweeps) {
    if (!b) return fail(FCD_ERR_ARG, "batch is null");
    int s = -1;
    for (int k = 0; k < fcd::BATCH_SHAPES; ++k)
        if (BT_ROWS[k] == tile_rows) s = k;
    if (s < 0) return fail(FCD_ERR_ARG, "tile_rows must be 1, 2, 4 or 8");
    if (block_sweeps < 1 || block_sweeps > (1 << 20) || block_sweeps % check_interval(b))
        return fail(FCD_ERR_ARG, "block_sweeps must be a positive multiple of pot_check_every, at most 2^20");
    if (!fused_allowed(b, fused_sweeps) || (fused_sweeps > 0 && block_sweeps % (2 * fused_sweeps)))
        return fail(FCD_ERR_ARG,
                    "fused_sweeps must be 0, 1 or 2 with pot_check_every a multiple of 2 fused_sweeps, or 4 with "
                    "pot_check_every a multiple of 4; block_sweeps a multiple of 2 fused_sweeps");
    b->shape = s;
    b->block_sweeps = block_sweeps;
    b->fused = fused_sweeps;
    return FCD_OK;
}

fcd_status fcd_batch_set_tail_fusion(fcd_batch* b, int32_t fused_sweeps, int32_t after_sweeps) {
    if (!b) return fail(FCD_ERR_ARG, "batch is null");
    if (after_sweeps < 0) return fail(FCD_ERR_ARG, "after_sweeps must be >= 0");
    if (fused_sweeps != 0 && (!fused_allowed(b, fused_sweeps) || fused_sweeps == 0))
        return fail(FCD_ERR_ARG, "tail fused_sweeps must be 0 (off) or a fusion the test interval allows");
    b->tail_fused = fused_sweeps;
    b->tail_after = after_sweeps;
    return FCD_OK;
}

size_t fcd_batch_adjoint_bytes(fcd_batch* b, int32_t nsteps, int32_t ckpt_every) {
    if (!b || nsteps < 1 || ckpt_every < 1) return 0;
    return batch_adj_layout(b, nsteps, ckpt_every).bytes;
}

fcd_status fcd_batch_adjoint_forward(fcd_batch* b, int32_t nsteps, int32_t ckpt_every, void* work, double* D_out) {
    if (!b || !work || !D_out) return fail(FCD_ERR_ARG, "null argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(FCD_ERR_ARG, "need nsteps >= 1 and ckpt_every >= 1");
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(FCD_ERR_ARG, "work must be 256-byte aligned");
    if (b->prm[0].pot_every > 1)
        return fail(FCD_ERR_ARG, "the adjoint needs a potential solve every step (pot_every <= 1)");
    return FCD_BDISPATCH(b, batch_adj_forward_impl)(b, nsteps, ckpt_every, static_cast<char*>(work), D_out);
}

fcd_status fcd_batch_adjoint_backward(fcd_batch* b, const double* dJ_dD, double* grad) {
    if (!b || !dJ_dD || !grad) return fail(FCD_ERR_ARG, "null argument");
    return FCD_BDISPATCH(b, batch_adj_backward_impl)(b, dJ_dD, grad);
}

fcd_status fcd_batch_stats(fcd_batch* b, double out[3]) {
    if (!b || !out) return fail(FCD_ERR_ARG, "null argument");
    out[0] = (double)b->steps;
    out[1] = (double)b->iters;
    out[2] = b->last_resid;
    return FCD_OK;
}

fcd_status fcd_batch_destroy(fcd_batch* b) {
    if (!b) return fail(FCD_ERR_ARG, "batch is null");
    fcd_status st = hip_check(hipStreamSynchronize(b->stream), "stream sync");
    (void)hipHostFree(b->host);
    delete b;
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// No-allocation deformation (fcd_deformation_noalloc).  The row partial sums and the
// centroids of the two diagnostic passes live in this file-scope device array instead of
// a caller's scratch buffer; each GPU holds its own copy until the process ends.  Host
// code never passes `scratch` itself to a kernel: its device address on each GPU comes
// from hipGetSymbolAddress, taken once per device with that device current.  Every value
// of the array is written before it is read (rows by the first pass, centroids by its
// final kernel), so nothing needs clearing between calls.
// ---------------------------------------------------------------------------------
namespace {

constexpr int NOALLOC_MAX_NY = FCD_NOALLOC_MAX_NY;
constexpr int NOALLOC_CENT = 32;  // doubles: centroids, masses and the pass-0 sums
constexpr size_t NOALLOC_DOUBLES = (size_t)NOALLOC_MAX_NY * 8 + NOALLOC_CENT;

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mutex;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's address of `scratch` (set up on the first call on that device).
fcd_status noalloc_scratch(double** out) {
    int dev = -1;
    fcd_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(FCD_ERR_UNSUPPORTED, "device index beyond 64");
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st) return st;
        if (!p) return fail(FCD_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
        g_noalloc_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return FCD_OK;
}

template <typename T>
fcd_status deformation_noalloc_impl(const fcd_lattice* lat, const void* phi, hipStream_t stream, double* out) {
    double* base = nullptr;
    fcd_status st = noalloc_scratch(&base);
    if (st) return st;
    fcd::StepConst<T> P{};
    P.nx = lat->nx;
    P.ny = lat->ny;
    P.pitch = lat->pitch;
    P.plane = (long long)lat->ny * lat->pitch;
    double* rows = base;
    double* cent = base + (size_t)NOALLOC_MAX_NY * 8;
    fcd::launch_diagnostics<T>(static_cast<const T*>(phi), P, rows, cent, out, stream);
    return hip_check(hipGetLastError(), "diagnostics launch");
}

}  // namespace

extern "C" {

fcd_status fcd_deformation_noalloc(const fcd_lattice* lat, const void* phi, void* hip_stream, double* out) {
    fcd_status st = check_lattice(lat);
    if (st) return st;
    if (!phi || !out) return fail(FCD_ERR_ARG, "null argument");
    if (lat->ny > NOALLOC_MAX_NY)
        return fail(FCD_ERR_ARG, "fcd_deformation_noalloc: ny exceeds FCD_NOALLOC_MAX_NY (" +
                                     std::to_string(NOALLOC_MAX_NY) + ")");
    if (reinterpret_cast<uintptr_t>(phi) % elem_size(lat->precision) || reinterpret_cast<uintptr_t>(out) % 8)
        return fail(FCD_ERR_ARG, "misaligned device buffer");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return lat->precision == FCD_FP64 ? deformation_noalloc_impl<double>(lat, phi, s, out)
                                      : deformation_noalloc_impl<float>(lat, phi, s, out);
}

}  // extern "C"

