// fcd_abi.hip -- the C ABI declared in include/fcd.h: argument checks, per-step
// orchestration of the kernels on the caller's stream, potential-solve control.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fcd.h"
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
constexpr size_t OFF_RES = 0;      // uint64: bit pattern of max |residual|
constexpr size_t OFF_CENT = 256;   // 8 doubles: centroids and masses
constexpr size_t OFF_RESULT = 512; // 4 doubles: D_o, D_i, mass1, mass2
constexpr size_t OFF_ROWS = 1024;  // ny * 8 doubles: per-row partial sums

size_t elem_size(int precision) { return precision == FCD_FP64 ? sizeof(double) : sizeof(float); }

// Over-relaxation factor: the caller's, or the optimum 2 / (1 + sin(pi h)) of SOR for
// the Laplacian between Dirichlet rows ny + 1 cells apart.
double sor_omega_of(const fcd_params& p, int ny) {
    if (p.sor_omega > 0.0) return p.sor_omega;
    return 2.0 / (1.0 + std::sin(3.14159265358979323846 / (ny + 1)));
}

}  // namespace

// Event pairs bracketing launches, resolved into per-class totals after a sync.
struct Timer {
    struct Pair {
        int kind;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<Pair> pending;
    std::vector<hipEvent_t> pool;
    double ms[4] = {0, 0, 0, 0};
    double count[4] = {0, 0, 0, 0};

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
        for (int k = 0; k < 4; ++k) ms[k] = count[k] = 0;
    }
    ~Timer() {
        for (const Pair& p : pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

enum { TK_COLLIDE = 0, TK_SWEEP = 1, TK_RESID = 2, TK_PHASE = 3 };

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
    if (!(p->sor_omega == 0.0 || (p->sor_omega > 0.0 && p->sor_omega < 2.0)))
        return fail(FCD_ERR_ARG, "sor_omega must be 0 (automatic) or lie in (0, 2)");
    if (!(p->sor_tol > 0.0)) return fail(FCD_ERR_ARG, "sor_tol must be positive");
    if (p->sor_check_every < 1 || p->sor_max_sweeps < 0) return fail(FCD_ERR_ARG, "bad SOR sweep counts");
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
    return c;
}

template <typename T>
T* plane_ptr(void* base, const fcd_handle* h, int q) {
    return static_cast<T*>(base) + (long long)q * h->lat.ny * h->lat.pitch;
}

unsigned long long* res_word(const fcd_handle* h) {
    return reinterpret_cast<unsigned long long*>(static_cast<char*>(h->buf.scratch) + OFF_RES);
}

template <typename T>
fcd_status read_residual(fcd_handle* h, const fcd::StepConst<T>& P, T* psi, const T* mur, double* r) {
    hipEvent_t ev = nullptr;
    const bool timed = h->timer.begin(h->stream, &ev);
    fcd::launch_residual<T>(psi, mur, P, res_word(h), h->stream);
    if (timed) h->timer.end(h->stream, TK_RESID, ev);
    fcd_status st = hip_check(hipGetLastError(), "residual launch");
    if (st) return st;
    st = hip_check(hipMemcpyAsync(h->host, res_word(h), sizeof(double), hipMemcpyDeviceToHost, h->stream),
                   "residual copy");
    if (st) return st;
    st = hip_check(hipStreamSynchronize(h->stream), "residual sync");
    if (st) return st;
    h->timer.resolve();
    std::memcpy(r, h->host, sizeof(double));
    return FCD_OK;
}

// Four-colour SOR on the current mu_r plane, warm-started from the stored psi'.
template <typename T>
fcd_status solve_impl(fcd_handle* h, double tol, int max_sweeps, int* sweeps_out, double* resid_out) {
    const fcd::StepConst<T> P = make_const<T>(h);
    T* psi = static_cast<T*>(h->buf.psi);
    const T* mur = plane_ptr<T>(h->buf.phi, h, 2);
    if (sweeps_out) *sweeps_out = 0;
    if (h->prm.H0 == 0.0) {  // no applied field: psi' = 0 exactly
        fcd::launch_fill<T>(psi, (long long)h->lat.ny * h->lat.pitch, T(0), h->stream);
        if (resid_out) *resid_out = 0.0;
        h->last_resid = 0.0;
        return hip_check(hipGetLastError(), "fill");
    }
    const double thr = tol * std::fabs(h->prm.H0);
    const int every = h->prm.sor_check_every;
    double r = 0.0;
    fcd_status st = read_residual<T>(h, P, psi, mur, &r);
    if (st) return st;
    int sw = 0;
    while (!(r <= thr)) {
        if (r != r) {
            h->last_resid = r;
            return fail(FCD_ERR_DIVERGED, "potential residual is NaN");
        }
        if (sw >= max_sweeps) break;
        const int m = every < max_sweeps - sw ? every : max_sweeps - sw;
        const T omega = T(sor_omega_of(h->prm, h->lat.ny));
        for (int s = 0; s < m; ++s) {
            hipEvent_t ev = nullptr;
            const bool timed = h->timer.begin(h->stream, &ev);
            fcd::launch_sor_sweep<T>(psi, mur, P, omega, h->stream);
            if (timed) h->timer.end(h->stream, TK_SWEEP, ev);
        }
        sw += m;
        st = read_residual<T>(h, P, psi, mur, &r);
        if (st) return st;
    }
    h->sweeps += sw;
    h->last_resid = r;
    if (sweeps_out) *sweeps_out = sw;
    if (resid_out) *resid_out = r;
    if (!(r <= thr)) return fail(FCD_ERR_NOT_CONVERGED, "potential solve reached max_sweeps");
    return FCD_OK;
}

template <typename T>
fcd_status step_impl(fcd_handle* h, int nsteps) {
    const fcd::StepConst<T> P = make_const<T>(h);
    T* phi = static_cast<T*>(h->buf.phi);
    for (int n = 0; n < nsteps; ++n) {
        const T* src = static_cast<const T*>(h->buf.dist[h->cur]);
        T* dst = static_cast<T*>(h->buf.dist[1 - h->cur]);
        hipEvent_t ev = nullptr;
        bool timed = h->timer.begin(h->stream, &ev);
        fcd::launch_phase<T>(src, phi, P, h->stream);
        if (timed) h->timer.end(h->stream, TK_PHASE, ev);
        fcd_status st = hip_check(hipGetLastError(), "phase launch");
        if (st) return st;
        st = solve_impl<T>(h, h->prm.sor_tol, h->prm.sor_max_sweeps, nullptr, nullptr);
        if (st) return st;
        timed = h->timer.begin(h->stream, &ev);
        fcd::launch_collide_stream<T>(src, dst, phi, static_cast<const T*>(h->buf.psi), P, h->stream);
        if (timed) h->timer.end(h->stream, TK_COLLIDE, ev);
        st = hip_check(hipGetLastError(), "collide-stream launch");
        if (st) return st;
        h->cur = 1 - h->cur;
        ++h->steps;
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
fcd_status init_fields_impl(fcd_handle* h, const double* phi1, const double* phi2, const double* ux,
                            const double* uy, const double* ps) {
    fcd::launch_init_fields<T>(static_cast<T*>(h->buf.dist[h->cur]), phi1, phi2, ux, uy, ps, h->lat.nx, h->lat.ny,
                               h->lat.pitch, h->stream);
    fcd::launch_fill<T>(static_cast<T*>(h->buf.psi), (long long)h->lat.ny * h->lat.pitch, T(0), h->stream);
    return hip_check(hipGetLastError(), "init launch");
}

template <typename T>
fcd_status init_droplet_impl(fcd_handle* h, double xc, double yc, double rc, double rs) {
    const double nu3 = h->prm.tau[2] / 3.0;
    const double u_scale = h->prm.drive_G / (2.0 * h->prm.rho[2] * nu3);
    fcd::launch_init_droplet<T>(static_cast<T*>(h->buf.dist[h->cur]), h->lat.nx, h->lat.ny, h->lat.pitch, xc, yc, rc,
                                rs, h->prm.xi, u_scale, h->stream);
    fcd::launch_fill<T>(static_cast<T*>(h->buf.psi), (long long)h->lat.ny * h->lat.pitch, T(0), h->stream);
    return hip_check(hipGetLastError(), "init launch");
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

}  // namespace

extern "C" {

size_t fcd_scratch_bytes(const fcd_lattice* lat) {
    if (!lat || lat->ny < 1) return 0;
    return OFF_ROWS + (size_t)lat->ny * 8 * sizeof(double);
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
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host), 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return fail(FCD_ERR_OOM, "pinned host allocation failed");
    }
    *out = h;
    return FCD_OK;
}

fcd_status fcd_set_params(fcd_handle* h, const fcd_params* prm) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = check_params(prm);
    if (st) return st;
    h->prm = *prm;
    return FCD_OK;
}

fcd_status fcd_init_compound_droplet(fcd_handle* h, double xc, double yc, double r_core, double r_shell) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (!(r_core >= 0.0) || !(r_shell >= r_core)) return fail(FCD_ERR_ARG, "need 0 <= r_core <= r_shell");
    return FCD_DISPATCH(h, init_droplet_impl)(h, xc, yc, r_core, r_shell);
}

fcd_status fcd_init_fields(fcd_handle* h, const double* phi1, const double* phi2, const double* ux,
                           const double* uy, const double* pstar) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (!phi1 || !phi2 || !ux || !uy) return fail(FCD_ERR_ARG, "a field pointer is null");
    return FCD_DISPATCH(h, init_fields_impl)(h, phi1, phi2, ux, uy, pstar);
}

fcd_status fcd_solve_potential(fcd_handle* h, double tol, int32_t max_sweeps, int32_t* sweeps_out,
                               double* resid_out) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (!(tol > 0.0) || max_sweeps < 0) return fail(FCD_ERR_ARG, "bad tolerance or sweep limit");
    fcd_status st = FCD_DISPATCH(h, refresh_phase)(h);
    if (st) return st;
    int sw = 0;
    st = FCD_DISPATCH(h, solve_impl)(h, tol, max_sweeps, &sw, resid_out);
    if (sweeps_out) *sweeps_out = sw;
    return st;
}

fcd_status fcd_step(fcd_handle* h, int32_t nsteps) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    if (nsteps < 0) return fail(FCD_ERR_ARG, "nsteps must be >= 0");
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
    return FCD_DISPATCH(h, copy_in_impl)(h, h->buf.dist[h->cur], 27, in);
}

fcd_status fcd_read_psi(fcd_handle* h, double* out) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    return FCD_DISPATCH(h, copy_out_impl)(h, h->buf.psi, 1, out);
}

fcd_status fcd_write_psi(fcd_handle* h, const double* in) {
    if (!h || !in) return fail(FCD_ERR_ARG, "null argument");
    return FCD_DISPATCH(h, copy_in_impl)(h, h->buf.psi, 1, in);
}

fcd_status fcd_deformation(fcd_handle* h, double out[4]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    return FCD_DISPATCH(h, diag_impl)(h, out);
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
    h->timer.on = enable != 0;
    return FCD_OK;
}

fcd_status fcd_timing_read(fcd_handle* h, double out[8]) {
    if (!h || !out) return fail(FCD_ERR_ARG, "null argument");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    if (st) return st;
    h->timer.resolve();
    for (int k = 0; k < 4; ++k) {
        out[2 * k] = h->timer.ms[k];
        out[2 * k + 1] = h->timer.count[k];
    }
    return FCD_OK;
}

fcd_status fcd_sync(fcd_handle* h) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    if (st) return st;
    return hip_check(hipGetLastError(), "async error");
}

fcd_status fcd_destroy(fcd_handle* h) {
    if (!h) return fail(FCD_ERR_ARG, "handle is null");
    fcd_status st = hip_check(hipStreamSynchronize(h->stream), "stream sync");
    (void)hipHostFree(h->host);
    delete h;
    return st;
}

const char* fcd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
