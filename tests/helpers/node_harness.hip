// Host-only harness (test infrastructure): exposes the library's per-node forward and
// its hand-written adjoint to Python so the adjoint can be checked against central
// finite differences of the forward on the CPU.
#include <cstring>

#include "fcd_adjoint.hpp"

using fcd::Nb9;
using fcd::StepConst;

namespace {
StepConst<double> unpack(const double* p) {
    StepConst<double> c{};
    c.nx = c.ny = c.pitch = 1;
    c.plane = 1;
    double* d[] = {&c.rho0, &c.rho1, &c.rho2, &c.tau0, &c.tau1, &c.tau2, &c.ic0, &c.ic1, &c.ic2,
                   &c.gam0, &c.gam1, &c.gam2, &c.igam0, &c.igam1, &c.igam2, &c.s12, &c.s13, &c.s23,
                   &c.eta, &c.c_bulk, &c.c_lap, &c.four_over_xi, &c.omega_phi, &c.H0x, &c.H0y,
                   &c.half_mu0, &c.drive, &c.grav_x, &c.grav_y, &c.eps2};
    for (int k = 0; k < 30; ++k) *d[k] = p[k];
    return c;
}
Nb9<double> nb(const double* v) {
    Nb9<double> n;
    n.c = v[0]; n.e = v[1]; n.n = v[2]; n.w = v[3]; n.s = v[4]; n.ne = v[5]; n.nw = v[6]; n.sw = v[7]; n.se = v[8];
    return n;
}
}  // namespace

// in: f[9], g1[9], g2[9], a1[9], a2[9], ps[9] (stencils ordered c, e, n, w, s, ne, nw, sw, se)
extern "C" void harness_forward(const double* prm, const double* in, double* out) {
    const StepConst<double> P = unpack(prm);
    fcd::node_forward(P, in, in + 9, in + 18, nb(in + 27), nb(in + 36), nb(in + 45), out, out + 9, out + 18);
}

// out: adjoint of f, g1, g2 (27); phi1 (p, gx, gy, lap), phi2 (same), grad psi' (2);
// parameter partials H0x, H0y, drive, s12, s13, s23, gam0..2, igam0..2, cbulk (13).
extern "C" void harness_vjp(const double* prm, const double* in, const double* ybar, double* out) {
    const StepConst<double> P = unpack(prm);
    const fcd::NodeAdj<double> R = fcd::node_adjoint(P, in, in + 9, in + 18, nb(in + 27), nb(in + 36), nb(in + 45),
                                                     ybar, ybar + 9, ybar + 18);
    std::memcpy(out, R.f, 9 * sizeof(double));
    std::memcpy(out + 9, R.g1, 9 * sizeof(double));
    std::memcpy(out + 18, R.g2, 9 * sizeof(double));
    const double rest[] = {R.p1, R.gx1, R.gy1, R.l1, R.p2, R.gx2, R.gy2, R.l2, R.gpx, R.gpy,
                           R.H0x, R.H0y, R.drive, R.s12, R.s13, R.s23, R.gam0, R.gam1, R.gam2,
                           R.igam0, R.igam1, R.igam2, R.cbulk};
    std::memcpy(out + 27, rest, sizeof(rest));
}
