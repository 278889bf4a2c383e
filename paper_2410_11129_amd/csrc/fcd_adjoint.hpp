// fcd_adjoint.hpp -- reverse (adjoint) of one node of the fused collide pass.
//
// Given the adjoints Y of the node's post-collision distributions (f*, g1*, g2*),
// node_adjoint returns the adjoints of everything the node update reads: its own
// distributions f, g1, g2, the phi1 / phi2 stencil quantities (centre value, isotropic
// gradient, Laplacian), the psi' gradient, and the step constants through which the
// parameters enter (H0 cos a, H0 sin a, the drive, the surface tensions and the
// coefficients derived from them).  The forward quantities are recomputed first in
// exactly the order of node_physics / collide_f / collide_g, then every assignment is
// reversed.  Callable from host code so it can be checked against finite differences
// of the forward node on the CPU.
#pragma once

#include <hip/hip_runtime.h>

#include "fcd_device.hpp"

namespace fcd {

template <typename T>
struct NodeAdj {
    T f[9], g1[9], g2[9];      // adjoint of the node's own distributions
    T p1, gx1, gy1, l1;        // phi1: centre value, gradient, Laplacian
    T p2, gx2, gy2, l2;        // phi2
    T gpx, gpy;                // gradient of psi'
    // step constants
    T H0x, H0y, drive, s12, s13, s23, gam0, gam1, gam2, igam0, igam1, igam2, cbulk;
};

template <typename T>
__host__ __device__ __forceinline__ void adj_collide_g(const NodeOut<T>& o, T om, T phi, T vx, T vy, const T Y[9],
                                                       T gbar[9], T& phibar, T& uxb, T& uyb, T& vxb, T& vyb) {
    const T ux = o.ux, uy = o.uy;
    const T usq = T(1.5) * (ux * ux + uy * uy);
    const T w0 = T(4) / T(9), wa = T(1) / T(9), wd = T(1) / T(36);
    const T keep = T(1) - om, op = om * phi, fs = T(1) - T(0.5) * om;
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    T opb = T(0), usqb = T(0), evb_x = T(0), evb_y = T(0), eub_x = T(0), eub_y = T(0);
    // rest: out0 = keep g0 + op w0 (1 - usq)
    gbar[0] = keep * Y[0];
    opb += Y[0] * w0 * (T(1) - usq);
    usqb -= Y[0] * op * w0;
    for (int a = 1; a < 9; ++a) {
        const T w = a < 5 ? wa : wd;
        const T eu = ex[a] * ux + ey[a] * uy;
        const T gam = w * (T(1) + T(3) * eu + T(4.5) * eu * eu - usq);
        gbar[a] = keep * Y[a];
        opb += Y[a] * gam;
        const T gamb = op * Y[a];
        const T eub = gamb * w * (T(3) + T(9) * eu);
        usqb -= gamb * w;
        eub_x += eub * ex[a];
        eub_y += eub * ey[a];
        const T evb = fs * w * Y[a];
        evb_x += evb * ex[a];
        evb_y += evb * ey[a];
    }
    phibar += om * opb;
    uxb += eub_x + usqb * T(3) * ux;
    uyb += eub_y + usqb * T(3) * uy;
    vxb += evb_x;
    vyb += evb_y;
    (void)vx;
    (void)vy;
}

template <typename T>
__host__ __device__ __forceinline__ void adj_collide_f(const NodeOut<T>& o, const T f[9], const T Y[9], T fbar[9],
                                                       T& pstarb, T& uxb, T& uyb, T& Ftxb, T& Ftyb, T& rhob,
                                                       T& taub) {
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const T w0 = T(4) / T(9), wa = T(1) / T(9), wd = T(1) / T(36);
    const T ux = o.ux, uy = o.uy;
    const T usq = T(1.5) * (ux * ux + uy * uy);
    const T fr = T(3) / o.rho;
    const T fx = fr * o.Ftx, fy = fr * o.Fty;
    // forward intermediates
    T fb[9], F[9], eu[9];
    F[0] = T(0);
    eu[0] = T(0);
    fb[0] = w0 * (o.pstar - usq);
    for (int a = 1; a < 9; ++a) {
        const T w = a < 5 ? wa : wd;
        eu[a] = ex[a] * ux + ey[a] * uy;
        F[a] = w * (ex[a] * fx + ey[a] * fy);
        fb[a] = w * (o.pstar + T(3) * eu[a] + T(4.5) * eu[a] * eu[a] - usq) - T(0.5) * F[a];
    }
    const T mxx = ((f[1] + f[3]) - (f[2] + f[4])) - ((fb[1] + fb[3]) - (fb[2] + fb[4]));
    const T mxy = ((f[5] + f[7]) - (f[6] + f[8])) - ((fb[5] + fb[7]) - (fb[6] + fb[8]));
    const T tp = o.tau + T(0.5);
    const T k = T(0.25) * (T(1) - T(1) / tp);
    // reverse
    T fbb[9], Fb[9];
    for (int a = 0; a < 9; ++a) {
        fbb[a] = Y[a];
        Fb[a] = a == 0 ? T(0) : Y[a];
        fbar[a] = T(0);
    }
    const T kxb = (Y[1] + Y[3]) - (Y[2] + Y[4]);
    const T kyb = (Y[5] + Y[7]) - (Y[6] + Y[8]);
    const T mxxb = k * kxb, mxyb = k * kyb;
    const T kb = mxx * kxb + mxy * kyb;
    taub += kb * T(0.25) / (tp * tp);
    fbar[1] += mxxb;
    fbar[3] += mxxb;
    fbar[2] -= mxxb;
    fbar[4] -= mxxb;
    fbb[1] -= mxxb;
    fbb[3] -= mxxb;
    fbb[2] += mxxb;
    fbb[4] += mxxb;
    fbar[5] += mxyb;
    fbar[7] += mxyb;
    fbar[6] -= mxyb;
    fbar[8] -= mxyb;
    fbb[5] -= mxyb;
    fbb[7] -= mxyb;
    fbb[6] += mxyb;
    fbb[8] += mxyb;
    T usqb = -w0 * fbb[0];
    pstarb += w0 * fbb[0];
    T eub_x = T(0), eub_y = T(0), fxb = T(0), fyb = T(0);
    for (int a = 1; a < 9; ++a) {
        const T w = a < 5 ? wa : wd;
        pstarb += w * fbb[a];
        const T eub = fbb[a] * w * (T(3) + T(9) * eu[a]);
        eub_x += eub * ex[a];
        eub_y += eub * ey[a];
        usqb -= w * fbb[a];
        Fb[a] -= T(0.5) * fbb[a];
        const T efb = w * Fb[a];
        fxb += efb * ex[a];
        fyb += efb * ey[a];
    }
    Ftxb += fr * fxb;
    Ftyb += fr * fyb;
    const T frb = o.Ftx * fxb + o.Fty * fyb;
    rhob += frb * (-T(3) / (o.rho * o.rho));
    uxb += eub_x + usqb * T(3) * ux;
    uyb += eub_y + usqb * T(3) * uy;
}

template <typename T>
__host__ __device__ inline NodeAdj<T> node_adjoint(const StepConst<T>& P, const T f[9], const T g1[9], const T g2[9],
                                                   const Nb9<T>& a1, const Nb9<T>& a2, const Nb9<T>& ps,
                                                   const T Yf[9], const T Yg1[9], const T Yg2[9]) {
    NodeAdj<T> R{};
    // ---------------- forward recomputation (as node_physics) ----------------
    const T p1 = a1.c, p2 = a2.c, p3 = T(1) - p1 - p2;
    T g1x, g1y, g2x, g2y;
    iso_grad(a1, g1x, g1y);
    iso_grad(a2, g2x, g2y);
    const T l1 = iso_lap(a1), l2 = iso_lap(a2);
    const T g3x = -(g1x + g2x), g3y = -(g1y + g2y), l3 = -(l1 + l2);
    const T fx_ = P.four_over_xi;
    const T t1 = fx_ * p1 * (T(1) - p1), t2 = fx_ * p2 * (T(1) - p2), t3 = fx_ * p3 * (T(1) - p3);
    const T q1 = g1x * g1x + g1y * g1y + P.eps2, q2 = g2x * g2x + g2y * g2y + P.eps2,
            q3 = g3x * g3x + g3y * g3y + P.eps2;
    const T n1 = rsqrt_t(q1), n2 = rsqrt_t(q2), n3 = rsqrt_t(q3);
    const T r1 = t1 * n1, r2 = t2 * n2, r3 = t3 * n3;
    const T rho = P.rho0 * p1 + P.rho1 * p2 + P.rho2 * p3;
    const T tau = P.tau0 * p1 + P.tau1 * p2 + P.tau2 * p3;
    const T grx = P.rho0 * g1x + P.rho1 * g2x + P.rho2 * g3x;
    const T gry = P.rho0 * g1y + P.rho1 * g2y + P.rho2 * g3y;
    const T S = P.ic0 * p1 + P.ic1 * p2 + P.ic2 * p3;
    const T iS2 = T(1) / (S * S);
    const T Gx = P.ic0 * g1x + P.ic1 * g2x + P.ic2 * g3x;
    const T Gy = P.ic0 * g1y + P.ic1 * g2y + P.ic2 * g3y;
    const T gcx = -Gx * iS2, gcy = -Gy * iS2;
    const T q = P.gam0 * p1 + P.gam1 * p2 + P.gam2 * p3;
    const T p123 = p1 * p2 * p3;
    const T e2 = T(2) * P.eta * p123;
    const T dH1 = T(2) * p1 * (P.s12 * p2 * p2 + P.s13 * p3 * p3) + p2 * p3 * q + p123 * P.gam0 + e2 * p2 * p3;
    const T dH2 = T(2) * p2 * (P.s12 * p1 * p1 + P.s23 * p3 * p3) + p1 * p3 * q + p123 * P.gam1 + e2 * p1 * p3;
    const T dH3 = T(2) * p3 * (P.s13 * p1 * p1 + P.s23 * p2 * p2) + p1 * p2 * q + p123 * P.gam2 + e2 * p1 * p2;
    const T m1 = P.c_bulk * ((dH1 - dH2) * P.igam1 + (dH1 - dH3) * P.igam2) - P.c_lap * P.gam0 * l1;
    const T m2 = P.c_bulk * ((dH2 - dH1) * P.igam0 + (dH2 - dH3) * P.igam2) - P.c_lap * P.gam1 * l2;
    const T m3 = P.c_bulk * ((dH3 - dH1) * P.igam0 + (dH3 - dH2) * P.igam1) - P.c_lap * P.gam2 * l3;
    T gpx, gpy;
    iso_grad(ps, gpx, gpy);
    const T Hx = P.H0x - gpx, Hy = P.H0y - gpy;
    const T kel = -P.half_mu0 * (Hx * Hx + Hy * Hy);
    const T pstar = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const T jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const T jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const T dd = (f[5] + f[6]) + (f[7] + f[8]);
    const T sxx = (f[1] + f[3]) + dd, syy = (f[2] + f[4]) + dd;
    const T sxy = (f[5] - f[6]) + (f[7] - f[8]);
    const T cp = -pstar * (T(1) / T(3));
    const T Fsx = m1 * g1x + m2 * g2x + m3 * g3x, Fsy = m1 * g1y + m2 * g2y + m3 * g3y;
    const T Fmx = kel * gcx, Fmy = kel * gcy;
    const T F0x = Fsx + Fmx + cp * grx + P.drive + rho * P.grav_x;
    const T F0y = Fsy + Fmy + cp * gry + rho * P.grav_y;
    const T ihr = T(0.5) / rho;
    const T u0x = jx + F0x * ihr, u0y = jy + F0y * ihr;
    const T A = sxx - pstar * (T(1) / T(3)) - u0x * u0x;
    const T B = syy - pstar * (T(1) / T(3)) - u0y * u0y;
    const T C = sxy - u0x * u0y;
    const T snu = T(1) / (tau + T(0.5));
    const T ho = T(0.5) * (T(1) - snu) * (A - B);
    const T Pxx = A - ho, Pyy = B + ho, Pxy = snu * C;
    const T Fmux = -tau * (Pxx * grx + Pxy * gry), Fmuy = -tau * (Pxy * grx + Pyy * gry);
    NodeOut<T> o;
    o.Ftx = F0x + Fmux;
    o.Fty = F0y + Fmuy;
    o.ux = jx + o.Ftx * ihr;
    o.uy = jy + o.Fty * ihr;
    o.pstar = pstar;
    o.rho = rho;
    o.tau = tau;
    o.phi1 = p1;
    o.phi2 = p2;
    const T sx = (r1 * g1x + r2 * g2x + r3 * g3x) * (T(1) / T(3));
    const T sy = (r1 * g1y + r2 * g2y + r3 * g3y) * (T(1) / T(3));
    o.v1x = r1 * g1x - sx;
    o.v1y = r1 * g1y - sy;
    o.v2x = r2 * g2x - sx;
    o.v2y = r2 * g2y - sy;

    // ---------------- reverse: collisions ----------------
    T uxb = T(0), uyb = T(0), Ftxb = T(0), Ftyb = T(0), rhob = T(0), taub = T(0), pstarb = T(0);
    T p1b = T(0), p2b = T(0), v1xb = T(0), v1yb = T(0), v2xb = T(0), v2yb = T(0);
    T fb_loc[9];
    adj_collide_f(o, f, Yf, fb_loc, pstarb, uxb, uyb, Ftxb, Ftyb, rhob, taub);
    adj_collide_g(o, P.omega_phi, p1, o.v1x, o.v1y, Yg1, R.g1, p1b, uxb, uyb, v1xb, v1yb);
    adj_collide_g(o, P.omega_phi, p2, o.v2x, o.v2y, Yg2, R.g2, p2b, uxb, uyb, v2xb, v2yb);

    // ---------------- reverse: forces and velocity ----------------
    T jxb = uxb, jyb = uyb, ihrb = uxb * o.Ftx + uyb * o.Fty;
    Ftxb += uxb * ihr;
    Ftyb += uyb * ihr;
    T F0xb = Ftxb, F0yb = Ftyb, Fmuxb = Ftxb, Fmuyb = Ftyb;
    T Pxxb = -tau * grx * Fmuxb, Pxyb = -tau * gry * Fmuxb - tau * grx * Fmuyb, Pyyb = -tau * gry * Fmuyb;
    taub += -(Pxx * grx + Pxy * gry) * Fmuxb - (Pxy * grx + Pyy * gry) * Fmuyb;
    T grxb = -tau * (Pxx * Fmuxb + Pxy * Fmuyb), gryb = -tau * (Pxy * Fmuxb + Pyy * Fmuyb);
    T snub = C * Pxyb;
    T Cb = snu * Pxyb;
    T Bb = Pyyb, hob = Pyyb - Pxxb, Ab = Pxxb;
    snub += -T(0.5) * (A - B) * hob;
    Ab += T(0.5) * (T(1) - snu) * hob;
    Bb -= T(0.5) * (T(1) - snu) * hob;
    taub += -snu * snu * snub;
    T sxyb = Cb, u0xb = -u0y * Cb, u0yb = -u0x * Cb;
    T syyb = Bb;
    pstarb -= Bb * (T(1) / T(3));
    u0yb -= T(2) * u0y * Bb;
    T sxxb = Ab;
    pstarb -= Ab * (T(1) / T(3));
    u0xb -= T(2) * u0x * Ab;
    jxb += u0xb;
    jyb += u0yb;
    F0xb += u0xb * ihr;
    F0yb += u0yb * ihr;
    ihrb += u0xb * F0x + u0yb * F0y;
    rhob += -T(0.5) / (rho * rho) * ihrb;
    T Fsxb = F0xb, Fsyb = F0yb, Fmxb = F0xb, Fmyb = F0yb;
    T cpb = grx * F0xb + gry * F0yb;
    grxb += cp * F0xb;
    gryb += cp * F0yb;
    R.drive += F0xb;
    rhob += P.grav_x * F0xb + P.grav_y * F0yb;
    pstarb -= cpb * (T(1) / T(3));
    // moments of f
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    for (int a = 0; a < 9; ++a)
        R.f[a] = fb_loc[a] + pstarb + ex[a] * jxb + ey[a] * jyb + (ex[a] * ex[a]) * sxxb + (ey[a] * ey[a]) * syyb +
                 (ex[a] * ey[a]) * sxyb;
    // Kelvin force and field
    const T kelb = gcx * Fmxb + gcy * Fmyb;
    T gcxb = kel * Fmxb, gcyb = kel * Fmyb;
    const T Hxb = -T(2) * P.half_mu0 * Hx * kelb, Hyb = -T(2) * P.half_mu0 * Hy * kelb;
    R.H0x += Hxb;
    R.H0y += Hyb;
    R.gpx = -Hxb;
    R.gpy = -Hyb;
    // surface tension force
    const T m1b = g1x * Fsxb + g1y * Fsyb, m2b = g2x * Fsxb + g2y * Fsyb, m3b = g3x * Fsxb + g3y * Fsyb;
    T g1xb = m1 * Fsxb, g1yb = m1 * Fsyb, g2xb = m2 * Fsxb, g2yb = m2 * Fsyb, g3xb = m3 * Fsxb, g3yb = m3 * Fsyb;
    // chemical potentials
    T dH1b = T(0), dH2b = T(0), dH3b = T(0), l1b = T(0), l2b = T(0), l3b = T(0);
    R.cbulk += ((dH1 - dH2) * P.igam1 + (dH1 - dH3) * P.igam2) * m1b;
    dH1b += P.c_bulk * (P.igam1 + P.igam2) * m1b;
    dH2b -= P.c_bulk * P.igam1 * m1b;
    dH3b -= P.c_bulk * P.igam2 * m1b;
    R.igam1 += P.c_bulk * (dH1 - dH2) * m1b;
    R.igam2 += P.c_bulk * (dH1 - dH3) * m1b;
    R.gam0 -= P.c_lap * l1 * m1b;
    l1b -= P.c_lap * P.gam0 * m1b;
    R.cbulk += ((dH2 - dH1) * P.igam0 + (dH2 - dH3) * P.igam2) * m2b;
    dH2b += P.c_bulk * (P.igam0 + P.igam2) * m2b;
    dH1b -= P.c_bulk * P.igam0 * m2b;
    dH3b -= P.c_bulk * P.igam2 * m2b;
    R.igam0 += P.c_bulk * (dH2 - dH1) * m2b;
    R.igam2 += P.c_bulk * (dH2 - dH3) * m2b;
    R.gam1 -= P.c_lap * l2 * m2b;
    l2b -= P.c_lap * P.gam1 * m2b;
    R.cbulk += ((dH3 - dH1) * P.igam0 + (dH3 - dH2) * P.igam1) * m3b;
    dH3b += P.c_bulk * (P.igam0 + P.igam1) * m3b;
    dH1b -= P.c_bulk * P.igam0 * m3b;
    dH2b -= P.c_bulk * P.igam1 * m3b;
    R.igam0 += P.c_bulk * (dH3 - dH1) * m3b;
    R.igam1 += P.c_bulk * (dH3 - dH2) * m3b;
    R.gam2 -= P.c_lap * l3 * m3b;
    l3b -= P.c_lap * P.gam2 * m3b;
    // dH derivatives of Eq. 28
    T p3b = T(0), qb = T(0), p123b = T(0), e2b = T(0);
    // dH3 = 2 p3 (s13 p1^2 + s23 p2^2) + p1 p2 q + p123 gam2 + e2 p1 p2
    p3b += T(2) * (P.s13 * p1 * p1 + P.s23 * p2 * p2) * dH3b;
    R.s13 += T(2) * p3 * p1 * p1 * dH3b;
    R.s23 += T(2) * p3 * p2 * p2 * dH3b;
    p1b += T(4) * p3 * P.s13 * p1 * dH3b + p2 * q * dH3b + e2 * p2 * dH3b;
    p2b += T(4) * p3 * P.s23 * p2 * dH3b + p1 * q * dH3b + e2 * p1 * dH3b;
    qb += p1 * p2 * dH3b;
    p123b += P.gam2 * dH3b;
    R.gam2 += p123 * dH3b;
    e2b += p1 * p2 * dH3b;
    // dH2 = 2 p2 (s12 p1^2 + s23 p3^2) + p1 p3 q + p123 gam1 + e2 p1 p3
    p2b += T(2) * (P.s12 * p1 * p1 + P.s23 * p3 * p3) * dH2b;
    R.s12 += T(2) * p2 * p1 * p1 * dH2b;
    R.s23 += T(2) * p2 * p3 * p3 * dH2b;
    p1b += T(4) * p2 * P.s12 * p1 * dH2b + p3 * q * dH2b + e2 * p3 * dH2b;
    p3b += T(4) * p2 * P.s23 * p3 * dH2b + p1 * q * dH2b + e2 * p1 * dH2b;
    qb += p1 * p3 * dH2b;
    p123b += P.gam1 * dH2b;
    R.gam1 += p123 * dH2b;
    e2b += p1 * p3 * dH2b;
    // dH1 = 2 p1 (s12 p2^2 + s13 p3^2) + p2 p3 q + p123 gam0 + e2 p2 p3
    p1b += T(2) * (P.s12 * p2 * p2 + P.s13 * p3 * p3) * dH1b;
    R.s12 += T(2) * p1 * p2 * p2 * dH1b;
    R.s13 += T(2) * p1 * p3 * p3 * dH1b;
    p2b += T(4) * p1 * P.s12 * p2 * dH1b + p3 * q * dH1b + e2 * p3 * dH1b;
    p3b += T(4) * p1 * P.s13 * p3 * dH1b + p2 * q * dH1b + e2 * p2 * dH1b;
    qb += p2 * p3 * dH1b;
    p123b += P.gam0 * dH1b;
    R.gam0 += p123 * dH1b;
    e2b += p2 * p3 * dH1b;
    p123b += T(2) * P.eta * e2b;
    p1b += p2 * p3 * p123b;
    p2b += p1 * p3 * p123b;
    p3b += p1 * p2 * p123b;
    R.gam0 += p1 * qb;
    R.gam1 += p2 * qb;
    R.gam2 += p3 * qb;
    p1b += P.gam0 * qb;
    p2b += P.gam1 * qb;
    p3b += P.gam2 * qb;
    // grad chi (Eq. 9)
    const T Gxb = -iS2 * gcxb, Gyb = -iS2 * gcyb;
    const T iS2b = -Gx * gcxb - Gy * gcyb;
    const T Sb = -T(2) / (S * S * S) * iS2b;
    g1xb += P.ic0 * Gxb;
    g2xb += P.ic1 * Gxb;
    g3xb += P.ic2 * Gxb;
    g1yb += P.ic0 * Gyb;
    g2yb += P.ic1 * Gyb;
    g3yb += P.ic2 * Gyb;
    p1b += P.ic0 * Sb;
    p2b += P.ic1 * Sb;
    p3b += P.ic2 * Sb;
    // mixture
    g1xb += P.rho0 * grxb;
    g2xb += P.rho1 * grxb;
    g3xb += P.rho2 * grxb;
    g1yb += P.rho0 * gryb;
    g2yb += P.rho1 * gryb;
    g3yb += P.rho2 * gryb;
    p1b += P.tau0 * taub + P.rho0 * rhob;
    p2b += P.tau1 * taub + P.rho1 * rhob;
    p3b += P.tau2 * taub + P.rho2 * rhob;
    // counter-diffusion fluxes
    T sxb = -(v1xb + v2xb), syb = -(v1yb + v2yb);
    T r1b = g1x * v1xb + g1y * v1yb, r2b = g2x * v2xb + g2y * v2yb, r3b = T(0);
    g1xb += r1 * v1xb;
    g1yb += r1 * v1yb;
    g2xb += r2 * v2xb;
    g2yb += r2 * v2yb;
    sxb *= T(1) / T(3);
    syb *= T(1) / T(3);
    r1b += g1x * sxb + g1y * syb;
    r2b += g2x * sxb + g2y * syb;
    r3b += g3x * sxb + g3y * syb;
    g1xb += r1 * sxb;
    g1yb += r1 * syb;
    g2xb += r2 * sxb;
    g2yb += r2 * syb;
    g3xb += r3 * sxb;
    g3yb += r3 * syb;
    // r = t n, n = q^(-1/2), q = |g|^2 + eps^2, t = (4/xi) p (1 - p)
    const T q1b = -T(0.5) * n1 * n1 * n1 * (t1 * r1b), q2b = -T(0.5) * n2 * n2 * n2 * (t2 * r2b),
            q3b = -T(0.5) * n3 * n3 * n3 * (t3 * r3b);
    p1b += fx_ * (T(1) - T(2) * p1) * (n1 * r1b);
    p2b += fx_ * (T(1) - T(2) * p2) * (n2 * r2b);
    p3b += fx_ * (T(1) - T(2) * p3) * (n3 * r3b);
    g1xb += T(2) * g1x * q1b;
    g1yb += T(2) * g1y * q1b;
    g2xb += T(2) * g2x * q2b;
    g2yb += T(2) * g2y * q2b;
    g3xb += T(2) * g3x * q3b;
    g3yb += T(2) * g3y * q3b;
    // phase 3 by linearity
    g1xb -= g3xb;
    g2xb -= g3xb;
    g1yb -= g3yb;
    g2yb -= g3yb;
    l1b -= l3b;
    l2b -= l3b;
    p1b -= p3b;
    p2b -= p3b;
    R.p1 = p1b;
    R.gx1 = g1xb;
    R.gy1 = g1yb;
    R.l1 = l1b;
    R.p2 = p2b;
    R.gx2 = g2xb;
    R.gy2 = g2yb;
    R.l2 = l2b;
    return R;
}

// Forward of one node with all collisions, for checks: outputs f*, g1*, g2*.
template <typename T>
__host__ __device__ inline void node_forward(const StepConst<T>& P, const T f[9], const T g1[9], const T g2[9],
                                             const Nb9<T>& a1, const Nb9<T>& a2, const Nb9<T>& ps, T of[9], T og1[9],
                                             T og2[9]) {
    const NodeOut<T> o = node_physics(P, f, a1, a2, ps);
    collide_f(o, f, of);
    collide_g(o, P.omega_phi, o.phi1, o.v1x, o.v1y, g1, og1);
    collide_g(o, P.omega_phi, o.phi2, o.v2x, o.v2y, g2, og2);
}

}  // namespace fcd
