// fcd_potential.hpp -- per-node evaluation of the potential operator on one level
// (shared by the single-channel and batched solvers).  See fcd_potential.hip for the
// discretisation and the wall rule.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "fcd_device.hpp"

namespace fcd {

template <typename T>
struct MgEval {
    T C;      // sum of the coefficients
    T acc;    // sum c_a u(x+e_a), ghost rows by the kappa rule
    T cself;  // kappa * c of the ghost that mirrors this node itself (edge rows)
    T rhs;    // right-hand side
};

// The operator at node row j from its mu and u neighbourhoods (rows beyond the walls
// clamped to the edge rows, as nb_index gives them); fval is the right-hand side when
// the level has an f plane.  This function, sor_value and residual_abs fix every fused
// multiply-add themselves (contraction off), so each kernel that uses them rounds the
// same way whatever code surrounds it, and the batch's fused sweeps, per-colour sweeps
// and residual passes agree bit for bit.
template <typename T>
__device__ __forceinline__ MgEval<T> mg_eval_nb(const PotLevel<T>& L, const Nb9<T>& m, Nb9<T> u, int j, T fval) {
#pragma clang fp contract(off)
    const T k = L.kappa, kt = L.kappa_top;
    if (j == 0) {
        u.s = -k * u.s;
        u.sw = -k * u.sw;
        u.se = -k * u.se;
    }
    if (j == L.ny - 1) {
        u.n = -kt * u.n;
        u.ne = -kt * u.ne;
        u.nw = -kt * u.nw;
    }
    const T a = L.inv_h2 * (T(1) / T(3)), d = L.inv_h2 * (T(1) / T(12));
    const T ce = a * (m.c + m.e), cw = a * (m.c + m.w), cn = a * (m.c + m.n), cs = a * (m.c + m.s);
    const T cne = d * (m.c + m.ne), cnw = d * (m.c + m.nw), csw = d * (m.c + m.sw), cse = d * (m.c + m.se);
    MgEval<T> r;
    r.C = ((ce + cw) + (cn + cs)) + ((cne + csw) + (cnw + cse));
    r.acc = (fma(ce, u.e, cw * u.w) + fma(cn, u.n, cs * u.s)) + (fma(cne, u.ne, csw * u.sw) + fma(cnw, u.nw, cse * u.se));
    r.cself = (j == 0 ? k * cs : T(0)) + (j == L.ny - 1 ? kt * cn : T(0));
    if (L.f) {
        r.rhs = fval;
    } else {
        const T sx = (ce - cw) + (cne - csw) + (cse - cnw);
        const T sy = (cn - cs) + (cne - csw) + (cnw - cse);
        r.rhs = fma(L.H0x, sx, L.H0y * sy);
    }
    return r;
}

template <typename T>
__device__ __forceinline__ MgEval<T> mg_eval(const PotLevel<T>& L, int i, int j) {
    const NbIdx x = nb_index(i, j, L.nx, L.ny, L.pitch);
    const Nb9<T> m = load_nb(L.mu, x);
    const Nb9<T> u = load_nb(static_cast<const T*>(L.u), x);  // rows clamped to the edge rows
    return mg_eval_nb(L, m, u, j, L.f ? L.f[x.c] : T(0));
}

// Gauss-Seidel / SOR value of a node: u + omega (u_GS - u), with the node's own ghost
// image taken implicitly.
template <typename T>
__device__ __forceinline__ T sor_value(const MgEval<T>& r, T old, T omega) {
#pragma clang fp contract(off)
    const T gs = (fma(r.cself, old, r.acc) - r.rhs) / (r.C + r.cself);
    return fma(omega, gs - old, old);
}

// |acc - C u - rhs|: the magnitude of the node's residual, in double.
template <typename T>
__device__ __forceinline__ double residual_abs(const MgEval<T>& r, T u) {
#pragma clang fp contract(off)
    return fabs((double)(fma(-r.C, u, r.acc) - r.rhs));
}

// One node of one colour of a Gauss-Seidel / SOR sweep.
template <typename T>
__device__ __forceinline__ void relax_node(const PotLevel<T>& L, int i, int j, T omega) {
    const MgEval<T> r = mg_eval(L, i, j);
    const long long k = (long long)j * L.pitch + i;
    L.u[k] = sor_value(r, L.u[k], omega);
}

__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

}  // namespace fcd
