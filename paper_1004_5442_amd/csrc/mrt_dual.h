// mrt_dual.h -- forward-mode dual numbers with four tangent directions.
//
// The adjoint of the initialisation needs d f^eq / d(rho, ux, uy, T):
// evaluating the templated equilibrium code on Dual4 gives those derivatives
// exactly (to rounding).  The step adjoint needs only a vector-Jacobian
// product of the equilibrium moments, done in reverse order below.
#pragma once

#include "mrt_transform.h"

namespace mrt {

template <typename C>
struct Dual4 {
    C v, d[4];
    MRT_HD Dual4() : v(0), d{0, 0, 0, 0} {}
    MRT_HD Dual4(double x) : v(C(x)), d{0, 0, 0, 0} {}
    MRT_HD static Dual4 var(C x, int k) {
        Dual4 r(0.0);
        r.v = x;
        r.d[k] = C(1);
        return r;
    }
};

template <typename C>
MRT_HD Dual4<C> operator+(const Dual4<C>& a, const Dual4<C>& b) {
    Dual4<C> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <typename C>
MRT_HD Dual4<C> operator-(const Dual4<C>& a, const Dual4<C>& b) {
    Dual4<C> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <typename C>
MRT_HD Dual4<C> operator-(const Dual4<C>& a) {
    Dual4<C> r;
    r.v = -a.v;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = -a.d[k];
    return r;
}
template <typename C>
MRT_HD Dual4<C> operator*(const Dual4<C>& a, const Dual4<C>& b) {
    Dual4<C> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <typename C>
MRT_HD Dual4<C> operator/(const Dual4<C>& a, const Dual4<C>& b) {
    Dual4<C> r;
    const C inv = C(1) / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
    return r;
}

}  // namespace mrt

namespace mrt {

// Vector-Jacobian product of the equilibrium moments (equilibrium_moments,
// Appendix, R = 1) with respect to the conserved moments q = (rho, jx, jy, e):
//   g_j = sum_{k >= 4} z_k d fhat^eq_k / d q_j          (j = 0..3)
// evaluated in reverse order through the intermediates of the forward
// formulas (ri = 1/rho, u = j ri, u2, rho u2, P = (e - rho u2)/b, d = ux^2 -
// uy^2, rho d, q = (b + 4) P + rho u2): every line below is the adjoint of one
// forward assignment.  (A forward-mode evaluation over the four tangent
// directions, Dual4, holds five values per intermediate in registers; this
// holds one.)  The host tests compare it with the oracle's complex-step
// Jacobian.
template <typename C>
MRT_HD void equilibrium_vjp(C rho, C jx, C jy, C e, C b, C binv, const C z[16], C g[4]) {
    // forward intermediates
    const C ri = recip(rho);
    const C ux = jx * ri, uy = jy * ri;
    const C u2 = ux * ux + uy * uy;
    const C rhou2 = rho * u2;
    const C P = (e - rhou2) * binv;
    const C d = ux * ux - uy * uy;
    const C rd = rho * d;
    const C q = (b + C(4)) * P + rhou2;
    // adjoints of the intermediates, accumulated from fhat^eq_5..16
    C aP = C(2) * z[4], ar = z[4], aux = C(0), auy = C(0), ard = z[5], aq = C(0), ad = C(0);
    C arho = z[6] * ux * uy, ae = C(0), au2 = C(0), ari = C(0);
    aux += z[6] * rho * uy;
    auy += z[6] * rho * ux;
    const C A = e + C(2) * P;                 // fhat^eq_8,9 = A u
    ae += z[7] * ux + z[8] * uy;
    aP += C(2) * (z[7] * ux + z[8] * uy);
    aux += z[7] * A;
    auy += z[8] * A;
    const C B4 = C(4) * P + rhou2;            // fhat^eq_10,11 = B4 u
    aP += C(4) * (z[9] * ux + z[10] * uy);
    ar += z[9] * ux + z[10] * uy;
    aux += z[9] * B4;
    auy += z[10] * B4;
    aP += C(2) * (z[11] * ux - z[12] * uy);   // fhat^eq_12 = (2P + rd) ux, 13 = (-2P + rd) uy
    ard += z[11] * ux + z[12] * uy;
    aux += z[11] * (C(2) * P + rd);
    auy += z[12] * (rd - C(2) * P);
    // fhat^eq_14 = 2 (b + 2) P^2 ri + (6 + b) P u2 + rhou2 u2
    aP += z[13] * (C(4) * (b + C(2)) * P * ri + (C(6) + b) * u2);
    ari += z[13] * C(2) * (b + C(2)) * P * P;
    au2 += z[13] * ((C(6) + b) * P + rhou2);
    ar += z[13] * u2;
    aq += z[14] * ux * uy + z[15] * d;        // fhat^eq_15 = q ux uy, 16 = q d
    aux += z[14] * q * uy;
    auy += z[14] * q * ux;
    ad += z[15] * q;
    // q = (b + 4) P + rhou2
    aP += (b + C(4)) * aq;
    ar += aq;
    // rd = rho d
    arho += ard * d;
    ad += ard * rho;
    // d = ux^2 - uy^2
    aux += C(2) * ux * ad;
    auy -= C(2) * uy * ad;
    // P = (e - rhou2) binv
    ae += binv * aP;
    ar -= binv * aP;
    // rhou2 = rho u2
    arho += u2 * ar;
    au2 += rho * ar;
    // u2 = ux^2 + uy^2
    aux += C(2) * ux * au2;
    auy += C(2) * uy * au2;
    // ux = jx ri, uy = jy ri
    g[1] = ri * aux;
    g[2] = ri * auy;
    ari += jx * aux + jy * auy;
    // ri = 1/rho
    arho -= ri * ri * ari;
    g[0] = arho;
    g[3] = ae;
}

// Collision part of the adjoint of one step at one cell (lam = lam^{n+1}):
//   coll = dt (dC/df)^T lam = M^T zeta,   zeta_k = s_k dt (Minv^T lam)_k  (k >= 5),
//          zeta_{1..4} = -sum_{k>=5} zeta_k d fhat^eq_k / d(rho, jx, jy, e)
//   dsk[k] = dt (fhat_k - fhat^eq_k)(Minv^T lam)_k: minus the cell's share of
//            dL/ds_k (dF/ds_k = -dt Minv[:,k](fhat_k - fhat^eq_k), Eq. 3).
// sdt[k] = s_{k+1} dt.
template <typename C, typename DP>
MRT_HD void cell_adjoint(const C f[16], const C lam[16], C b, C binv, DP sdt, C dt,
                         C coll[16], C dsk[16]) {
    C m[16], mu[16], eq[16], zeta[16], g[4];
    pops_to_moments(f, m);
    inverse_T(lam, mu);
    equilibrium_moments(m[0], m[1], m[2], m[3], b, binv, eq);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dsk[k] = C(0);
        zeta[k] = C(0);
    }
#pragma unroll
    for (int k = 4; k < 16; ++k) {
        zeta[k] = C(sdt[k]) * mu[k];
        dsk[k] = dt * (m[k] - eq[k]) * mu[k];
    }
    equilibrium_vjp(m[0], m[1], m[2], m[3], b, binv, zeta, g);
#pragma unroll
    for (int j = 0; j < 4; ++j) zeta[j] = -g[j];
    moments_T(zeta, coll);
}

}  // namespace mrt
