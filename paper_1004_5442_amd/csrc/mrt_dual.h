// mrt_dual.h -- forward-mode dual numbers with four tangent directions.
//
// The adjoint kernels need d fhat^eq / d(rho, jx, jy, e) (collision Jacobian)
// and d f^eq / d(rho, ux, uy, T) (initialisation).  Evaluating the same
// templated equilibrium code on Dual4 gives those derivatives exactly (to
// rounding), so no derivative of the Appendix formulas is written by hand.
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

// Collision part of the adjoint of one step at one cell (lam = lam^{n+1}):
//   coll = dt (dC/df)^T lam = M^T zeta,   zeta_k = s_k dt (Minv^T lam)_k  (k >= 5),
//          zeta_{1..4} = -sum_{k>=5} zeta_k d fhat^eq_k / d(rho, jx, jy, e)
//   dsk[k] = dt (fhat_k - fhat^eq_k)(Minv^T lam)_k: minus the cell's share of
//            dL/ds_k (dF/ds_k = -dt Minv[:,k](fhat_k - fhat^eq_k), Eq. 3).
// sdt[k] = s_{k+1} dt.
template <typename C>
MRT_HD void cell_adjoint(const C f[16], const C lam[16], C b, const double* sdt, C dt,
                         C coll[16], C dsk[16]) {
    C m[16], mu[16];
    pops_to_moments(f, m);
    inverse_T(lam, mu);
    Dual4<C> q[4], eqd[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = Dual4<C>::var(m[k], k);
    equilibrium_moments(q[0], q[1], q[2], q[3], Dual4<C>(double(b)), Dual4<C>(1.0 / double(b)), eqd);
    C zeta[16];
    C g[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
    for (int k = 0; k < 4; ++k) dsk[k] = C(0);
#pragma unroll
    for (int k = 4; k < 16; ++k) {
        const C zk = C(sdt[k]) * mu[k];
        zeta[k] = zk;
#pragma unroll
        for (int j = 0; j < 4; ++j) g[j] += zk * eqd[k].d[j];
        dsk[k] = dt * (m[k] - eqd[k].v) * mu[k];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) zeta[j] = -g[j];
    moments_T(zeta, coll);
}

}  // namespace mrt
