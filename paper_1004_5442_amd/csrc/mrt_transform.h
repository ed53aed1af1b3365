// mrt_transform.h -- moment transform of the D2V16 MRT scheme in factored form.
//
// The paper's transformation matrix M (Appendix, rows m_1..m_16) is built from
// monomials of the velocity, and the 16 velocities form four shells of four
// related by 90-degree rotations (section "Construction", velocity display).
// Both facts let M factor as M = B * T:
//   T  per-shell butterfly: (f0..f3) -> (sigma, X, Y, Q) = shell sum, signed x
//      sum, signed y sum and the signed quadrupole sum (x^2 - y^2 on the axis
//      shells, xy on the diagonal shells);
//   B  block diagonal: the scalar moments (m1, m4, m5, m14) mix only the four
//      sigma's, the x-odd moments (m2, m8, m10, m12) only the X's, the y-odd
//      ones (m3, m9, m11, m13) only the Y's, (m6, m16) the axis-shell Q's and
//      (m7, m15) the diagonal-shell Q's.
// so M f costs 24 adds plus ~50 multiply-adds instead of 176, and
// Minv = Tinv * Binv likewise.  The block inverses below are exact rationals
// (times sqrt 2 in the X/Y blocks) obtained by symbolic inversion; they hold
// for eta = 5/2 on shell 1, the value the paper fixes.
//
// Velocity order: shell 1 (speed 1) and shell 2 (speed 6): (+x, +y, -x, -y);
// shell 3 (sqrt 2 (+-1, +-1)) and shell 4 ((3/sqrt 2)(+-1, +-1)): (++, -+, --, +-).
// Moment m[k-1] is the paper's fhat_k.
//
// Everything here is __host__ __device__ so the host library evaluates boundary
// equilibria with exactly the code the kernels run.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#define MRT_HD __host__ __device__ __forceinline__

namespace mrt {

constexpr double kR2 = 1.41421356237309504880;      // sqrt(2): x speed on shell 3
constexpr double kR32 = 2.12132034355964257320;     // 3/sqrt(2): x speed on shell 4

// x-component magnitude of each shell (1, 6, sqrt 2, 3/sqrt 2)
MRT_HD double shell_speed(int k) {
    return k == 0 ? 1.0 : k == 1 ? 6.0 : k == 2 ? kR2 : kR32;
}

// f (16) -> m (16): m = M f.
template <typename C>
MRT_HD void pops_to_moments(const C f[16], C m[16]) {
    C sg[4], X[4], Y[4], Q[4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {           // axis shells: (+x, +y, -x, -y)
        const C a0 = f[4 * k], a1 = f[4 * k + 1], a2 = f[4 * k + 2], a3 = f[4 * k + 3];
        const C px = a0 + a2, py = a1 + a3;
        sg[k] = px + py;
        Q[k] = px - py;
        X[k] = a0 - a2;
        Y[k] = a1 - a3;
    }
#pragma unroll
    for (int k = 2; k < 4; ++k) {           // diagonal shells: (++, -+, --, +-)
        const C d0 = f[4 * k], d1 = f[4 * k + 1], d2 = f[4 * k + 2], d3 = f[4 * k + 3];
        const C p02 = d0 + d2, p13 = d1 + d3, m02 = d0 - d2, m31 = d3 - d1;
        sg[k] = p02 + p13;
        Q[k] = p02 - p13;
        X[k] = m02 + m31;
        Y[k] = m02 - m31;
    }
    const C R2 = C(kR2), R32 = C(kR32);
    // scalar block
    m[0] = (sg[0] + sg[1]) + (sg[2] + sg[3]);
    const C t5 = C(36) * sg[1] + C(4) * sg[2] + C(9) * sg[3];
    m[4] = sg[0] + t5;
    m[3] = C(7.25) * sg[0] + t5;
    m[13] = C(7.25) * sg[0] + C(1296) * sg[1] + C(16) * sg[2] + C(81) * sg[3];
    // x-odd block
    const C x3 = C(216) * X[1] + C(4) * R2 * X[2] + C(9) * R32 * X[3];
    m[1] = X[0] + C(6) * X[1] + R2 * X[2] + R32 * X[3];
    m[7] = C(7.25) * X[0] + x3;
    m[9] = X[0] + x3;
    m[11] = X[0] + C(216) * X[1];
    // y-odd block
    const C y3 = C(216) * Y[1] + C(4) * R2 * Y[2] + C(9) * R32 * Y[3];
    m[2] = Y[0] + C(6) * Y[1] + R2 * Y[2] + R32 * Y[3];
    m[8] = C(7.25) * Y[0] + y3;
    m[10] = Y[0] + y3;
    m[12] = -(Y[0] + C(216) * Y[1]);
    // quadrupole blocks
    m[5] = Q[0] + C(36) * Q[1];
    m[15] = C(7.25) * Q[0] + C(1296) * Q[1];
    m[6] = C(2) * Q[2] + C(4.5) * Q[3];
    m[14] = C(8) * Q[2] + C(40.5) * Q[3];
}

// m (16) -> f (16): f = Minv m.
template <typename C>
MRT_HD void moments_to_pops(const C m[16], C f[16]) {
    // Binv, then the inverse butterfly.  The butterfly's factors (1/4 on the
    // shell sums and quadrupole sums, 1/2 on the axis shells' signed sums,
    // 1/4 on the diagonal shells' signed sums) are carried in the Binv
    // constants: scaling by a power of two is exact, so the result is the
    // same as applying them after the sums.
    const C R2q = C(0.25 * kR2);
    C sg[4], X[4], Y[4], Q[4];
    sg[0] = C(0.25 * 0.16) * (m[3] - m[4]);
    sg[1] = m[0] * C(0.25 / 24.0) - C(0.25 * (121.0 / 21600.0)) * m[3]
          - C(0.25 * (17.0 / 1800.0)) * m[4] + C(0.25 / 864.0) * m[13];
    sg[2] = C(0.25 * (81.0 / 40.0)) * m[0] - C(0.25 * (229.0 / 800.0)) * m[3]
          + C(0.25 / 200.0) * m[4] + C(0.25 / 160.0) * m[13];
    sg[3] = C(0.25 * (-16.0 / 15.0)) * m[0] + C(0.25 * (89.0 / 675.0)) * m[3]
          + C(0.25 * (37.0 / 225.0)) * m[4] - C(0.25 / 135.0) * m[13];
    const C xa[4] = {m[1], m[7], m[9], m[11]};
    const C ya[4] = {m[2], m[8], m[10], -m[12]};
    const C* src[2] = {xa, ya};
    C* dst[2] = {X, Y};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const C* s = src[a];
        C* d = dst[a];
        d[0] = C(0.5 * 0.16) * (s[1] - s[2]);
        d[1] = (s[2] - s[1]) * C(0.5 / 1350.0) + s[3] * C(0.5 / 216.0);
        d[2] = R2q * (C(0.9) * s[0] - C(0.14) * s[1] + C(0.04) * s[2] + C(0.075) * s[3]);
        d[3] = R2q * (C(-4.0 / 15.0) * s[0] + C(28.0 / 675.0) * s[1] + C(17.0 / 675.0) * s[2]
                      - C(8.0 / 135.0) * s[3]);
    }
    Q[0] = C(0.25 * (144.0 / 115.0)) * m[5] - C(0.25 * (4.0 / 115.0)) * m[15];
    Q[1] = C(0.25 * (-29.0 / 4140.0)) * m[5] + C(0.25 / 1035.0) * m[15];
    Q[2] = C(0.25 * 0.9) * m[6] - C(0.25 * 0.1) * m[14];
    Q[3] = C(0.25 * (-8.0 / 45.0)) * m[6] + C(0.25 * (2.0 / 45.0)) * m[14];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const C sp = sg[k] + Q[k], sm = sg[k] - Q[k];
        f[4 * k] = sp + X[k];
        f[4 * k + 1] = sm + Y[k];
        f[4 * k + 2] = sp - X[k];
        f[4 * k + 3] = sm - Y[k];
    }
#pragma unroll
    for (int k = 2; k < 4; ++k) {
        const C sq = sg[k] + Q[k], dq = sg[k] - Q[k];
        const C xy = X[k] + Y[k], yx = Y[k] - X[k];
        f[4 * k] = sq + xy;
        f[4 * k + 1] = dq + yx;
        f[4 * k + 2] = sq - xy;
        f[4 * k + 3] = dq - yx;
    }
}

template <typename C>
MRT_HD void moments_T(const C z[16], C g[16]) {
    const C R2 = C(kR2), R32 = C(kR32);
    C sg[4], X[4], Y[4], Q[4];
    // columns of the scalar block (1, eps_k, |v_k|^2, |v_k|^2 eps_k)
    sg[0] = z[0] + C(7.25) * z[3] + z[4] + C(7.25) * z[13];
    sg[1] = z[0] + C(36) * z[3] + C(36) * z[4] + C(1296) * z[13];
    sg[2] = z[0] + C(4) * z[3] + C(4) * z[4] + C(16) * z[13];
    sg[3] = z[0] + C(9) * z[3] + C(9) * z[4] + C(81) * z[13];
    // columns of the x-odd block (rows m2, m8, m10, m12)
    X[0] = z[1] + C(7.25) * z[7] + z[9] + z[11];
    X[1] = C(6) * z[1] + C(216) * (z[7] + z[9] + z[11]);
    X[2] = R2 * (z[1] + C(4) * (z[7] + z[9]));
    X[3] = R32 * (z[1] + C(9) * (z[7] + z[9]));
    // y-odd block (rows m3, m9, m11, m13 with m13 = -(Y0 + 216 Y1))
    Y[0] = z[2] + C(7.25) * z[8] + z[10] - z[12];
    Y[1] = C(6) * z[2] + C(216) * (z[8] + z[10] - z[12]);
    Y[2] = R2 * (z[2] + C(4) * (z[8] + z[10]));
    Y[3] = R32 * (z[2] + C(9) * (z[8] + z[10]));
    // quadrupole blocks
    Q[0] = z[5] + C(7.25) * z[15];
    Q[1] = C(36) * z[5] + C(1296) * z[15];
    Q[2] = C(2) * z[6] + C(8) * z[14];
    Q[3] = C(4.5) * z[6] + C(40.5) * z[14];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        g[4 * k] = sg[k] + X[k] + Q[k];
        g[4 * k + 1] = sg[k] + Y[k] - Q[k];
        g[4 * k + 2] = sg[k] - X[k] + Q[k];
        g[4 * k + 3] = sg[k] - Y[k] - Q[k];
    }
#pragma unroll
    for (int k = 2; k < 4; ++k) {
        const C sq = sg[k] + Q[k], dq = sg[k] - Q[k];
        const C xy = X[k] + Y[k], yx = Y[k] - X[k];
        g[4 * k] = sq + xy;
        g[4 * k + 1] = dq + yx;
        g[4 * k + 2] = sq - xy;
        g[4 * k + 3] = dq - yx;
    }
}

// l (population space, 16) -> Minv^T l (moment space, 16): the transposed
// butterfly inverse followed by the transposed block inverses.
template <typename C>
MRT_HD void inverse_T(const C l[16], C z[16]) {
    const C R2 = C(kR2);
    C sg[4], X[4], Y[4], Q[4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const C a0 = l[4 * k], a1 = l[4 * k + 1], a2 = l[4 * k + 2], a3 = l[4 * k + 3];
        sg[k] = C(0.25) * ((a0 + a2) + (a1 + a3));
        Q[k] = C(0.25) * ((a0 + a2) - (a1 + a3));
        X[k] = C(0.5) * (a0 - a2);
        Y[k] = C(0.5) * (a1 - a3);
    }
#pragma unroll
    for (int k = 2; k < 4; ++k) {
        const C d0 = l[4 * k], d1 = l[4 * k + 1], d2 = l[4 * k + 2], d3 = l[4 * k + 3];
        const C p02 = d0 + d2, p13 = d1 + d3, m02 = d0 - d2, m31 = d3 - d1;
        sg[k] = C(0.25) * (p02 + p13);
        Q[k] = C(0.25) * (p02 - p13);
        X[k] = C(0.25) * (m02 + m31);
        Y[k] = C(0.25) * (m02 - m31);
    }
    z[0] = sg[1] * C(1.0 / 24.0) + C(81.0 / 40.0) * sg[2] - C(16.0 / 15.0) * sg[3];
    z[3] = C(0.16) * sg[0] - C(121.0 / 21600.0) * sg[1] - C(229.0 / 800.0) * sg[2]
         + C(89.0 / 675.0) * sg[3];
    z[4] = C(-0.16) * sg[0] - C(17.0 / 1800.0) * sg[1] + C(1.0 / 200.0) * sg[2]
         + C(37.0 / 225.0) * sg[3];
    z[13] = sg[1] * C(1.0 / 864.0) + sg[2] * C(1.0 / 160.0) - sg[3] * C(1.0 / 135.0);
    const C* src[2] = {X, Y};
    const int r0[2] = {1, 2}, r1[2] = {7, 8}, r2[2] = {9, 10}, r3[2] = {11, 12};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const C* s = src[a];
        const C last = s[1] * C(1.0 / 216.0) + R2 * (C(0.075) * s[2] - C(8.0 / 135.0) * s[3]);
        z[r0[a]] = R2 * (C(0.9) * s[2] - C(4.0 / 15.0) * s[3]);
        z[r1[a]] = C(0.16) * s[0] - s[1] * C(1.0 / 1350.0)
                 + R2 * (C(-0.14) * s[2] + C(28.0 / 675.0) * s[3]);
        z[r2[a]] = C(-0.16) * s[0] + s[1] * C(1.0 / 1350.0)
                 + R2 * (C(0.04) * s[2] + C(17.0 / 675.0) * s[3]);
        z[r3[a]] = a == 0 ? last : -last;
    }
    z[5] = C(144.0 / 115.0) * Q[0] - C(29.0 / 4140.0) * Q[1];
    z[15] = C(-4.0 / 115.0) * Q[0] + Q[1] * C(1.0 / 1035.0);
    z[6] = C(0.9) * Q[2] - C(8.0 / 45.0) * Q[3];
    z[14] = C(-0.1) * Q[2] + C(2.0 / 45.0) * Q[3];
}

// Equilibrium kinetic moments fhat^eq_5..16 (Appendix) from the conserved
// moments, R = 1: P = (e - j^2/rho)/b; written with u = j/rho:
//   5: 2P + rho u^2          6: rho(ux^2 - uy^2)        7: rho ux uy
//   8,9: (e + 2P) u          10,11: (4P + rho u^2) u
//   12: (2P + rho(ux^2-uy^2)) ux     13: (-2P + rho(ux^2-uy^2)) uy
//   14: 2(b+2) P^2/rho + (6+b) P u^2 + rho u^4
//   15: ((b+4)P + rho u^2) ux uy     16: ((b+4)P + rho u^2)(ux^2 - uy^2)
// Entries 0..3 are set to the conserved moments themselves.  binv = 1/b.
// Returns P.
// 1/x.  FP64 on the device: the hardware reciprocal refined by two Newton
// steps r <- r + r (1 - x r) (within an ulp of the rounded quotient, half
// the instructions of the IEEE division sequence); other types divide.
template <typename C>
MRT_HD C recip(C x) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (std::is_same<C, double>::value) {
        double r = __builtin_amdgcn_rcp(x);
        r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
        r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
        return r;
    }
#endif
    return C(1) / x;
}

template <typename C>
MRT_HD C equilibrium_moments(C rho, C jx, C jy, C e, C b, C binv, C eq[16]) {
    const C ri = recip(rho);
    const C ux = jx * ri, uy = jy * ri;
    const C u2 = ux * ux + uy * uy;
    const C rhou2 = rho * u2;
    const C P = (e - rhou2) * binv;
    const C d = ux * ux - uy * uy;
    const C rd = rho * d;
    const C q = (b + C(4)) * P + rhou2;
    eq[0] = rho;
    eq[1] = jx;
    eq[2] = jy;
    eq[3] = e;
    eq[4] = C(2) * P + rhou2;
    eq[5] = rd;
    eq[6] = rho * ux * uy;
    eq[7] = (e + C(2) * P) * ux;
    eq[8] = (e + C(2) * P) * uy;
    eq[9] = (C(4) * P + rhou2) * ux;
    eq[10] = (C(4) * P + rhou2) * uy;
    eq[11] = (C(2) * P + rd) * ux;
    eq[12] = (C(-2) * P + rd) * uy;
    eq[13] = C(2) * (b + C(2)) * P * P * ri + (C(6) + b) * P * u2 + rhou2 * u2;
    eq[14] = q * ux * uy;
    eq[15] = q * d;
    return P;
}

// f^eq = Minv fhat^eq of a primitive state (rho, ux, uy, T), R = 1.
template <typename C>
MRT_HD void equilibrium_pops(C rho, C ux, C uy, C T, C b, C f[16]) {
    const C jx = rho * ux, jy = rho * uy;
    const C e = b * rho * T + rho * (ux * ux + uy * uy);
    C m[16];
    equilibrium_moments(rho, jx, jy, e, b, C(1) / b, m);
    moments_to_pops(m, f);
}

// dt * C with C = Minv diag(s) (M f - fhat^eq) (Eq. 3); sdt[k] = s_{k+1} dt.
// The conserved rows (k < 4) are zero by construction.  Also returns rho and
// P for the health check.
template <typename C>
MRT_HD void collision_dt(const C f[16], C b, const C sdt[16], C out[16], C& rho, C& P) {
    C m[16], eq[16], dm[16];
    pops_to_moments(f, m);
    rho = m[0];
    P = equilibrium_moments(m[0], m[1], m[2], m[3], b, C(1) / b, eq);
    dm[0] = dm[1] = dm[2] = dm[3] = C(0);
#pragma unroll
    for (int k = 4; k < 16; ++k) dm[k] = sdt[k] * (m[k] - eq[k]);
    moments_to_pops(dm, out);
}

}  // namespace mrt
