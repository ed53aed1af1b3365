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

// Products fused into FMAs only within one expression, as written (for the
// FP32-only compensated sums and the FP32 transforms below).
#define MRT_CONTRACT_IN_EXPRESSIONS _Pragma("clang fp contract(on)")

namespace mrt {

constexpr double kR2 = 1.41421356237309504880;      // sqrt(2): x speed on shell 3
constexpr double kR32 = 2.12132034355964257320;     // 3/sqrt(2): x speed on shell 4

// x-component magnitude of each shell (1, 6, sqrt 2, 3/sqrt 2)
MRT_HD double shell_speed(int k) {
    return k == 0 ? 1.0 : k == 1 ? 6.0 : k == 2 ? kR2 : kR32;
}

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

// The transforms, the equilibrium and the collision are compiled twice:
//  * fused:  the compiler may fuse a product with an addition into an FMA
//    across statements (the default), which it does for the FP64 collision;
//  * inexpr: only within one expression, as written.  The fusion of every
//    formula is then the same in every inlined copy, so the FP32 collision
//    gives bit-identical results in each unrolled row of the marching kernels
//    (with cross-statement fusion the compiler fused differently per row, and
//    two steps per pass differed from two single steps in the last bits).
// The FP32 instantiations use inexpr; every other type (double, the dual
// numbers of the adjoint) uses fused, whose FP64 code it keeps 3 % shorter.
namespace fused {
#include "mrt_transform_impl.inc"
}  // namespace fused
namespace inexpr {
#pragma clang fp contract(on)
#include "mrt_transform_impl.inc"
#pragma clang fp contract(fast)
}  // namespace inexpr

#define MRT_DISPATCH(name, params, args)                                  \
    template <typename C>                                                 \
    MRT_HD auto name params {                                             \
        if constexpr (std::is_same<C, float>::value) return inexpr::name##_impl args; \
        else return fused::name##_impl args;                                     \
    }
MRT_DISPATCH(pops_to_moments, (const C f[16], C m[16]), (f, m))
MRT_DISPATCH(moments_to_pops, (const C m[16], C f[16]), (m, f))
MRT_DISPATCH(moments_T, (const C z[16], C g[16]), (z, g))
MRT_DISPATCH(inverse_T, (const C l[16], C z[16]), (l, z))
MRT_DISPATCH(equilibrium_moments, (C rho, C jx, C jy, C e, C b, C binv, C eq[16]),
             (rho, jx, jy, e, b, binv, eq))
MRT_DISPATCH(equilibrium_pops, (C rho, C ux, C uy, C T, C b, C f[16]), (rho, ux, uy, T, b, f))
MRT_DISPATCH(collision_dt, (const C f[16], C b, const C sdt[16], C out[16], C& rho, C& P),
             (f, b, sdt, out, rho, P))
#undef MRT_DISPATCH

// ---------------------------------------------- compensated FP32 moments
// The conserved moments rho = sum f, j = sum v f, e = sum (|v|^2 + eta^2) f
// (rows m1..m4 of M) of FP32 populations as compensated FP32 sums, for the
// all-FP32 form.  The sums follow the butterfly of pops_to_moments (shell
// sums, signed x and y sums, then the four shells combined), and every
// addition and product on that path is an error-free transformation: the
// rounded result plus its exact rounding error (Knuth's branch-free TwoSum;
// the product's error from one FMA).  The errors are added up in plain FP32
// and added to the rounded sum once, so the result is within one unit in the
// last place of the exact sum of the FP32 terms (the velocity and eta^2
// constants as FP32 values), and in nearly every case the correctly rounded
// value.  Following the butterfly shares its rounded sums with the moment
// transform and costs about 260 instructions per cell (one TwoSum per
// addend into four running sums took about 430).

// a + b = s + e exactly (round to nearest, no overflow), any magnitudes.
MRT_HD float two_sum(float a, float b, float& e) {
    MRT_CONTRACT_IN_EXPRESSIONS
    const float s = a + b;
    const float bp = s - a;
    const float ap = s - bp;
    e = (a - ap) + (b - bp);
    return s;
}
// a * b = p + e exactly (no overflow or underflow).
MRT_HD float two_prod(float a, float b, float& e) {
    MRT_CONTRACT_IN_EXPRESSIONS
    const float p = a * b;
    e = __builtin_fmaf(a, b, -p);
    return p;
}

MRT_HD void conserved_compensated(const float f[16], float q[4]) {
    MRT_CONTRACT_IN_EXPRESSIONS
    float sg[4], esg[4], X[4], eX[4], Y[4], eY[4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {           // axis shells: (+x, +y, -x, -y)
        const float a0 = f[4 * k], a1 = f[4 * k + 1], a2 = f[4 * k + 2], a3 = f[4 * k + 3];
        float e1, e2, e3;
        const float px = two_sum(a0, a2, e1), py = two_sum(a1, a3, e2);
        sg[k] = two_sum(px, py, e3);
        esg[k] = (e1 + e2) + e3;
        X[k] = two_sum(a0, -a2, eX[k]);
        Y[k] = two_sum(a1, -a3, eY[k]);
    }
#pragma unroll
    for (int k = 2; k < 4; ++k) {           // diagonal shells: (++, -+, --, +-)
        const float d0 = f[4 * k], d1 = f[4 * k + 1], d2 = f[4 * k + 2], d3 = f[4 * k + 3];
        float e1, e2, e3, e4, e5, e6, e7;
        const float p02 = two_sum(d0, d2, e1), p13 = two_sum(d1, d3, e2);
        sg[k] = two_sum(p02, p13, e3);
        esg[k] = (e1 + e2) + e3;
        const float m02 = two_sum(d0, -d2, e4), m31 = two_sum(d3, -d1, e5);
        X[k] = two_sum(m02, m31, e6);
        eX[k] = (e4 + e5) + e6;
        Y[k] = two_sum(m02, -m31, e7);
        eY[k] = (e4 - e5) + e7;
    }
    {   // rho = sum of the shell sums
        float r1, r2, r3;
        const float a = two_sum(sg[0], sg[1], r1), b = two_sum(sg[2], sg[3], r2);
        const float s = two_sum(a, b, r3);
        q[0] = s + (((esg[0] + esg[1]) + (esg[2] + esg[3])) + ((r1 + r2) + r3));
    }
    // j = X_1 + 6 X_2 + sqrt 2 X_3 + (3 / sqrt 2) X_4 (and Y): the x speeds of the shells
    const float sp1 = 6.0f, sp2 = float(kR2), sp3 = float(kR32);
    const float* odd[2] = {X, Y};
    const float* eodd[2] = {eX, eY};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const float* v = odd[a];
        const float* ev = eodd[a];
        float p1, p2, p3, r1, r2, r3;
        const float t1 = two_prod(sp1, v[1], p1), t2 = two_prod(sp2, v[2], p2),
                    t3 = two_prod(sp3, v[3], p3);
        const float u = two_sum(v[0], t1, r1), w = two_sum(t2, t3, r2);
        const float s = two_sum(u, w, r3);
        q[1 + a] = s + (((ev[0] + sp1 * ev[1]) + (sp2 * ev[2] + sp3 * ev[3])) + ((p1 + p2) + p3)
                        + ((r1 + r2) + r3));
    }
    {   // e = 7.25 sg_1 + 36 sg_2 + 4 sg_3 + 9 sg_4  (|v|^2 + eta^2 per shell)
        float p0, p1, p3, r1, r2, r3;
        const float t0 = two_prod(7.25f, sg[0], p0), t1 = two_prod(36.0f, sg[1], p1);
        const float t2 = 4.0f * sg[2];      // exact
        const float t3 = two_prod(9.0f, sg[3], p3);
        const float u = two_sum(t0, t1, r1), w = two_sum(t2, t3, r2);
        const float s = two_sum(u, w, r3);
        q[3] = s + (((7.25f * esg[0] + 36.0f * esg[1]) + (4.0f * esg[2] + 9.0f * esg[3]))
                    + ((p0 + p1) + p3) + ((r1 + r2) + r3));
    }
}

}  // namespace mrt
