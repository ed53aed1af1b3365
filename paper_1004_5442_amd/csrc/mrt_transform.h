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

}  // namespace mrt
