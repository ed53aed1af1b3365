// mrt_kernels.hip -- gfx950 kernels of the D2V16 MRT finite-difference LB step.
//
// One time step of the paper's scheme (Eq. 3, forward Euler in time,
// Lax-Wendroff in space, section "Construction"):
//   f_i(x)^{n+1} = f_i(x) - dt C_i(f(x)) + LW_i(f)(x)
//   C = Minv diag(s) (M f - fhat^eq(rho, j, e))        (Appendix for M, fhat^eq)
//   LW_i = sum_a w_down (f(x+e_a) - f(x)) + w_up (f(x-e_a) - f(x))
// is done by ONE fused kernel per step (step_kernel): each wave owns 64
// consecutive columns of a band of rows and marches up the band, keeping the
// rows y-1, y, y+1 of the 16 populations in registers; x neighbours come from
// the adjacent lanes by DPP wavefront shifts, the two halo columns by a load
// on lanes 0 and 63; the collision runs in registers in the factored
// moment space of mrt_transform.h.  Every population is read from HBM once
// and written once per step (SoA planes, 256-byte rows per wave, coalesced).
//
// Boundary ghosts (MRT_BC_*) are produced in the same pass: periodic sides
// load the wrapped row/column, EQ sides use precomputed equilibria, outflow
// sides copy the boundary cell, reflecting sides evaluate the equilibrium of
// the boundary cell's moments with the normal momentum reversed.
#include <hip/hip_runtime.h>

#include "mrt_dual.h"
#include "mrt_internal.h"

namespace mrt {

// ------------------------------------------------------------------ lanes

__device__ __forceinline__ int dpp_from_left(int v, int old) {    // lane l <- lane l-1
    return __builtin_amdgcn_update_dpp(old, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_right(int v, int old) {   // lane l <- lane l+1
    return __builtin_amdgcn_update_dpp(old, v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
// value of lane l-1; lane 0 keeps `old`
__device__ __forceinline__ float from_left(float v, float old) {
    return __builtin_bit_cast(float, dpp_from_left(__builtin_bit_cast(int, v), __builtin_bit_cast(int, old)));
}
__device__ __forceinline__ float from_right(float v, float old) {
    return __builtin_bit_cast(float, dpp_from_right(__builtin_bit_cast(int, v), __builtin_bit_cast(int, old)));
}
__device__ __forceinline__ double from_left(double v, double old) {
    int2 a = __builtin_bit_cast(int2, v), o = __builtin_bit_cast(int2, old);
    int2 r;
    r.x = dpp_from_left(a.x, o.x);
    r.y = dpp_from_left(a.y, o.y);
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double from_right(double v, double old) {
    int2 a = __builtin_bit_cast(int2, v), o = __builtin_bit_cast(int2, old);
    int2 r;
    r.x = dpp_from_right(a.x, o.x);
    r.y = dpp_from_right(a.y, o.y);
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// -------------------------------------------------------------- populations

constexpr bool moves_x(int i) { return i < 8 ? (i & 1) == 0 : true; }
constexpr bool moves_y(int i) { return i < 8 ? (i & 1) == 1 : true; }

// Conserved moments as compensated (Neumaier) FP32 sums over the 16
// populations: rho = sum f, j = sum v f, e = sum (v^2 + eta^2) f.
__device__ __forceinline__ void neumaier(float& s, float& c, float x) {
    const float t = s + x;
    c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}
__device__ __forceinline__ void conserved_compensated(const float f[16], float q[4]) {
    const float sp[4] = {1.0f, 6.0f, float(kR2), float(kR32)};
    const float eps[4] = {7.25f, 36.0f, 4.0f, 9.0f};
    float s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int k = i >> 2;
        neumaier(s[0], c[0], f[i]);
        if (sgn_x(i) != 0) neumaier(s[1], c[1], float(sgn_x(i)) * sp[k] * f[i]);
        if (sgn_y(i) != 0) neumaier(s[2], c[2], float(sgn_y(i)) * sp[k] * f[i]);
        neumaier(s[3], c[3], eps[k] * f[i]);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) q[m] = s[m] + c[m];
}

// dt * C for one cell in precision C (see collision_dt), converted to the
// storage type; COMP replaces the conserved moments by compensated FP32 sums.
template <typename C, bool COMP, typename S>
__device__ __forceinline__ void cell_collision(const S fs[16], C b, C binv, const double* sdt,
                                               S out[16], C& rho, C& P) {
    C f[16], m[16], eq[16], dm[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = C(fs[i]);
    pops_to_moments(f, m);
    if constexpr (COMP) {
        float q[4];
        conserved_compensated(fs, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) m[k] = q[k];
    }
    rho = m[0];
    P = equilibrium_moments(m[0], m[1], m[2], m[3], b, binv, eq);
    dm[0] = dm[1] = dm[2] = dm[3] = C(0);
#pragma unroll
    for (int k = 4; k < 16; ++k) dm[k] = C(sdt[k]) * (m[k] - eq[k]);
    moments_to_pops(dm, o);
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = S(o[i]);
}

template <typename S>
struct Weights;
template <>
struct Weights<float> {
    __device__ static float get(const Inst* P, int ax, int k, int j) { return P->lwf[ax][k][j]; }
};
template <>
struct Weights<double> {
    __device__ static double get(const Inst* P, int ax, int k, int j) { return P->lw[ax][k][j]; }
};

// ------------------------------------------------------------------ ghosts

// Fill the ghost ring of one instance (x = -1 and x = nx for 0 <= y < ny;
// y = -1 and y = ny for 0 <= x < nx) from the current populations:
// periodic -> the wrapped cell, MRT_BC_EQ -> the side's equilibrium,
// outflow -> the adjacent cell, reflecting -> the equilibrium of the
// adjacent cell with its normal velocity reversed.  Corners are never read.
template <typename S, typename C>
__global__ __launch_bounds__(256) void ghost_kernel(const Inst* __restrict__ insts,
                                                    S* __restrict__ f, int force_periodic) {
    const Inst* __restrict__ P = insts + blockIdx.y;
    const int nx = P->nx, ny = P->ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (nx + ny)) return;
    int side, gx, gy, ix, iy, px, py;
    if (t < ny) {
        side = XLO; gx = -1; gy = t; ix = 0; iy = t; px = nx - 1; py = t;
    } else if (t < 2 * ny) {
        side = XHI; gx = nx; gy = t - ny; ix = nx - 1; iy = gy; px = 0; py = gy;
    } else if (t < 2 * ny + nx) {
        side = YLO; gx = t - 2 * ny; gy = -1; ix = gx; iy = 0; px = gx; py = ny - 1;
    } else {
        side = YHI; gx = t - 2 * ny - nx; gy = ny; ix = gx; iy = ny - 1; px = gx; py = 0;
    }
    const int kind = force_periodic ? int(BC_PERIODIC) : P->bc[side];
    S* __restrict__ base = f + P->off + P->origin;
    const long long plane = P->plane;
    const long long go = (long long)gy * P->pitch + gx;
    S g[16];
    if (kind == BC_EQ) {
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = S(P->ghost[side][i]);
    } else {
        const bool per = kind == BC_PERIODIC;
        const long long so = (long long)(per ? py : iy) * P->pitch + (per ? px : ix);
        S c[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = base[i * plane + so];
        if (kind == BC_REFLECT) {
            C fc[16], m[16], eq[16], out[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) fc[i] = C(c[i]);
            pops_to_moments(fc, m);
            const bool nxs = side == XLO || side == XHI;
            equilibrium_moments(m[0], nxs ? -m[1] : m[1], nxs ? m[2] : -m[2], m[3], C(P->b),
                                C(P->binv), eq);
            moments_to_pops(eq, out);
#pragma unroll
            for (int i = 0; i < 16; ++i) g[i] = S(out[i]);
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) g[i] = c[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) base[i * plane + go] = g[i];
}

// ------------------------------------------------------------------- step

// Advance one work item: columns [x0, x0+64) of rows [y0, y1) of one
// instance.  The ghost ring holds every out-of-grid neighbour, so all
// neighbours are plain loads: rows y-1 / y+1 from the register window,
// columns x-1 / x+1 from the adjacent lanes (DPP wavefront shifts) and, on
// lanes 0 and 63, from one halo load.  Lanes past the last column load the
// ghost column / padding (in bounds: the pitch covers x0 + 64) and store
// nothing.
template <typename S, typename C, bool COMP>
__device__ __forceinline__ void step_item(const Inst* __restrict__ P, int x0, int y0, int y1,
                                          const S* __restrict__ fin, S* __restrict__ fout,
                                          unsigned* __restrict__ health) {
    const int lane = lane_id();
    const unsigned pitch = unsigned(P->pitch);
    const long long plane = P->plane;
    const S* __restrict__ fi = fin + P->off;
    S* __restrict__ fo = fout + P->off;
    const int x = x0 + lane;
    const bool act = x < P->nx;
    const C b = C(P->b), binv = C(P->binv);
    // uniform plane base + 32-bit lane offset (global_load with saddr)
    auto ld = [&](int i, unsigned off) -> S { return (fi + (long long)i * plane)[off]; };
    const unsigned hoff = (lane == 0) ? unsigned(-1) : 1u;   // halo column relative to x
    const bool hload = (lane == 0 || lane == 63);
    const unsigned o_start = unsigned(P->origin) + unsigned(y0) * pitch + unsigned(x);

    auto body = [&](const S (&rm)[16], const S (&r0)[16], const S (&rp)[16], S (&rn)[16],
                    int y, unsigned o) {
        if (y + 1 < y1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) rn[i] = ld(i, o + 2 * pitch);
        }
        S h[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) h[i] = S(0);
        if (hload) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) h[i] = ld(i, o + hoff);
        }
        S cdt[16];
        C rho, Pp;
        cell_collision<C, COMP>(r0, b, binv, P->sdt, cdt, rho, Pp);
        if (act && !(rho > C(0) && Pp > C(0))) atomicOr(health, 1u);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = i >> 2, sx = sgn_x(i), sy = sgn_y(i);
            // increment d = sum_a w_down (f(x+e_a) - f(x)) + w_up (f(x-e_a) - f(x)),
            // formed as w_down f(x+e) + w_up f(x-e) - c^2 f(x) (the terms
            // cancel to d; every rounding is c^2 times smaller than f)
            S d = S(0);
            if (sx != 0) {
                const S W = from_left(r0[i], h[i]);
                const S E = from_right(r0[i], h[i]);
                const S wd = Weights<S>::get(P, 0, k, 0), wu = Weights<S>::get(P, 0, k, 1);
                const S we = sx > 0 ? wd : wu, ww = sx > 0 ? wu : wd;
                d = we * E + (ww * W - (wd + wu) * r0[i]);
            }
            if (sy != 0) {
                const S wd = Weights<S>::get(P, 1, k, 0), wu = Weights<S>::get(P, 1, k, 1);
                const S wn = sy > 0 ? wd : wu, ws = sy > 0 ? wu : wd;
                d += wn * rp[i] + (ws * rm[i] - (wd + wu) * r0[i]);
            }
            const S out = r0[i] + (d - cdt[i]);
            if (act) (fo + (long long)i * plane)[o] = out;
        }
    };

    S A[16], B[16], Cw[16], D[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        B[i] = ld(i, o_start);
        Cw[i] = ld(i, o_start + pitch);
        A[i] = moves_y(i) ? ld(i, o_start - pitch) : S(0);
        D[i] = S(0);
    }
    // rows rotate through four register sets, so no copies between rows
    unsigned o = o_start;
    for (int y = y0; y < y1;) {
        body(A, B, Cw, D, y, o); ++y; o += pitch;
        if (y >= y1) break;
        body(B, Cw, D, A, y, o); ++y; o += pitch;
        if (y >= y1) break;
        body(Cw, D, A, B, y, o); ++y; o += pitch;
        if (y >= y1) break;
        body(D, A, B, Cw, y, o); ++y; o += pitch;
    }
}

template <typename S, typename C, bool COMP>
__global__ __launch_bounds__(256) void step_kernel(const Inst* __restrict__ insts,
                                                   const Item* __restrict__ items, int nitems,
                                                   const S* __restrict__ fin, S* __restrict__ fout,
                                                   unsigned* __restrict__ health) {
    const int wpb = blockDim.x >> 6;
    int w = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const int nw = gridDim.x * wpb;
    for (; w < nitems; w += nw) {
        const Item it = items[w];
        step_item<S, C, COMP>(insts + it.inst, it.x0, it.y0, it.y1, fin, fout, health);
    }
}

// ---------------------------------------------------------------- adjoint

// Adjoint of one step on a periodic grid (the ghost ring of lam^{n+1} holds
// the wrapped values), per cell x (lam = lam^{n+1}):
//   lam^n(x) = lam(x) + LW^T(lam)(x) - dt (dC/df(x))^T lam(x)
// with the collision part from cell_adjoint (mrt_dual.h).  Partial sums of
// the rate gradient per work item go to `partial` (16 doubles per item),
// reduced in a fixed order by reduce_partials.
template <typename S, typename C>
__device__ __forceinline__ void adjoint_item(const Inst* __restrict__ P, int item, int x0, int y0,
                                             int y1, const S* __restrict__ lin,
                                             const S* __restrict__ fn, S* __restrict__ lout,
                                             double* __restrict__ partial) {
    const int lane = lane_id();
    const unsigned pitch = unsigned(P->pitch);
    const long long plane = P->plane;
    const S* __restrict__ li = lin + P->off;
    const S* __restrict__ fi = fn + P->off;
    S* __restrict__ lo = lout + P->off;
    const int x = x0 + lane;
    const bool act = x < P->nx;
    const C b = C(P->b);
    const unsigned hoff = (lane == 0) ? unsigned(-1) : 1u;
    const bool hload = (lane == 0 || lane == 63);
    auto ldl = [&](int i, unsigned off) -> S { return (li + (long long)i * plane)[off]; };
    auto ldf = [&](int i, unsigned off) -> S { return (fi + (long long)i * plane)[off]; };
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    unsigned o = unsigned(P->origin) + unsigned(y0) * pitch + unsigned(x);
    for (int y = y0; y < y1; ++y, o += pitch) {
        S l0[16], lm[16], lp[16], fc[16], h[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            l0[i] = ldl(i, o);
            fc[i] = ldf(i, o);
            lm[i] = moves_y(i) ? ldl(i, o - pitch) : S(0);
            lp[i] = moves_y(i) ? ldl(i, o + pitch) : S(0);
            h[i] = S(0);
        }
        if (hload) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) h[i] = ldl(i, o + hoff);
        }
        C f[16], lam[16], coll[16], dsk[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            f[i] = C(fc[i]);
            lam[i] = C(l0[i]);
        }
        cell_adjoint(f, lam, b, P->sdt, C(P->dt), coll, dsk);
        if (act) {
#pragma unroll
            for (int k = 4; k < 16; ++k) acc[k] -= double(dsk[k]);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = i >> 2, sx = sgn_x(i), sy = sgn_y(i);
            S d = S(0);
            // transpose of the forward stencil: the weight that f(x+1) had in
            // F(x) now multiplies lam(x-1), and vice versa
            if (sx != 0) {
                const S W = from_left(l0[i], h[i]);
                const S E = from_right(l0[i], h[i]);
                const S wd = Weights<S>::get(P, 0, k, 0), wu = Weights<S>::get(P, 0, k, 1);
                const S e = E - l0[i], w = W - l0[i];
                d = sx > 0 ? (wd * w + wu * e) : (wu * w + wd * e);
            }
            if (sy != 0) {
                const S wd = Weights<S>::get(P, 1, k, 0), wu = Weights<S>::get(P, 1, k, 1);
                const S n = lp[i] - l0[i], s = lm[i] - l0[i];
                d += sy > 0 ? (wd * s + wu * n) : (wu * s + wd * n);
            }
            const S out = l0[i] + (d - S(coll[i]));
            if (act) (lo + (long long)i * plane)[o] = out;
        }
    }
    // wave reduction of the 12 non-trivial rate gradients
#pragma unroll
    for (int k = 4; k < 16; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[k] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) partial[(long long)item * 16 + k] = k < 4 ? 0.0 : acc[k];
    }
}

template <typename S, typename C>
__global__ __launch_bounds__(256) void adjoint_kernel(const Inst* __restrict__ insts,
                                                      const Item* __restrict__ items, int nitems,
                                                      const S* __restrict__ lin,
                                                      const S* __restrict__ fn,
                                                      S* __restrict__ lout,
                                                      double* __restrict__ partial) {
    const int wpb = blockDim.x >> 6;
    int w = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const int nw = gridDim.x * wpb;
    for (; w < nitems; w += nw) {
        const Item it = items[w];
        adjoint_item<S, C>(insts + it.inst, w, it.x0, it.y0, it.y1, lin, fn, lout, partial);
    }
}

// ds[k] += sum over items of partial[item][k], one block, fixed order.
__global__ __launch_bounds__(256) void reduce_partials(const double* __restrict__ partial,
                                                       int nitems, double* __restrict__ ds) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    for (int k = 0; k < 16; ++k) {
        double v = 0.0;
        for (int i = t; i < nitems; i += 256) v += partial[(long long)i * 16 + k];
        red[t] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (t < s) red[t] += red[t + s];
            __syncthreads();
        }
        if (t == 0) ds[k] += red[0];
        __syncthreads();
    }
}

// ------------------------------------------------------- per-cell kernels

__device__ __forceinline__ long long cell_offset(const Inst* __restrict__ P, long long c) {
    const int y = int(c / P->nx), x = int(c - (long long)y * P->nx);
    return P->off + P->origin + (long long)y * P->pitch + x;
}

// f = Minv fhat^eq(rho, u, T) from row-major FP64 fields.
template <typename S, typename C>
__global__ __launch_bounds__(256) void init_kernel(const Inst* __restrict__ P, const double* rho,
                                                   const double* ux, const double* uy,
                                                   const double* T, S* __restrict__ f) {
    const long long n = (long long)P->nx * P->ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        C g[16];
        equilibrium_pops(C(rho[c]), C(ux[c]), C(uy[c]), C(T[c]), C(P->b), g);
        S* base = f + cell_offset(P, c);
#pragma unroll
        for (int i = 0; i < 16; ++i) base[(long long)i * P->plane] = S(g[i]);
    }
}

// Macroscopic fields (FP64) and health of each cell.
template <typename S>
__global__ __launch_bounds__(256) void moments_kernel(const Inst* __restrict__ P,
                                                      const S* __restrict__ f, double* rho,
                                                      double* ux, double* uy, double* T,
                                                      unsigned* __restrict__ health) {
    const long long n = (long long)P->nx * P->ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const S* base = f + cell_offset(P, c);
        double g[16], m[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = double(base[(long long)i * P->plane]);
        pops_to_moments(g, m);
        const double r = m[0], u = m[1] / r, v = m[2] / r;
        const double t = (m[3] - r * (u * u + v * v)) / (P->b * r);
        if (rho) rho[c] = r;
        if (ux) ux[c] = u;
        if (uy) uy[c] = v;
        if (T) T[c] = t;
        if (!(r > 0.0 && t > 0.0)) atomicOr(health, 1u);
    }
}

// rho = sum_i f_i (FP64 output) and its adjoint lam_i = g.
template <typename S>
__global__ __launch_bounds__(256) void density_kernel(const Inst* __restrict__ P,
                                                      const S* __restrict__ f, double* rho) {
    const long long n = (long long)P->nx * P->ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const S* base = f + cell_offset(P, c);
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) s += double(base[(long long)i * P->plane]);
        rho[c] = s;
    }
}
template <typename S>
__global__ __launch_bounds__(256) void density_adjoint_kernel(const Inst* __restrict__ P,
                                                              const double* g,
                                                              S* __restrict__ lam) {
    const long long n = (long long)P->nx * P->ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        S* base = lam + cell_offset(P, c);
        const S v = S(g[c]);
#pragma unroll
        for (int i = 0; i < 16; ++i) base[(long long)i * P->plane] = v;
    }
}

// g_q = sum_i lam0_i d f^0_i / d q for q in (rho, ux, uy, T).
template <typename S, typename C>
__global__ __launch_bounds__(256) void init_adjoint_kernel(
    const Inst* __restrict__ P, const S* __restrict__ lam, const double* rho, const double* ux,
    const double* uy, const double* T, double* g_rho, double* g_ux, double* g_uy, double* g_T) {
    const long long n = (long long)P->nx * P->ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        Dual4<C> f[16];
        equilibrium_pops(Dual4<C>::var(C(rho[c]), 0), Dual4<C>::var(C(ux[c]), 1),
                         Dual4<C>::var(C(uy[c]), 2), Dual4<C>::var(C(T[c]), 3),
                         Dual4<C>(P->b), f);
        const S* base = lam + cell_offset(P, c);
        C g[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const C l = C(base[(long long)i * P->plane]);
#pragma unroll
            for (int j = 0; j < 4; ++j) g[j] += l * f[i].d[j];
        }
        if (g_rho) g_rho[c] = double(g[0]);
        if (g_ux) g_ux[c] = double(g[1]);
        if (g_uy) g_uy[c] = double(g[2]);
        if (g_T) g_T[c] = double(g[3]);
    }
}

// Padded storage <-> unpadded FP64 copies of the populations.
template <typename S>
__global__ __launch_bounds__(256) void export_kernel(const Inst* __restrict__ P,
                                                     const S* __restrict__ f, double* out) {
    const long long nc = (long long)P->nx * P->ny;
    const long long n = 16 * nc;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const long long i = c / nc;
        out[c] = double(f[cell_offset(P, c - i * nc) + i * P->plane]);
    }
}
template <typename S>
__global__ __launch_bounds__(256) void import_kernel(const Inst* __restrict__ P, const double* in,
                                                     S* __restrict__ f) {
    const long long nc = (long long)P->nx * P->ny;
    const long long n = 16 * nc;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const long long i = c / nc;
        f[cell_offset(P, c - i * nc) + i * P->plane] = S(in[c]);
    }
}

// -------------------------------------------------------- launch wrappers

template <typename S, typename C, bool COMP>
hipError_t launch_step(const Inst* insts, const Item* items, int nitems, const void* fin,
                       void* fout, unsigned* health, int grid, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int blocks = grid > 0 ? grid : (nitems + 3) / 4;
    hipLaunchKernelGGL((step_kernel<S, C, COMP>), dim3(blocks), dim3(256), 0, st, insts, items,
                       nitems, static_cast<const S*>(fin), static_cast<S*>(fout), health);
    return hipGetLastError();
}

}  // namespace mrt

// Entry points used by the host library (mrt_api.hip); precision codes as in
// mrtlb.h.
namespace mrt {

static int grid_for(long long n) {
    long long g = (n + 255) / 256;
    return int(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

// Ghost ring of `count` instances (instance table `insts`, longest
// perimeter 2 * (nx + ny) = perim) in buffer f.
hipError_t k_ghost(int prec, const Inst* insts, int count, int perim, void* f, bool force_periodic,
                   hipStream_t st) {
    const dim3 grid((perim + 255) / 256, count);
    switch (prec) {
        case 0: hipLaunchKernelGGL((ghost_kernel<double, double>), grid, dim3(256), 0, st, insts, static_cast<double*>(f), int(force_periodic)); break;
        case 1: hipLaunchKernelGGL((ghost_kernel<float, float>), grid, dim3(256), 0, st, insts, static_cast<float*>(f), int(force_periodic)); break;
        default: hipLaunchKernelGGL((ghost_kernel<float, double>), grid, dim3(256), 0, st, insts, static_cast<float*>(f), int(force_periodic)); break;
    }
    return hipGetLastError();
}

hipError_t k_step(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                  void* fout, unsigned* health, int grid, hipStream_t st) {
    switch (prec) {
        case 0: return launch_step<double, double, false>(insts, items, nitems, fin, fout, health, grid, st);
        case 1: return launch_step<float, float, true>(insts, items, nitems, fin, fout, health, grid, st);
        default: return launch_step<float, double, false>(insts, items, nitems, fin, fout, health, grid, st);
    }
}

hipError_t k_adjoint(int prec, const Inst* insts, const Item* items, int nitems, const void* lin,
                     const void* fn, void* lout, double* partial, double* ds, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int blocks = (nitems + 3) / 4;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL((adjoint_kernel<double, double>), dim3(blocks), dim3(256), 0, st,
                               insts, items, nitems, static_cast<const double*>(lin),
                               static_cast<const double*>(fn), static_cast<double*>(lout), partial);
            break;
        case 1:
            hipLaunchKernelGGL((adjoint_kernel<float, float>), dim3(blocks), dim3(256), 0, st,
                               insts, items, nitems, static_cast<const float*>(lin),
                               static_cast<const float*>(fn), static_cast<float*>(lout), partial);
            break;
        default:
            hipLaunchKernelGGL((adjoint_kernel<float, double>), dim3(blocks), dim3(256), 0, st,
                               insts, items, nitems, static_cast<const float*>(lin),
                               static_cast<const float*>(fn), static_cast<float*>(lout), partial);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, st, partial, nitems, ds);
    return hipGetLastError();
}

hipError_t k_init(int prec, const Inst* P, long long cells, const double* rho, const double* ux,
                  const double* uy, const double* T, void* f, hipStream_t st) {
    const int g = grid_for(cells);
    switch (prec) {
        case 0: hipLaunchKernelGGL((init_kernel<double, double>), dim3(g), dim3(256), 0, st, P, rho, ux, uy, T, static_cast<double*>(f)); break;
        case 1: hipLaunchKernelGGL((init_kernel<float, float>), dim3(g), dim3(256), 0, st, P, rho, ux, uy, T, static_cast<float*>(f)); break;
        default: hipLaunchKernelGGL((init_kernel<float, double>), dim3(g), dim3(256), 0, st, P, rho, ux, uy, T, static_cast<float*>(f)); break;
    }
    return hipGetLastError();
}

hipError_t k_moments(int prec, const Inst* P, long long cells, const void* f, double* rho,
                     double* ux, double* uy, double* T, unsigned* health, hipStream_t st) {
    const int g = grid_for(cells);
    if (prec == 0)
        hipLaunchKernelGGL((moments_kernel<double>), dim3(g), dim3(256), 0, st, P, static_cast<const double*>(f), rho, ux, uy, T, health);
    else
        hipLaunchKernelGGL((moments_kernel<float>), dim3(g), dim3(256), 0, st, P, static_cast<const float*>(f), rho, ux, uy, T, health);
    return hipGetLastError();
}

hipError_t k_density(int prec, const Inst* P, long long cells, const void* f, double* rho,
                     hipStream_t st) {
    const int g = grid_for(cells);
    if (prec == 0)
        hipLaunchKernelGGL((density_kernel<double>), dim3(g), dim3(256), 0, st, P, static_cast<const double*>(f), rho);
    else
        hipLaunchKernelGGL((density_kernel<float>), dim3(g), dim3(256), 0, st, P, static_cast<const float*>(f), rho);
    return hipGetLastError();
}

hipError_t k_density_adjoint(int prec, const Inst* P, long long cells, const double* g_rho,
                             void* lam, hipStream_t st) {
    const int g = grid_for(cells);
    if (prec == 0)
        hipLaunchKernelGGL((density_adjoint_kernel<double>), dim3(g), dim3(256), 0, st, P, g_rho, static_cast<double*>(lam));
    else
        hipLaunchKernelGGL((density_adjoint_kernel<float>), dim3(g), dim3(256), 0, st, P, g_rho, static_cast<float*>(lam));
    return hipGetLastError();
}

hipError_t k_init_adjoint(int prec, const Inst* P, long long cells, const void* lam,
                          const double* rho, const double* ux, const double* uy, const double* T,
                          double* g_rho, double* g_ux, double* g_uy, double* g_T, hipStream_t st) {
    const int g = grid_for(cells);
    switch (prec) {
        case 0: hipLaunchKernelGGL((init_adjoint_kernel<double, double>), dim3(g), dim3(256), 0, st, P, static_cast<const double*>(lam), rho, ux, uy, T, g_rho, g_ux, g_uy, g_T); break;
        case 1: hipLaunchKernelGGL((init_adjoint_kernel<float, float>), dim3(g), dim3(256), 0, st, P, static_cast<const float*>(lam), rho, ux, uy, T, g_rho, g_ux, g_uy, g_T); break;
        default: hipLaunchKernelGGL((init_adjoint_kernel<float, double>), dim3(g), dim3(256), 0, st, P, static_cast<const float*>(lam), rho, ux, uy, T, g_rho, g_ux, g_uy, g_T); break;
    }
    return hipGetLastError();
}

hipError_t k_export(int prec, const Inst* P, long long cells, const void* f, double* out,
                    hipStream_t st) {
    const int g = grid_for(16 * cells);
    if (prec == 0)
        hipLaunchKernelGGL((export_kernel<double>), dim3(g), dim3(256), 0, st, P, static_cast<const double*>(f), out);
    else
        hipLaunchKernelGGL((export_kernel<float>), dim3(g), dim3(256), 0, st, P, static_cast<const float*>(f), out);
    return hipGetLastError();
}

hipError_t k_import(int prec, const Inst* P, long long cells, const double* in, void* f,
                    hipStream_t st) {
    const int g = grid_for(16 * cells);
    if (prec == 0)
        hipLaunchKernelGGL((import_kernel<double>), dim3(g), dim3(256), 0, st, P, in, static_cast<double*>(f));
    else
        hipLaunchKernelGGL((import_kernel<float>), dim3(g), dim3(256), 0, st, P, in, static_cast<float*>(f));
    return hipGetLastError();
}

}  // namespace mrt
