// mrt_kernels.hip -- gfx950 kernels of the D2V16 MRT finite-difference LB step.
//
// One time step of the paper's scheme (Eq. 3, forward Euler in time,
// Lax-Wendroff in space, section "Construction"):
//   f_i(x)^{n+1} = f_i(x) - dt C_i(f(x)) + LW_i(f)(x)
//   C = Minv diag(s) (M f - fhat^eq(rho, j, e))        (Appendix for M, fhat^eq)
//   LW_i = sum_a w_down (f(x+e_a) - f(x)) + w_up (f(x-e_a) - f(x))
// is done by ONE fused kernel per step (step_kernel), or per two steps
// (step2_kernel, FP32 storage: f^{n+1} stays in registers; see "two steps"
// below): a block of four waves
// owns 256 consecutive columns of a band of rows and marches up the band,
// keeping the rows y-1, y, y+1 of the 16 populations in registers; x
// neighbours come from the adjacent lanes by DPP wavefront shifts and from
// the neighbouring waves through LDS, the two halo columns of the block by a
// load on one lane each; the collision runs in registers in the factored
// moment space of mrt_transform.h.  Every population is read from HBM once
// (plus the halo rows of each band) and written once per step (256-byte
// sub-row segments per wave, coalesced; the 16 population sub-rows of a grid
// row are contiguous).
//
// Boundaries (MRT_BC_*): periodic and outflow sides are read through an index
// remap (the wrapped or the adjacent row/column), fixed-equilibrium sides
// from a ghost ring written once per buffer, reflecting sides from a ghost
// ring that ghost_kernel rewrites before each step (the equilibrium of the
// adjacent cell's moments with the normal momentum reversed).
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

// The x neighbours that lanes 0 and 63 take from outside their wave are the
// values the DPP shifts keep in the lane that has no source lane; the
// marching kernels assign them in those two lanes only.  In every other lane
// their value does not matter (the shift overwrites it there).  An empty asm
// statement declares the registers written, so they are defined without an
// instruction: zero-filling them cost 12 vector instructions per cell (the
// two-step kernel measured 0.45 % slower with it).
template <typename S>
__device__ __forceinline__ void no_value(S (&h)[16]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) asm volatile("" : "=v"(h[i]));
}

// -------------------------------------------------------------- populations

constexpr bool moves_x(int i) { return i < 8 ? (i & 1) == 0 : true; }
constexpr bool moves_y(int i) { return i < 8 ? (i & 1) == 1 : true; }

// dt * C for one cell in precision C (see collision_dt), converted to the
// storage type; COMP replaces the conserved moments by compensated FP32 sums
// (conserved_compensated, mrt_transform.h).
template <typename C, bool COMP, typename S, typename DP>
__device__ __forceinline__ void cell_collision(const S fs[16], C b, C binv, DP sdt,
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
    template <typename IP>
    __device__ static float get(IP P, int ax, int k, int j) { return P->lwf[ax][k][j]; }
    template <typename IP>
    __device__ static float sum(IP P, int ax, int k) { return P->lwsf[ax][k]; }
    __device__ static float cross(const Inst* P, int k) { return P->lwcf[k]; }
};
template <>
struct Weights<double> {
    template <typename IP>
    __device__ static double get(IP P, int ax, int k, int j) { return P->lw[ax][k][j]; }
    template <typename IP>
    __device__ static double sum(IP P, int ax, int k) { return P->lws[ax][k]; }
    __device__ static double cross(const Inst* P, int k) { return P->lwc[k]; }
};

// New value of population i of a site: f + LW_i(f) - dt C_i, with the
// neighbour values W / E (x - 1 / x + 1; used if population i moves in x)
// and So / N (y - 1 / y + 1; used if it moves in y).  Per axis the
// Lax-Wendroff increment sum_a w_down (f(x+e_a) - f(x)) + w_up (f(x-e_a) - f(x))
// is w_down f(x+e) + w_up f(x-e) - c^2 f(x) (c^2 = w_down + w_up, summed on
// the host in the precision of S).  The whole increment, from -dt C_i, is
// accumulated in one chain of FMAs, so that every rounding is at the
// magnitude of the increment, and f is added once at the end.
template <typename S>
__device__ __forceinline__ S fma_s(S a, S b, S c) {
    if constexpr (sizeof(S) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}
template <typename S, typename IP>
__device__ __forceinline__ S lw_increment(IP P, int i, S f, S W, S E, S So, S N, S cdt) {
    const int k = i >> 2, sx = sgn_x(i), sy = sgn_y(i);
    S d = -cdt;
    if (sx != 0) {
        const S wd = Weights<S>::get(P, 0, k, 0), wu = Weights<S>::get(P, 0, k, 1);
        const S we = sx > 0 ? wd : wu, ww = sx > 0 ? wu : wd;
        d = fma_s(-Weights<S>::sum(P, 0, k), f, d);
        d = fma_s(ww, W, d);
        d = fma_s(we, E, d);
    }
    if (sy != 0) {
        const S wd = Weights<S>::get(P, 1, k, 0), wu = Weights<S>::get(P, 1, k, 1);
        const S wn = sy > 0 ? wd : wu, ws = sy > 0 ? wu : wd;
        d = fma_s(-Weights<S>::sum(P, 1, k), f, d);
        d = fma_s(ws, So, d);
        d = fma_s(wn, N, d);
    }
    return d;
}
template <typename S, typename IP>
__device__ __forceinline__ S site_update(IP P, int i, S f, S W, S E, S So, S N, S cdt) {
    return f + lw_increment(P, i, f, W, E, So, N, cdt);
}

// ------------------------------------------------------------------ ghosts

// Ghost cells that are not read through the index remap of Inst: the
// equilibria of MRT_BC_EQ sides (written once per buffer, `mode` bit 1) and
// the reflected equilibria of MRT_BC_REFLECT sides (the adjacent cell with
// its normal velocity reversed, `mode` bit 0: for a state set from outside a
// step, and before each step of the per-cell variant kernels; the step
// kernel writes those of its own output).  Ghosts x = -1 / x = nx for 0 <= y < ny, y = -1 / y = ny for
// 0 <= x < nx, and the four corners, which only the nine-point stencil
// reads: a corner is the y side's rule applied to the x-side ghost next to
// it (x sides first, then y sides over the full width), written where both
// its sides keep ghosts in the ring (EQ or REFLECT); otherwise the index
// remap reaches it through an interior row or column.
// The reflecting-wall ghost of a cell: f^eq of its moments with the
// velocity component along `axis` (0: x, 1: y) reversed (section (d)).
template <typename C, typename S>
__device__ __forceinline__ void reflected_eq(const S in[16], int axis, C b, C binv, S out[16]) {
    C f[16], m[16], eq[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = C(in[i]);
    pops_to_moments(f, m);
    equilibrium_moments(m[0], axis == 0 ? -m[1] : m[1], axis == 0 ? m[2] : -m[2], m[3], b, binv, eq);
    moments_to_pops(eq, o);
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = S(o[i]);
}

// Corner c (0: (-1, -1), 1: (nx, -1), 2: (-1, ny), 3: (nx, ny)) of the
// ghost ring (see ghost_kernel).
template <typename S, typename C>
__device__ void ghost_corner(const Inst* __restrict__ P, S* __restrict__ f, int c, int mode) {
    const int nx = P->nx, ny = P->ny;
    const int xside = (c & 1) ? XHI : XLO, yside = c < 2 ? YLO : YHI;
    const int xkind = P->bc[xside], ykind = P->bc[yside];
    if (!(xkind == BC_EQ || xkind == BC_REFLECT)) return;
    const bool do_eq = ykind == BC_EQ && (mode & 2);
    const bool do_ref = ykind == BC_REFLECT && (mode & 1);
    if (!do_eq && !do_ref) return;
    const int gx = (c & 1) ? nx : -1, gy = c < 2 ? -1 : ny;
    const int ix = (c & 1) ? nx - 1 : 0, iy = c < 2 ? 0 : ny - 1;
    S* __restrict__ base = f + P->off + P->origin;
    const long long plane = P->plane;
    S g[16];
    if (do_eq) {
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = S(P->ghost[yside][i]);
    } else {
        // the x-side ghost next to the corner, then its y reflection
        C xg[16], m[16], eq[16], out[16];
        if (xkind == BC_EQ) {
#pragma unroll
            for (int i = 0; i < 16; ++i) xg[i] = C(P->ghost[xside][i]);
        } else {
            const long long so = (long long)iy * P->pitch + ix;
#pragma unroll
            for (int i = 0; i < 16; ++i) xg[i] = C(base[i * plane + so]);
            pops_to_moments(xg, m);
            equilibrium_moments(m[0], -m[1], m[2], m[3], C(P->b), C(P->binv), eq);
            moments_to_pops(eq, xg);
        }
        pops_to_moments(xg, m);
        equilibrium_moments(m[0], m[1], -m[2], m[3], C(P->b), C(P->binv), eq);
        moments_to_pops(eq, out);
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = S(out[i]);
    }
    const long long go = (long long)gy * P->pitch + gx;
#pragma unroll
    for (int i = 0; i < 16; ++i) base[i * plane + go] = g[i];
}

template <typename S, typename C>
__global__ __launch_bounds__(256) void ghost_kernel(const Inst* __restrict__ insts,
                                                    S* __restrict__ f, int mode) {
    const Inst* __restrict__ P = insts + blockIdx.y;
    const int nx = P->nx, ny = P->ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (nx + ny) + 4) return;
    if (t >= 2 * (nx + ny)) {
        ghost_corner<S, C>(P, f, t - 2 * (nx + ny), mode);
        return;
    }
    int side, gx, gy, ix, iy;
    if (t < ny) {
        side = XLO; gx = -1; gy = t; ix = 0; iy = t;
    } else if (t < 2 * ny) {
        side = XHI; gx = nx; gy = t - ny; ix = nx - 1; iy = gy;
    } else if (t < 2 * ny + nx) {
        side = YLO; gx = t - 2 * ny; gy = -1; ix = gx; iy = 0;
    } else {
        side = YHI; gx = t - 2 * ny - nx; gy = ny; ix = gx; iy = ny - 1;
    }
    const int kind = P->bc[side];
    const bool do_eq = kind == BC_EQ && (mode & 2);
    const bool do_ref = kind == BC_REFLECT && (mode & 1);
    if (!do_eq && !do_ref) return;
    S* __restrict__ base = f + P->off + P->origin;
    const long long plane = P->plane;
    const long long go = (long long)gy * P->pitch + gx;
    S g[16];
    if (do_eq) {
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = S(P->ghost[side][i]);
    } else {
        const long long so = (long long)iy * P->pitch + ix;
        S fc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) fc[i] = base[i * plane + so];
        reflected_eq<C>(fc, (side == XLO || side == XHI) ? 0 : 1, C(P->b), C(P->binv), g);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) base[i * plane + go] = g[i];
}

// offset in a plane of row y, -1 <= y <= ny, with the boundary remap
// (unsigned arithmetic: r = -1 wraps to origin - pitch; the library keeps
// every instance below 2^32 elements, so the offset itself never wraps)
template <typename IP>
__device__ __forceinline__ unsigned row_offset(IP P, int y) {
    const int r = y < 0 ? P->row_lo : (y >= P->ny ? P->row_hi : y);
    return unsigned(P->origin) + unsigned(r) * unsigned(P->pitch);
}

// ------------------------------------------------------------------- step

// One work item is a block of 4 waves covering 256 columns [x0, x0 + 256)
// of rows [y0, y1) of one instance (the sub-row length is a multiple of 256,
// so the block never leaves its sub-rows).  Lane l of wave w owns column
// x0 + 64 w + l and the block marches up the band together:
//  * rows y-1 / y+1 come from a register window (four register sets rotate,
//    no copies), row y+2 is prefetched while row y is computed;
//  * columns x-1 / x+1 come from the adjacent lanes by DPP wavefront shifts;
//    the edge lanes of the four waves swap their values through LDS (double
//    buffered, one barrier per row) and only lanes 0 of wave 0 and 63 of
//    wave 3 load a halo column from memory;
//  * out-of-grid neighbours come through the boundary remap of Inst (the
//    wrapped or adjacent cell, or the ghost ring), so there is no boundary
//    code; lanes past the last column compute on those values and store
//    into column nx + 1, which is never read.
constexpr int kWaves = 4;

template <typename S>
struct EdgeBuf {
    // [slot][wave][0: lane 0, 1: lane 63][x-moving population]
    S v[2][kWaves][2][12];
};

// index of an x-moving population among the 12 (0, 2, 4, 6, 8..15)
constexpr int xslot(int i) { return i < 8 ? i >> 1 : i - 4; }

template <typename S, typename C, bool COMP, bool NT, bool WALLS>
__device__ __forceinline__ void step_block(const Inst* __restrict__ P, int x0, int y0, int y1,
                                           const S* __restrict__ fin, S* __restrict__ fout,
                                           unsigned* __restrict__ health, EdgeBuf<S>& lds) {
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long plane = P->plane;
    const S* __restrict__ fi = fin + P->off;
    S* __restrict__ fo = fout + P->off;
    const int nx = P->nx;
    const int x = x0 + 64 * wv + lane;
    const bool act = x < nx;
    // per-lane load column (lanes past the grid read the x >= nx neighbour)
    // and store column (lanes past the grid write the unread column nx + 1)
    const unsigned cx = unsigned(act ? x : P->col_hi);
    const unsigned xs = unsigned(act ? x : nx + 1);
    const C b = C(P->b), binv = C(P->binv);
    // uniform row offset + per-lane column, summed in 32 bits (the ghost
    // column is col = -1: row + col is then row - 1 >= 63; row >= 64)
    auto ld = [&](int i, unsigned row, unsigned col) -> S {
        return (fi + (long long)i * plane)[row + col];
    };
    // the two lanes that load a halo column from memory
    const bool hmem = (wv == 0 && lane == 0) || (wv == kWaves - 1 && lane == 63);
    unsigned hx = cx;
    if (wv == 0 && lane == 0) hx = unsigned(x0 > 0 ? x0 - 1 : P->col_lo);
    if (wv == kWaves - 1 && lane == 63) hx = unsigned(x0 + 256 < nx ? x0 + 256 : P->col_hi);
    const bool edge_lane = lane == 0 || lane == 63;
    const int eside = lane == 0 ? 0 : 1;
    // neighbour wave whose edge value this lane needs (lane 0: west wave's
    // lane 63; lane 63: east wave's lane 0)
    const int nwave = lane == 0 ? wv - 1 : wv + 1;
    const int nside = lane == 0 ? 1 : 0;
    const bool hlds = edge_lane && !hmem;
    // reflecting walls (see the end of body)
    const bool ref_ylo = P->bc[YLO] == BC_REFLECT, ref_yhi = P->bc[YHI] == BC_REFLECT;
    const int wx0 = x0 + 64 * wv;
    const bool ref_xwave = (P->bc[XLO] == BC_REFLECT && wx0 == 0) ||
                           (P->bc[XHI] == BC_REFLECT && wx0 <= nx - 1 && nx - 1 < wx0 + 64);
    const bool ref_w = P->bc[XLO] == BC_REFLECT && x == 0;
    const bool ref_e = P->bc[XHI] == BC_REFLECT && x == nx - 1;

    auto publish = [&](const S (&r)[16], int slot) {
        if (edge_lane) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) lds.v[slot][wv][eside][xslot(i)] = r[i];
        }
    };

    auto body = [&](const S (&rm)[16], const S (&r0)[16], const S (&rp)[16], S (&rn)[16],
                    int y) {
        const bool more = y + 1 < y1;
        if (more) {
            const unsigned on = row_offset(P, y + 2);
#pragma unroll
            for (int i = 0; i < 16; ++i) rn[i] = ld(i, on, cx);
        }
        const unsigned o = row_offset(P, y);
        S h[16];
        no_value(h);
        if (hmem) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) h[i] = ld(i, o, hx);
        } else if (hlds) {
            const int slot = y & 1;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) h[i] = lds.v[slot][nwave][nside][xslot(i)];
        }
        S cdt[16];
        C rho, Pp;
        cell_collision<C, COMP>(r0, b, binv, P->sdt, cdt, rho, Pp);
        if (act && !(rho > C(0) && Pp > C(0))) atomicOr(health, 1u);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const S W = moves_x(i) ? from_left(r0[i], h[i]) : S(0);
            const S E = moves_x(i) ? from_right(r0[i], h[i]) : S(0);
            // NT (grids far larger than the last-level cache): non-temporal
            // stores, so the new rows do not displace the halo rows that
            // other blocks still read; smaller grids keep them cached for
            // the next step
            S* dst = &(fo + (long long)i * plane)[o + xs];
            const S v = site_update(P, i, r0[i], W, E, rm[i], rp[i], cdt[i]);
            if constexpr (NT)
                __builtin_nontemporal_store(v, dst);
            else
                *dst = v;
        }
        // WALLS: reflecting walls of the next step.  The ghosts of the new
        // state next to a wall are the reflections of the wall cells just
        // stored, so the lanes that stored them read them back and write the
        // ghosts (no ghost pass between steps: one launch per step instead
        // of two, which pays on small, launch-bound grids; the extra
        // registers cost large grids more than the ghost launch saves)
        const bool wall_lo = ref_ylo && y == 0, wall_hi = ref_yhi && y == P->ny - 1;
        if (WALLS && (wall_lo || wall_hi || ref_xwave)) {
            S v[16], g[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = (fo + (long long)i * plane)[o + xs];
            if (wall_lo || wall_hi) {
                reflected_eq<C>(v, 1, b, binv, g);
                if (wall_lo) {
                    const unsigned og = row_offset(P, -1) + xs;
#pragma unroll
                    for (int i = 0; i < 16; ++i) (fo + (long long)i * plane)[og] = g[i];
                }
                if (wall_hi) {
                    const unsigned og = row_offset(P, P->ny) + xs;
#pragma unroll
                    for (int i = 0; i < 16; ++i) (fo + (long long)i * plane)[og] = g[i];
                }
            }
            if (ref_xwave) {
                reflected_eq<C>(v, 0, b, binv, g);
                // column -1 and / or nx of this row (both on a one-column
                // grid; 32-bit sums: o >= 64)
                if (ref_w) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) (fo + (long long)i * plane)[o - 1u] = g[i];
                }
                if (ref_e) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) (fo + (long long)i * plane)[o + unsigned(nx)] = g[i];
                }
            }
        }
        // hand row y+1's edge values to the neighbour waves
        if (more) publish(rp, (y + 1) & 1);
        __syncthreads();
    };

    S A[16], B[16], Cw[16], D[16];
    {
        const unsigned om = row_offset(P, y0 - 1), o0 = row_offset(P, y0), op = row_offset(P, y0 + 1);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            B[i] = ld(i, o0, cx);
            Cw[i] = ld(i, op, cx);
            A[i] = moves_y(i) ? ld(i, om, cx) : S(0);
            D[i] = S(0);
        }
    }
    publish(B, y0 & 1);
    __syncthreads();
    // rows rotate through four register sets, so no copies between rows
    for (int y = y0; y < y1;) {
        body(A, B, Cw, D, y); ++y;
        if (y >= y1) break;
        body(B, Cw, D, A, y); ++y;
        if (y >= y1) break;
        body(Cw, D, A, B, y); ++y;
        if (y >= y1) break;
        body(D, A, B, Cw, y); ++y;
    }
}

// Waves per SIMD the WALLS step kernel is held to: three for FP32 storage
// with FP64 collision (168 VGPRs, as the plain kernel uses by itself), two
// otherwise.  The plain kernel is left to the compiler.
template <typename S, bool COMP, bool WALLS>
constexpr int step_waves() { return (WALLS && sizeof(S) == 4 && !COMP) ? 3 : 1; }

template <typename S, typename C, bool COMP, bool NT, bool WALLS>
__global__ __launch_bounds__(256, (step_waves<S, COMP, WALLS>())) void step_kernel(const Inst* __restrict__ insts,
                                                   const Item* __restrict__ items, int nitems,
                                                   const S* __restrict__ fin, S* __restrict__ fout,
                                                   unsigned* __restrict__ health) {
    __shared__ EdgeBuf<S> lds;
    // Workgroups are dealt round-robin to the 8 XCDs (workgroup g -> XCD
    // g % 8), each with its own L2.  Ordinal q of the launch runs item
    // (q % 8) * per + q / 8, so every XCD sweeps one contiguous run of the
    // item table (row bands, x fastest) and neighbouring items, which share
    // halo cache lines, meet in the same L2 at about the same time.
    const int per = (nitems + 7) >> 3;
    for (int q = blockIdx.x; q < 8 * per; q += gridDim.x) {
        const int w = (q & 7) * per + (q >> 3);
        if (w >= nitems) continue;
        const Item it = items[w];
        step_block<S, C, COMP, NT, WALLS>(insts + it.inst, it.x0, it.y0, it.y1, fin, fout, health, lds);
        __syncthreads();   // the next item reuses the edge buffer
    }
}

// ---------------------------------------------------------------- two steps

// Two time steps per pass over the populations (temporal blocking), FP32
// storage.  The single-step kernel moves 128 B per site update and is bound
// by HBM; here a block reads f^n once, keeps f^{n+1} in registers only and
// writes f^{n+2}: half the memory traffic per step for a little recomputation
// at the band edges.  A work item is 256 columns [x0, x0 + 256) of rows
// [y0, y1), y1 - y0 <= kBand2; the block marches rows y = y0 - 1 .. y1 and
// at row y
//  * computes f^{n+1} of row y from the f^n window (rows y-1, y, y+1; the
//    single-step arithmetic, x neighbours by DPP / LDS / the two halo-column
//    loads, row y + 2 prefetched), the halo rows y0 - 1 and y1 included;
//  * computes f^{n+2} of row y - 1 from the f^{n+1} window (rows y-2, y-1,
//    y) and stores it (y0 < y <= y1).
// The x neighbours of f^{n+1} outside the block (columns x0 - 1 and
// min(x0 + 256, nx)) are computed before the march, one lane per row and
// side (cell_update; the rows dealt to the four waves), and kept in LDS.
// Boundaries at the intermediate level follow the same rules as a stored
// state: periodic sides are computed at the wrapped cell (rows -2 / ny + 1
// are read through a two-deep wrap), outflow, reflecting and
// fixed-equilibrium ghosts are the adjacent f^{n+1} cell, its reflection,
// and the side's equilibrium.  The f^{n+2} ghost ring is refilled by the
// ghost pass before the next launch.
constexpr int kBand2 = 64;

// The instance pointer made opaque to the compiler, so that the parameters
// read through it (rates, Lax-Wendroff weights) are loaded again where they
// are used instead of being held in scalar registers across the whole march
// (which spills them to vector-register lanes); as a constant-address-space
// pointer, so that the loads stay scalar.
using ConstInst = const __attribute__((address_space(4))) Inst;
using ConstItem = const __attribute__((address_space(4))) Item;
__device__ __forceinline__ ConstInst* reload(ConstInst* p) {
    unsigned long long a = reinterpret_cast<unsigned long long>(p);
    asm volatile("" : "+s"(a));
    return reinterpret_cast<ConstInst*>(a);
}

// The march addresses population i of a row as a wave-uniform 64-bit
// pointer (scalar registers) plus the lane's 32-bit byte offset, which the
// memory instruction adds itself (no vector arithmetic per access).  The
// pointer steps from population to population through an opaque register,
// so the sixteen population bases are formed per row (two scalar adds each)
// instead of being held, and spilled, across the march.
using GByte = __attribute__((address_space(1))) char;
// The lane's byte offset, re-formed where a row's accesses are issued: the
// instruction selector takes the scalar-base form only when it sees the
// offset as a 32-bit value in the same block.
__device__ __forceinline__ unsigned lane_off(unsigned o) {
    asm volatile("" : "+v"(o));
    return o;
}
__device__ __forceinline__ unsigned long long next_pop(unsigned long long a, unsigned long long step) {
    a += step;
    asm("" : "+s"(a));
    return a;
}
template <typename S>
__device__ __forceinline__ S gload(unsigned long long a, unsigned boff) {
    using GS = const __attribute__((address_space(1))) S;
    return *reinterpret_cast<GS*>(reinterpret_cast<const GByte*>(a) + boff);
}
template <typename S, bool NT>
__device__ __forceinline__ void gstore(unsigned long long a, unsigned boff, S v) {
    using GS = __attribute__((address_space(1))) S;
    GS* p = reinterpret_cast<GS*>(reinterpret_cast<GByte*>(a) + boff);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <typename S>
struct EdgeBuf2 {
    S v[2][2][kWaves][2][12];      // [slot][level][wave][lane 0 / 63][x-moving population]
    S halo[2][kBand2][12];         // [west / east][row - y0]: f^{n+1} of the halo columns
};

// f^{n+1} of the grid cell (sx, y), 0 <= sx < nx, 0 <= y < ny, from f^n
// with the neighbours through the one-deep remap (one lane's single step).
template <typename S, typename C, bool COMP>
__device__ void cell_update(ConstInst* __restrict__ P, const S* __restrict__ fi, int sx, int y,
                            C b, C binv, S out[16]) {
    const long long plane = P->plane;
    const unsigned o = row_offset(P, y), om = row_offset(P, y - 1), op = row_offset(P, y + 1);
    const unsigned c = unsigned(sx);
    const unsigned cw = unsigned(sx > 0 ? sx - 1 : P->col_lo);
    const unsigned ce = unsigned(sx + 1 < P->nx ? sx + 1 : P->col_hi);
    auto ld = [&](int i, unsigned row, unsigned col) -> S {
        return (fi + (long long)i * plane)[row + col];
    };
    S f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = ld(i, o, c);
    S cdt[16];
    C rho, Pp;
    cell_collision<C, COMP>(f, b, binv, P->sdt, cdt, rho, Pp);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const S W = moves_x(i) ? ld(i, o, cw) : S(0);
        const S E = moves_x(i) ? ld(i, o, ce) : S(0);
        const S So = moves_y(i) ? ld(i, om, c) : S(0);
        const S N = moves_y(i) ? ld(i, op, c) : S(0);
        out[i] = site_update(P, i, f[i], W, E, So, N, cdt[i]);
    }
}

// The f^{n+1} ghost row of a non-periodic y side from the adjacent row
// `v` (fixed equilibrium, outflow copy, or reflection).
template <typename S, typename C>
__device__ __forceinline__ void ghost_row_rule(ConstInst* __restrict__ P, int side, const S (&v)[16],
                                               C b, C binv, S (&g)[16]) {
    const int kind = P->bc[side];
    if (kind == BC_EQ) {
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = S(P->ghost[side][i]);
    } else if (kind == BC_REFLECT) {
        reflected_eq<C>(v, 1, b, binv, g);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = v[i];
    }
}

template <typename S, typename C, bool COMP, bool NT, bool W4>
__device__ __forceinline__ void step2_block(ConstInst* __restrict__ P, int x0, int y0, int y1,
                                            const S* __restrict__ fin, S* __restrict__ fout,
                                            unsigned* __restrict__ health, EdgeBuf2<S>& lds) {
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long plane = P->plane;
    const S* __restrict__ fi = fin + P->off;
    S* __restrict__ fo = fout + P->off;
    const int nx = P->nx, ny = P->ny;
    const int x = x0 + 64 * wv + lane;
    const bool act = x < nx;
    const unsigned cx = unsigned(act ? x : P->col_hi);
    const unsigned xs = unsigned(act ? x : nx + 1);
    const C b = C(P->b), binv = C(P->binv);
    auto ld = [&](int i, unsigned row, unsigned col) -> S {
        return (fi + (long long)i * plane)[row + col];
    };
    const bool west = wv == 0 && lane == 0, east = wv == kWaves - 1 && lane == 63;
    const bool hmem = west || east;
    unsigned hx = cx;
    if (west) hx = unsigned(x0 > 0 ? x0 - 1 : P->col_lo);
    if (east) hx = unsigned(x0 + 256 < nx ? x0 + 256 : P->col_hi);
    // Row pointers of the march point at column -1 (the west ghost column,
    // the lowest column read: col_lo is -1 on fixed-equilibrium and
    // reflecting sides), so the lanes' byte offsets (column + 1) * sizeof(S)
    // are never negative; a row holds fewer than 2^28 elements, so they fit
    // 32 bits.
    const unsigned long long fib = reinterpret_cast<unsigned long long>(fi);
    const unsigned long long fob = reinterpret_cast<unsigned long long>(fo);
    const unsigned long long pstep = (unsigned long long)plane * sizeof(S);
    const unsigned bcx = (cx + 1u) * unsigned(sizeof(S)), bhx = (hx + 1u) * unsigned(sizeof(S));
    const unsigned bxs = (xs + 1u) * unsigned(sizeof(S));
    auto row_at = [&](unsigned long long base, unsigned o) {
        return base + ((unsigned long long)o - 1u) * sizeof(S);
    };
    const bool edge_lane = lane == 0 || lane == 63;
    const int eside = lane == 0 ? 0 : 1;
    const int nwave = lane == 0 ? wv - 1 : wv + 1;
    const int nside = lane == 0 ? 1 : 0;
    const bool hlds = edge_lane && !hmem;
    // When the grid ends inside the block, the first lane past it (x = nx,
    // inactive) holds the east halo column's f^{n+1} of the rows the block
    // advances, so that the DPP shift or the neighbour wave hands the last
    // grid column that value as its east neighbour.
    const int xe = x0 + 256 < nx ? x0 + 256 : nx;
    const bool east_src = x == xe;
    const bool per_lo = P->bc[YLO] == BC_PERIODIC, per_hi = P->bc[YHI] == BC_PERIODIC;
    // W4: the launch holds bands that are a whole periodic height of four
    // rows (a separate instantiation, so that other launches keep the
    // registers and schedule of the plain march)
    const bool wrap4 = W4 && per_lo && per_hi && y0 == 0 && y1 == ny && ny == 4;
    // row offsets from values read once per item (the march reads the
    // instance only through reload(); periodic sides wrap two rows deep,
    // other sides go through the one-deep remap: rows -2 / ny + 1 are then
    // read only for values the boundary rule replaces)
    const unsigned origin = unsigned(P->origin), pitch = unsigned(P->pitch);
    const int row_lo = P->row_lo, row_hi = P->row_hi;
    auto roff = [&](int y) -> unsigned {
        const int r = y < 0 ? row_lo : (y >= ny ? row_hi : y);
        return origin + unsigned(r) * pitch;
    };
    auto roff2 = [&](int y) -> unsigned {
        int r = y;
        if (y < 0) {
            if (per_lo) {
                r = y + ny;
                if (r < 0) r += ny;
            } else {
                r = row_lo;
            }
        } else if (y >= ny) {
            if (per_hi) {
                r = y - ny;
                if (r >= ny) r -= ny;
            } else {
                r = row_hi;
            }
        }
        return origin + unsigned(r) * pitch;
    };

    auto publish = [&](const S (&r)[16], int slot, int level) {
        if (edge_lane) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) lds.v[slot][level][wv][eside][xslot(i)] = r[i];
        }
    };

    // f^{n+1} of the halo columns, rows [y0, y1), run after the initial row
    // loads are issued, so that they are in flight during it.  Lanes 0-31 of
    // a wave take the west column, 32-63 the east; row r goes to wave r % 4
    // (each wave runs the cell update once, in parallel, instead of three
    // waves waiting at the first barrier for wave 0 to do all rows: measured
    // 1.3 % faster on the 4096^2 grid, with identical results), except in
    // four-row periodic bands, where wave 0 does all four rows (one cell
    // update in place of four against a march of four rows).
    auto halo_prologue = [&]() {
        const int side = lane >> 5, j = lane & 31;
        const int r = W4 ? j : wv + kWaves * j, y = y0 + r;
        const bool mine = W4 ? wv == 0 : j < kBand2 / kWaves;
        if (mine && y < y1) {
            const int hc = side == 0 ? x0 - 1 : xe;
            const int bside = side == 0 ? XLO : XHI;
            int src = hc, rule = 0;          // 0: f^{n+1}(src); 1: its reflection; 2: equilibrium
            if (hc < 0 || hc >= nx) {
                const int kind = P->bc[bside];
                if (kind == BC_PERIODIC) {
                    src = side == 0 ? nx - 1 : 0;
                } else if (kind == BC_EQ) {
                    rule = 2;
                } else {
                    src = side == 0 ? 0 : nx - 1;
                    rule = kind == BC_REFLECT ? 1 : 0;
                }
            }
            S g[16];
            if (rule == 2) {
#pragma unroll
                for (int i = 0; i < 16; ++i) g[i] = S(P->ghost[bside][i]);
            } else {
                S u[16];
                cell_update<S, C, COMP>(P, fi, src, y, b, binv, u);
                if (rule == 1) {
                    reflected_eq<C>(u, 0, b, binv, g);
                } else {
#pragma unroll
                    for (int i = 0; i < 16; ++i) g[i] = u[i];
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) lds.halo[side][r][xslot(i)] = g[i];
        }
    };
    // rm, r0, rp, rn: f^n rows y-1, y, y+1, y+2 (prefetched);
    // q2, q1, qn: f^{n+1} rows y-2, y-1, y (qn computed here).  Health is
    // accumulated per lane and reported once per item (FP64 collision;
    // measured faster) or reported per row (pure FP32; measured faster).
    bool healthy = true;
    auto check = [&](bool ok) {
        if constexpr (COMP) {
            if (act && !ok) atomicOr(health, 1u);
        } else {
            healthy = healthy && ok;
        }
    };
    auto body = [&](const S (&rm)[16], const S (&r0)[16], const S (&rp)[16], S (&rn)[16],
                    const S (&q2)[16], S (&q1)[16], S (&qn)[16], int y) {
        const bool more = y < y1;
        // A band that is a whole periodic height of four rows already holds
        // what the march would compute or load from row y1 - 1 on, in the
        // register sets those rows rotate into: f^{n+1} of rows y1 - 1 and
        // y1 (the wrapped rows y0 - 1 and y0, computed first) and f^n of
        // rows y0 + 2 and y0 + 3 (the wrapped rows y0 - 2 and y0 - 1, loaded
        // first).  Such a band loads each f^n row once, all four before the
        // march, and computes each f^{n+1} row once.
        const bool fresh = !(wrap4 && y >= y1 - 1);
        if (more && !wrap4) {
            unsigned long long a = row_at(fib, roff2(y + 2));
            const unsigned bo = lane_off(bcx);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                rn[i] = gload<S>(a, bo);
                if (i < 15) a = next_pop(a, pstep);
            }
        }
        // f^{n+1}, row y
        if (fresh) {
            ConstInst* __restrict__ Pc = reload(P);
            const unsigned o = roff2(y);
            S h[16];
            no_value(h);
            if (hmem) {
                unsigned long long a = row_at(fib, o);
                const unsigned bo = lane_off(bhx);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    if (moves_x(i)) h[i] = gload<S>(a, bo);
                    if (i < 15) a = next_pop(a, pstep);
                }
            } else if (hlds) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (moves_x(i)) h[i] = lds.v[y & 1][0][nwave][nside][xslot(i)];
            }
            S cdt[16];
            C rho, Pp;
            cell_collision<C, COMP>(r0, b, binv, Pc->sdt, cdt, rho, Pp);
            check(!((y >= 0 && y < ny) || wrap4) || (rho > C(0) && Pp > C(0)));
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const S W = moves_x(i) ? from_left(r0[i], h[i]) : S(0);
                const S E = moves_x(i) ? from_right(r0[i], h[i]) : S(0);
                qn[i] = site_update(Pc, i, r0[i], W, E, rm[i], rp[i], cdt[i]);
            }
        }
        if (east_src && y >= y0 && y < y1) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) qn[i] = lds.halo[1][y - y0][xslot(i)];
        }
        // ghost rows of f^{n+1} on non-periodic y sides
        if (y == 0 && !per_lo) ghost_row_rule<S, C>(P, YLO, qn, b, binv, q1);
        if (y == ny && !per_hi) ghost_row_rule<S, C>(P, YHI, q1, b, binv, qn);
        // f^{n+2}, row y - 1
        if (y > y0) {
            ConstInst* __restrict__ Pc = reload(P);
            const int r = y - 1 - y0;
            S h[16];
            no_value(h);
            if (hmem) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (moves_x(i)) h[i] = lds.halo[west ? 0 : 1][r][xslot(i)];
            } else if (hlds) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (moves_x(i)) h[i] = lds.v[(y - 1) & 1][1][nwave][nside][xslot(i)];
            }
            S cdt[16];
            C rho, Pp;
            cell_collision<C, COMP>(q1, b, binv, Pc->sdt, cdt, rho, Pp);
            check(rho > C(0) && Pp > C(0));
            unsigned long long a = row_at(fob, roff(y - 1));
            const unsigned bo = lane_off(bxs);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const S W = moves_x(i) ? from_left(q1[i], h[i]) : S(0);
                const S E = moves_x(i) ? from_right(q1[i], h[i]) : S(0);
                gstore<S, NT>(a, bo, site_update(Pc, i, q1[i], W, E, q2[i], qn[i], cdt[i]));
                if (i < 15) a = next_pop(a, pstep);
            }
        }
        // hand the edge values of f^n row y+1 and f^{n+1} row y to the
        // neighbour waves
        if (more) {
            publish(rp, (y + 1) & 1, 0);
            publish(qn, y & 1, 1);
        }
        __syncthreads();
    };

    S A[16], B[16], Cw[16], D[16], E[16], F[16], G[16], H[16];
    {
        const unsigned om = roff2(y0 - 2), o0 = roff2(y0 - 1), op = roff2(y0), on = roff2(y0 + 1);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            A[i] = (moves_y(i) || wrap4) ? ld(i, om, cx) : S(0);
            B[i] = ld(i, o0, cx);
            Cw[i] = ld(i, op, cx);
            D[i] = wrap4 ? ld(i, on, cx) : S(0);
            E[i] = F[i] = G[i] = H[i] = S(0);
        }
    }
    halo_prologue();
    publish(B, (y0 - 1) & 1, 0);
    __syncthreads();
    // four register sets per level rotate, so no copies between rows
    for (int y = y0 - 1; y <= y1;) {
        body(A, B, Cw, D, G, H, E, y); ++y;
        if (y > y1) break;
        body(B, Cw, D, A, H, E, F, y); ++y;
        if (y > y1) break;
        body(Cw, D, A, B, E, F, G, y); ++y;
        if (y > y1) break;
        body(D, A, B, Cw, F, G, H, y); ++y;
    }
    // Reflecting y-wall ghosts of f^{n+2} (section (d)), after the march
    // rather than in it (inlined in the march's row rotations they cost the
    // loop 5 %): a band holding a wall row reads back the elements each lane
    // stored itself (its own earlier stores to the same addresses, so the
    // reads see them) and writes their reflection into the ghost row, so the
    // next launch needs no ghost pass for y walls.  A one-row grid writes
    // both ghost rows from its one row.
    const bool ref_lo = P->bc[YLO] == BC_REFLECT && y0 == 0;
    const bool ref_hi = P->bc[YHI] == BC_REFLECT && y1 == ny;
    if (ref_lo || ref_hi) {
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            if (!(side == 0 ? ref_lo : ref_hi)) continue;
            const unsigned o = roff(side == 0 ? 0 : ny - 1) + xs;
            const unsigned og = roff(side == 0 ? -1 : ny) + xs;
            S v[16], g[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = (fo + (long long)i * plane)[o];
            reflected_eq<C>(v, 1, b, binv, g);
#pragma unroll
            for (int i = 0; i < 16; ++i) (fo + (long long)i * plane)[og] = g[i];
        }
    }
    if (act && !healthy) atomicOr(health, 1u);
}

// FP32 storage: two blocks (two waves per SIMD) per CU, the occupancy its
// 213-249 VGPRs (by form) allow; stating it let the compiler schedule for it
// (measured 1 % faster).  FP64 storage holds both register windows in twice
// the registers (320-370 VGPRs): one block per CU.
template <typename S>
constexpr int step2_waves() { return sizeof(S) == 4 ? 2 : 1; }

template <typename S, typename C, bool COMP, bool NT, bool W4>
__global__ __launch_bounds__(256, (step2_waves<S>())) void step2_kernel(const Inst* __restrict__ insts,
                                                    const Item* __restrict__ items, int nitems,
                                                    const S* __restrict__ fin, S* __restrict__ fout,
                                                    unsigned* __restrict__ health) {
    __shared__ EdgeBuf2<S> lds;
    // the instance and item tables do not change during the launch: read
    // them through the constant address space (scalar loads)
    ConstInst* cinsts = (ConstInst*)insts;
    ConstItem* citems = (ConstItem*)items;
    // XCD-aware item order as in step_kernel
    const int per = (nitems + 7) >> 3;
    for (int q = blockIdx.x; q < 8 * per; q += gridDim.x) {
        const int w = (q & 7) * per + (q >> 3);
        if (w >= nitems) continue;
        const int inst = citems[w].inst, x0 = citems[w].x0, y0 = citems[w].y0, y1 = citems[w].y1;
        step2_block<S, C, COMP, NT, W4>(cinsts + inst, x0, y0, y1, fin, fout, health, lds);
        __syncthreads();   // the next item reuses the LDS buffers
    }
}

// ---------------------------------------------------------------- adjoint

// Adjoint of one step on a periodic grid (neighbours wrap through the
// boundary remap of Inst), per cell x (lam = lam^{n+1}):
//   lam^n(x) = lam(x) + LW^T(lam)(x) - dt (dC/df(x))^T lam(x)
// with the collision part from cell_adjoint (mrt_dual.h).  LW^T is the
// forward stencil with mirrored neighbours: the weight f(x+1) had in F(x)
// now multiplies lam(x-1) and vice versa, so lam^n is site_update with the
// W / E and So / N arguments swapped and dt (dC/df)^T lam in place of dt C.
//
// A work item is a block of four waves over 256 columns of a band of rows,
// marching up the band as step_block does: lam rows y-1 .. y+2 in a register
// window of four rotating sets (row y + 2 prefetched), f^n of row y and y + 1
// in two alternating sets (f^n is read at the cell only), x neighbours by
// DPP lane shifts, the edge lanes' values through LDS and the two halo
// columns by a load on one lane each.  Each of lam^{n+1}, f^n and lam^n then
// crosses the memory interface once per cell (plus the band's two halo rows
// of lam), 192 B per cell in FP32 storage.  Partial sums of the rate
// gradient per item go to `partial` (16 doubles per item: the four waves'
// sums added in a fixed order; with `accumulate` they are added to what the
// row holds, so a sweep of many steps is reduced once), reduced in a fixed
// order by reduce_stripes and reduce_partials.
template <typename S, typename C, bool NT>
__device__ __forceinline__ void adjoint_block(ConstInst* __restrict__ P, int item, int x0, int y0,
                                              int y1, const S* __restrict__ lin,
                                              const S* __restrict__ fn, S* __restrict__ lout,
                                              double* __restrict__ partial, bool accumulate,
                                              EdgeBuf<S>& lds, double (&red)[kWaves][12]) {
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = P->nx;
    const int x = x0 + 64 * wv + lane;
    const bool act = x < nx;
    // load column (lanes past the grid read the wrapped neighbour) and store
    // column (lanes past the grid write the unread column nx + 1)
    const unsigned cx = unsigned(act ? x : P->col_hi);
    const unsigned xs = unsigned(act ? x : nx + 1);
    const C b = C(P->b), binv = C(P->binv), dt = C(P->dt);
    const bool hmem = (wv == 0 && lane == 0) || (wv == kWaves - 1 && lane == 63);
    unsigned hx = cx;
    if (wv == 0 && lane == 0) hx = unsigned(x0 > 0 ? x0 - 1 : P->col_lo);
    if (wv == kWaves - 1 && lane == 63) hx = unsigned(x0 + 256 < nx ? x0 + 256 : P->col_hi);
    // scalar row pointers at column -1 plus the lane's byte offset, as in
    // step2_block (no vector address arithmetic per access)
    const unsigned long long lib = reinterpret_cast<unsigned long long>(lin + P->off);
    const unsigned long long fib = reinterpret_cast<unsigned long long>(fn + P->off);
    const unsigned long long lob = reinterpret_cast<unsigned long long>(lout + P->off);
    const unsigned long long pstep = (unsigned long long)P->plane * sizeof(S);
    const unsigned bcx = (cx + 1u) * unsigned(sizeof(S)), bhx = (hx + 1u) * unsigned(sizeof(S));
    const unsigned bxs = (xs + 1u) * unsigned(sizeof(S));
    auto row_at = [&](unsigned long long base, unsigned o) {
        return base + ((unsigned long long)o - 1u) * sizeof(S);
    };
    auto load_row = [&](unsigned long long base, unsigned o, unsigned boff, S (&r)[16], bool ymoving) {
        unsigned long long a = row_at(base, o);
        const unsigned bo = lane_off(boff);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            r[i] = (!ymoving || moves_y(i)) ? gload<S>(a, bo) : S(0);
            if (i < 15) a = next_pop(a, pstep);
        }
    };
    const bool edge_lane = lane == 0 || lane == 63;
    const int eside = lane == 0 ? 0 : 1;
    const int nwave = lane == 0 ? wv - 1 : wv + 1;
    const int nside = lane == 0 ? 1 : 0;
    const bool hlds = edge_lane && !hmem;
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;

    auto publish = [&](const S (&r)[16], int slot) {
        if (edge_lane) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) lds.v[slot][wv][eside][xslot(i)] = r[i];
        }
    };

    // row y: lam window rm / r0 / rp (rows y-1, y, y+1), rn <- row y + 2;
    // fc = f^n of row y, fnx <- f^n of row y + 1
    auto body = [&](const S (&rm)[16], const S (&r0)[16], const S (&rp)[16], S (&rn)[16],
                    const S (&fc)[16], S (&fnx)[16], int y) {
        const bool more = y + 1 < y1;
        if (more) {
            load_row(lib, row_offset(P, y + 2), bcx, rn, false);
            load_row(fib, row_offset(P, y + 1), bcx, fnx, false);
        }
        const unsigned o = row_offset(P, y);
        S h[16];
        no_value(h);
        if (hmem) {
            unsigned long long a = row_at(lib, o);
            const unsigned bo = lane_off(bhx);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if (moves_x(i)) h[i] = gload<S>(a, bo);
                if (i < 15) a = next_pop(a, pstep);
            }
        } else if (hlds) {
            const int slot = y & 1;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (moves_x(i)) h[i] = lds.v[slot][nwave][nside][xslot(i)];
        }
        ConstInst* __restrict__ Pc = reload(P);
        C f[16], lam[16], coll[16], dsk[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            f[i] = C(fc[i]);
            lam[i] = C(r0[i]);
        }
        cell_adjoint(f, lam, b, binv, Pc->sdt, dt, coll, dsk);
        if (act) {
#pragma unroll
            for (int k = 4; k < 16; ++k) acc[k] -= double(dsk[k]);
        }
        unsigned long long a = row_at(lob, o);
        const unsigned bo = lane_off(bxs);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const S W = moves_x(i) ? from_left(r0[i], h[i]) : S(0);
            const S E = moves_x(i) ? from_right(r0[i], h[i]) : S(0);
            // mirrored neighbours: (E, W) and (N, So) in the (W, E), (So, N) slots
            gstore<S, NT>(a, bo, site_update(Pc, i, r0[i], E, W, rp[i], rm[i], S(coll[i])));
            if (i < 15) a = next_pop(a, pstep);
        }
        if (more) publish(rp, (y + 1) & 1);
        __syncthreads();
    };

    S A[16], B[16], Cw[16], D[16], F0[16], F1[16];
    load_row(lib, row_offset(P, y0), bcx, B, false);
    load_row(lib, row_offset(P, y0 + 1), bcx, Cw, false);
    load_row(lib, row_offset(P, y0 - 1), bcx, A, true);
    load_row(fib, row_offset(P, y0), bcx, F0, false);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        D[i] = S(0);
        F1[i] = S(0);
    }
    publish(B, y0 & 1);
    __syncthreads();
    for (int y = y0; y < y1;) {
        body(A, B, Cw, D, F0, F1, y); ++y;
        if (y >= y1) break;
        body(B, Cw, D, A, F1, F0, y); ++y;
        if (y >= y1) break;
        body(Cw, D, A, B, F0, F1, y); ++y;
        if (y >= y1) break;
        body(D, A, B, Cw, F1, F0, y); ++y;
    }
    // wave reduction of the 12 non-trivial rate gradients, then the four
    // waves' sums in a fixed order into the item's partial row
#pragma unroll
    for (int k = 4; k < 16; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[k] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 4; k < 16; ++k) red[wv][k - 4] = acc[k];
    }
    __syncthreads();
    if (wv == 0 && lane < 16) {
        double* row = &partial[(long long)item * 16];
        const double v = lane < 4 ? 0.0
                                  : ((red[0][lane - 4] + red[1][lane - 4]) + red[2][lane - 4]) + red[3][lane - 4];
        row[lane] = accumulate ? row[lane] + v : v;
    }
}

// Two blocks per CU (two waves per SIMD, at most 256 VGPRs) for FP32
// storage; FP64 storage holds twice the register window and runs one.
template <typename S>
constexpr int adjoint_waves() { return sizeof(S) == 4 ? 2 : 1; }

template <typename S, typename C, bool NT>
__global__ __launch_bounds__(256, (adjoint_waves<S>())) void adjoint_kernel(const Inst* __restrict__ insts,
                                                         const Item* __restrict__ items, int nitems,
                                                         const S* __restrict__ lin,
                                                         const S* __restrict__ fn,
                                                         S* __restrict__ lout,
                                                         double* __restrict__ partial,
                                                         int accumulate) {
    __shared__ EdgeBuf<S> lds;
    __shared__ double red[kWaves][12];
    ConstInst* cinsts = (ConstInst*)insts;
    ConstItem* citems = (ConstItem*)items;
    // XCD-aware item order as in step_kernel
    const int per = (nitems + 7) >> 3;
    for (int q = blockIdx.x; q < 8 * per; q += gridDim.x) {
        const int w = (q & 7) * per + (q >> 3);
        if (w >= nitems) continue;
        const int inst = citems[w].inst, x0 = citems[w].x0, y0 = citems[w].y0, y1 = citems[w].y1;
        adjoint_block<S, C, NT>(cinsts + inst, w, x0, y0, y1, lin, fn, lout, partial,
                                accumulate != 0, lds, red);
        __syncthreads();   // the next item reuses the edge buffer
    }
}

// First stage of the rate-gradient reduction: block g of the launch sums
// the partial rows [g * per, min(n, (g + 1) * per)) into stage[g][16]
// (thread t: column t % 16, rows t / 16, t / 16 + 16, ... of the range,
// four running sums added in a fixed order, then the 16 stripes pairwise);
// reduce_partials then adds the stage rows into ds.  Many blocks read the
// partial rows in parallel (one 1024-thread block reading 2,048 rows took
// 23 us of a 2048^2 adjoint step); the order of every addition is fixed, so
// ds is bitwise reproducible.
constexpr int kStageBlocks = 64;
constexpr int kSingleStageRows = 1024;
__global__ __launch_bounds__(256) void reduce_stripes(const double* __restrict__ partial, int n,
                                                      int per, double* __restrict__ stage) {
    __shared__ double red[16][16];
    const int t = threadIdx.x, k = t & 15, stripe = t >> 4;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double a[4] = {0, 0, 0, 0};
    int i = r0 + stripe;
    for (; i + 48 < r1; i += 64) {
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] += partial[(long long)(i + 16 * j) * 16 + k];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)      // fewer than four rows left
        if (i + 16 * j < r1) a[j] += partial[(long long)(i + 16 * j) * 16 + k];
    red[stripe][k] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    for (int half = 8; half >= 1; half >>= 1) {
        if (stripe < half) red[stripe][k] += red[stripe + half][k];
        __syncthreads();
    }
    if (t < 16) stage[blockIdx.x * 16 + t] = red[0][t];
}

// ds[k] += sum over the n partial rows of partial[row][k]: one block of
// 1024 threads, thread t sums column t % 16 over rows t / 16, t / 16 + 64,
// ... (eight at a time into eight sums: the serial chain of dependent loads
// took 1.6 us of a 256^2 adjoint step); the 64 stripe sums are then added
// pairwise in six stages (a fixed order, so the result is bitwise
// reproducible).  A separate launch: having
// the adjoint kernel's last block reduce instead (every block releasing its
// rows device-wide) measured 2.2x slower at 256^2, the release fences
// writing back the L2.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void reduce_partials(const double* __restrict__ partial,
                                                                  int n, double* __restrict__ ds) {
    constexpr int kStripes = kReduceThreads / 16;
    __shared__ double red[kStripes][16];
    const int t = threadIdx.x, k = t & 15, stripe = t >> 4;
    // eight accumulators over the stripe's rows i, i + 64, ..., i + 448 of
    // each group (eight loads in flight instead of a chain of dependent
    // ones), added in a fixed order
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = stripe;
    for (; i + 7 * kStripes < n; i += 8 * kStripes) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] += partial[(long long)(i + j * kStripes) * 16 + k];
    }
#pragma unroll
    for (int j = 0; j < 7; ++j)      // fewer than eight rows left
        if (i + j * kStripes < n) a[j] += partial[(long long)(i + j * kStripes) * 16 + k];
    red[stripe][k] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    // a stage writes only the stripes below `half` and reads only those from
    // `half` on
    for (int half = kStripes / 2; half >= 1; half >>= 1) {
        if (stripe < half) red[stripe][k] += red[stripe + half][k];
        __syncthreads();
    }
    if (t < 16) ds[t] += red[0][t];
}

// ------------------------------------------------------------- tube march

}  // namespace mrt

#include "mrt_tube.h"

namespace mrt {

// Several time steps per pass for grids of NY = 1, 2 or 4 periodic rows
// whose x sides hold fixed equilibria (the shock tubes of section (b)).  All
// rows of a tube sit in the registers of one block, so the block can
// advance them L steps before it stores: level k + 1 of row r is the
// single-step update of rows r - 1, r, r + 1 (mod NY) of level k.  A block
// covers the 256 columns x0 - L .. x0 + 255 - L (lane l = 64 w + lane at
// x0 - L + l); level k is exact on the lanes k <= l <= 255 - k, since each
// level needs one more column on either side, so a block stores f^{n+L} of
// the 256 - 2L columns x0 .. x0 + 255 - 2L and the tube's next block starts
// there (the overlap is recomputed: 2L of 256 lanes; L = kTubeSteps,
// kTubeWidth stored columns).  No column outside the block is needed: the
// halo-column computation of the two-step march disappears.  The ghost
// columns x = -1 and x = nx keep their side's equilibrium at every level;
// lanes further out carry values that reach no stored cell.  Per level the
// edge lanes of the four waves swap the rows' x-moving populations through
// LDS (double buffered: one barrier per level).  The state crosses the
// memory interface once per L steps.

template <typename S>
struct TubeEdges {
    S v[2][kWaves][2][4][12];      // [slot][wave][lane 0 / 63][row][x-moving population]
};

template <typename S, typename C, bool COMP, bool NT, int L, int NY>
__device__ __forceinline__ void tube_block(ConstInst* __restrict__ P, int x0,
                                           const S* __restrict__ fin, S* __restrict__ fout,
                                           unsigned* __restrict__ health, TubeEdges<S>& lds) {
    static_assert(L % 2 == 0, "levels alternate between two register sets");
    static_assert(NY == 1 || NY == 2 || NY == 4, "one, two or four rows");
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = 64 * wv + lane;
    const int nx = P->nx;
    const int x = x0 - L + l;
    const long long plane = P->plane;
    const S* __restrict__ fi = fin + P->off;
    S* __restrict__ fo = fout + P->off;
    const unsigned origin = unsigned(P->origin), pitch = unsigned(P->pitch);
    // load column: lanes outside the grid and its ghost ring read the ghost
    // column of their side (values that reach no stored cell)
    const unsigned cx = unsigned(x < -1 ? -1 : (x > nx ? nx : x));
    const C b = C(P->b), binv = C(P->binv);
    // whether this wave holds the west (x = -1) or east (x = nx) ghost column
    const int xw = x0 - L + 64 * wv;
    const bool wave_west = xw <= -1 && xw + 63 >= -1, wave_east = xw <= nx && xw + 63 >= nx;
    const bool edge_lane = lane == 0 || lane == 63;
    const int eside = lane == 0 ? 0 : 1;
    const int nwave = lane == 0 ? wv - 1 : wv + 1;
    const int nside = lane == 0 ? 1 : 0;
    const bool hlds = edge_lane && nwave >= 0 && nwave < kWaves;
    bool healthy = true;

    S A[NY][16], B[NY][16];
#pragma unroll
    for (int r = 0; r < NY; ++r) {
        const unsigned o = origin + unsigned(r) * pitch;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            A[r][i] = (fi + (long long)i * plane)[o + cx];
            B[r][i] = S(0);
        }
    }
    // dst = level k + 1 from src = level k
    auto level = [&](S (&src)[NY][16], S (&dst)[NY][16], int k) {
        // the ghost columns: their side's equilibrium at every level (the
        // side index is wave-uniform, so the values come from scalar loads)
        if (k > 0 && wave_west && x == -1) {
#pragma unroll
            for (int r = 0; r < NY; ++r)
#pragma unroll
                for (int i = 0; i < 16; ++i) src[r][i] = S(P->ghost[XLO][i]);
        }
        if (k > 0 && wave_east && x == nx) {
#pragma unroll
            for (int r = 0; r < NY; ++r)
#pragma unroll
                for (int i = 0; i < 16; ++i) src[r][i] = S(P->ghost[XHI][i]);
        }
        if (edge_lane) {
#pragma unroll
            for (int r = 0; r < NY; ++r)
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (moves_x(i)) lds.v[k & 1][wv][eside][r][xslot(i)] = src[r][i];
        }
        __syncthreads();
        const bool valid = l > k && l < 255 - k && x >= 0 && x < nx;
        ConstInst* __restrict__ Pc = reload(P);
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            S h[16];
            no_value(h);
            if (hlds) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (moves_x(i)) h[i] = lds.v[k & 1][nwave][nside][r][xslot(i)];
            }
            S cdt[16];
            C rho, Pp;
            cell_collision<C, COMP>(src[r], b, binv, Pc->sdt, cdt, rho, Pp);
            healthy = healthy && (!valid || (rho > C(0) && Pp > C(0)));
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const S W = moves_x(i) ? from_left(src[r][i], h[i]) : S(0);
                const S E = moves_x(i) ? from_right(src[r][i], h[i]) : S(0);
                dst[r][i] = site_update(Pc, i, src[r][i], W, E, src[(r + NY - 1) % NY][i],
                                        src[(r + 1) % NY][i], cdt[i]);
            }
            // the row's new values are materialised here, in row order: left
            // free, the compiler sinks every row's update to the next level
            // and overlaps the four rows' collisions (412 registers)
#pragma unroll
            for (int i = 0; i < 16; ++i) asm volatile("" : "+v"(dst[r][i]));
        }
    };
    for (int k = 0; k < L; k += 2) {
        level(A, B, k);
        level(B, A, k + 1);
    }
    if (x >= 0 && x < nx && l >= L && l <= 255 - L) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const unsigned o = origin + unsigned(r) * pitch + unsigned(x);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                S* p = fo + (long long)i * plane + o;
                if constexpr (NT)
                    __builtin_nontemporal_store(A[r][i], p);
                else
                    *p = A[r][i];
            }
        }
    }
    if (!healthy) atomicOr(health, 1u);
}

// Two blocks (two waves per SIMD) per CU; FP64 storage with four rows holds
// two register sets of 64 doubles per lane: one.
template <typename S, int NY>
constexpr int tube_waves() { return sizeof(S) == 8 && NY == 4 ? 1 : 2; }

template <typename S, typename C, bool COMP, bool NT, int L, int NY>
__global__ __launch_bounds__(256, (tube_waves<S, NY>())) void tube_kernel(
        const Inst* __restrict__ insts, const Item* __restrict__ items, int nitems,
        const S* __restrict__ fin, S* __restrict__ fout, unsigned* __restrict__ health) {
    __shared__ TubeEdges<S> lds;
    ConstInst* cinsts = (ConstInst*)insts;
    ConstItem* citems = (ConstItem*)items;
    // XCD-aware item order as in step_kernel
    const int per = (nitems + 7) >> 3;
    for (int q = blockIdx.x; q < 8 * per; q += gridDim.x) {
        const int w = (q & 7) * per + (q >> 3);
        if (w >= nitems) continue;
        tube_block<S, C, COMP, NT, L, NY>(cinsts + citems[w].inst, citems[w].x0, fin, fout, health, lds);
        __syncthreads();   // the next item reuses the LDS buffers
    }
}

// ------------------------------------------------- scheme variants
//
// The two other readings of the paper's time/space discretisation, one
// thread per cell (they are for comparing readings, not the tuned path):
//  * collide-then-stream: collide_kernel writes h = f - dt C(f), then
//    cell_step_kernel<COLLIDE = false> convects h: f^{n+1} = h + LW(h);
//  * nine-point Lax-Wendroff: cell_step_kernel<CROSS = true> adds the
//    mixed-derivative term (|c_x c_y| / 4) s_x s_y (NE - NW - SE + SW) for the
//    diagonal populations; with COLLIDE it is the unsplit step.
// Neighbours come through the boundary remap of Inst (corner ghosts: see
// ghost_kernel).

__device__ __forceinline__ unsigned col_remap(const Inst* __restrict__ P, int x) {
    return unsigned(x < 0 ? P->col_lo : (x >= P->nx ? P->col_hi : x));
}

template <typename S, typename C, bool COMP>
__global__ __launch_bounds__(256) void collide_kernel(const Inst* __restrict__ P,
                                                      const S* __restrict__ fin,
                                                      S* __restrict__ fout,
                                                      unsigned* __restrict__ health) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= P->nx) return;
    const long long plane = P->plane;
    const S* __restrict__ fi = fin + P->off;
    S* __restrict__ fo = fout + P->off;
    const C b = C(P->b), binv = C(P->binv);
    for (int y = blockIdx.y; y < P->ny; y += gridDim.y) {
        const unsigned o = row_offset(P, y) + unsigned(x);
        S f[16], cdt[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) f[i] = (fi + (long long)i * plane)[o];
        C rho, Pp;
        cell_collision<C, COMP>(f, b, binv, P->sdt, cdt, rho, Pp);
        if (!(rho > C(0) && Pp > C(0))) atomicOr(health, 1u);
#pragma unroll
        for (int i = 0; i < 16; ++i) (fo + (long long)i * plane)[o] = f[i] - cdt[i];
    }
}

template <typename S, typename C, bool COMP, bool COLLIDE, bool CROSS>
__global__ __launch_bounds__(256) void cell_step_kernel(const Inst* __restrict__ P,
                                                        const S* __restrict__ fin,
                                                        S* __restrict__ fout,
                                                        unsigned* __restrict__ health) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= P->nx) return;
    const long long plane = P->plane;
    const S* __restrict__ fi = fin + P->off;
    S* __restrict__ fo = fout + P->off;
    const C b = C(P->b), binv = C(P->binv);
    const unsigned xc = unsigned(x), xw = col_remap(P, x - 1), xe = col_remap(P, x + 1);
    for (int y = blockIdx.y; y < P->ny; y += gridDim.y) {
        const unsigned o = row_offset(P, y), on = row_offset(P, y + 1), os = row_offset(P, y - 1);
        auto ld = [&](int i, unsigned row, unsigned col) -> S {
            return (fi + (long long)i * plane)[row + col];
        };
        S f[16], cdt[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            f[i] = ld(i, o, xc);
            cdt[i] = S(0);
        }
        if constexpr (COLLIDE) {
            C rho, Pp;
            cell_collision<C, COMP>(f, b, binv, P->sdt, cdt, rho, Pp);
            if (!(rho > C(0) && Pp > C(0))) atomicOr(health, 1u);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = i >> 2, sx = sgn_x(i), sy = sgn_y(i);
            const S E = sx != 0 ? ld(i, o, xe) : S(0), W = sx != 0 ? ld(i, o, xw) : S(0);
            const S N = sy != 0 ? ld(i, on, xc) : S(0), So = sy != 0 ? ld(i, os, xc) : S(0);
            // the per-axis increment exactly as the marching kernels form it;
            // the mixed-derivative term (nine-point stencil) is added last
            S d = lw_increment(P, i, f[i], W, E, So, N, cdt[i]);
            if constexpr (CROSS) {
                if (sx != 0 && sy != 0) {
                    const S ne = ld(i, on, xe), nw = ld(i, on, xw);
                    const S se = ld(i, os, xe), sw = ld(i, os, xw);
                    const S wc = Weights<S>::cross(P, k);
                    const S sxy = S(sx * sy);
                    d = fma_s(sxy * wc, (ne - nw) - (se - sw), d);
                }
            }
            (fo + (long long)i * plane)[o + xc] = f[i] + d;
        }
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

template <typename S, typename C, bool COMP, bool NT, bool WALLS>
void launch_step_kernel(int blocks, const Inst* insts, const Item* items, int nitems,
                        const void* fin, void* fout, unsigned* health, hipStream_t st) {
    hipLaunchKernelGGL((step_kernel<S, C, COMP, NT, WALLS>), dim3(blocks), dim3(256), 0, st, insts,
                       items, nitems, static_cast<const S*>(fin), static_cast<S*>(fout), health);
}

template <typename S, typename C, bool COMP>
hipError_t launch_step(const Inst* insts, const Item* items, int nitems, const void* fin,
                       void* fout, unsigned* health, int grid, bool nt, bool walls, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int blocks = grid > 0 ? grid : 8 * ((nitems + 7) / 8);
    if (nt) {
        if (walls) launch_step_kernel<S, C, COMP, true, true>(blocks, insts, items, nitems, fin, fout, health, st);
        else launch_step_kernel<S, C, COMP, true, false>(blocks, insts, items, nitems, fin, fout, health, st);
    } else {
        if (walls) launch_step_kernel<S, C, COMP, false, true>(blocks, insts, items, nitems, fin, fout, health, st);
        else launch_step_kernel<S, C, COMP, false, false>(blocks, insts, items, nitems, fin, fout, health, st);
    }
    return hipGetLastError();
}

template <typename S, typename C, bool COMP, bool NT>
void launch_step2_w(const Inst* insts, const Item* items, int nitems, const void* fin, void* fout,
                    unsigned* health, int blocks, bool wrap4, hipStream_t st) {
    if (wrap4)
        hipLaunchKernelGGL((step2_kernel<S, C, COMP, NT, true>), dim3(blocks), dim3(256), 0, st, insts,
                           items, nitems, static_cast<const S*>(fin), static_cast<S*>(fout), health);
    else
        hipLaunchKernelGGL((step2_kernel<S, C, COMP, NT, false>), dim3(blocks), dim3(256), 0, st, insts,
                           items, nitems, static_cast<const S*>(fin), static_cast<S*>(fout), health);
}

template <typename S, typename C, bool COMP>
hipError_t launch_step2(const Inst* insts, const Item* items, int nitems, const void* fin,
                        void* fout, unsigned* health, int grid, bool nt, bool wrap4, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int blocks = grid > 0 ? grid : 8 * ((nitems + 7) / 8);
    if (nt)
        launch_step2_w<S, C, COMP, true>(insts, items, nitems, fin, fout, health, blocks, wrap4, st);
    else
        launch_step2_w<S, C, COMP, false>(insts, items, nitems, fin, fout, health, blocks, wrap4, st);
    return hipGetLastError();
}

template <typename S, typename C, bool COMP, bool NT>
void launch_tube_nt(const Inst* insts, const Item* items, int nitems, const S* fin, S* fout,
                    unsigned* health, int blocks, int ny, hipStream_t st) {
    switch (ny) {
        case 1:
            hipLaunchKernelGGL((tube_kernel<S, C, COMP, NT, kTubeSteps, 1>), dim3(blocks), dim3(256), 0,
                               st, insts, items, nitems, fin, fout, health);
            break;
        case 2:
            hipLaunchKernelGGL((tube_kernel<S, C, COMP, NT, kTubeSteps, 2>), dim3(blocks), dim3(256), 0,
                               st, insts, items, nitems, fin, fout, health);
            break;
        default:
            hipLaunchKernelGGL((tube_kernel<S, C, COMP, NT, kTubeSteps, 4>), dim3(blocks), dim3(256), 0,
                               st, insts, items, nitems, fin, fout, health);
            break;
    }
}

template <typename S, typename C, bool COMP>
hipError_t launch_tube(const Inst* insts, const Item* items, int nitems, const void* fin, void* fout,
                       unsigned* health, int grid, bool nt, int ny, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (ny != 1 && ny != 2 && ny != 4) return hipErrorInvalidValue;
    const int blocks = grid > 0 ? grid : 8 * ((nitems + 7) / 8);
    const S* in = static_cast<const S*>(fin);
    S* out = static_cast<S*>(fout);
    if (nt)
        launch_tube_nt<S, C, COMP, true>(insts, items, nitems, in, out, health, blocks, ny, st);
    else
        launch_tube_nt<S, C, COMP, false>(insts, items, nitems, in, out, health, blocks, ny, st);
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

// Ghost cells of `count` instances (instance table `insts`, longest
// perimeter 2 * (nx + ny) = perim) in buffer f; mode bit 0: reflecting
// sides, bit 1: fixed-equilibrium sides.
hipError_t k_ghost(int prec, const Inst* insts, int count, int perim, void* f, int mode,
                   hipStream_t st) {
    const dim3 grid((perim + 4 + 255) / 256, count);   // + the four corners
    switch (prec) {
        case 0: hipLaunchKernelGGL((ghost_kernel<double, double>), grid, dim3(256), 0, st, insts, static_cast<double*>(f), mode); break;
        case 1: hipLaunchKernelGGL((ghost_kernel<float, float>), grid, dim3(256), 0, st, insts, static_cast<float*>(f), mode); break;
        default: hipLaunchKernelGGL((ghost_kernel<float, double>), grid, dim3(256), 0, st, insts, static_cast<float*>(f), mode); break;
    }
    return hipGetLastError();
}

// walls: the kernel writes the reflecting-wall ghosts of its output (see
// step_block); otherwise the caller refills them before each step.
hipError_t k_step(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                  void* fout, unsigned* health, int grid, bool nt, bool walls, hipStream_t st) {
    switch (prec) {
        case 0: return launch_step<double, double, false>(insts, items, nitems, fin, fout, health, grid, nt, walls, st);
        case 1: return launch_step<float, float, true>(insts, items, nitems, fin, fout, health, grid, nt, walls, st);
        default: return launch_step<float, double, false>(insts, items, nitems, fin, fout, health, grid, nt, walls, st);
    }
}

// Two steps from fin to fout (bands of at most kBand2 rows); the
// reflecting-wall ghosts of fin must be current.  wrap4:
// some item is a band that is a whole periodic height of four rows.
hipError_t k_step2(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                   void* fout, unsigned* health, int grid, bool nt, bool wrap4, hipStream_t st) {
    switch (prec) {
        case 0: return launch_step2<double, double, false>(insts, items, nitems, fin, fout, health, grid, nt, wrap4, st);
        case 1: return launch_step2<float, float, true>(insts, items, nitems, fin, fout, health, grid, nt, wrap4, st);
        case 2: return launch_step2<float, double, false>(insts, items, nitems, fin, fout, health, grid, nt, wrap4, st);
        default: return hipErrorInvalidValue;
    }
}

// kTubeSteps steps of tubes of ny = 1, 2 or 4 periodic rows (every
// instance of the launch) with fixed-equilibrium x sides, from fin to fout.
hipError_t k_tube(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                  void* fout, unsigned* health, int grid, bool nt, int ny, hipStream_t st) {
    switch (prec) {
        case 0: return launch_tube<double, double, false>(insts, items, nitems, fin, fout, health, grid, nt, ny, st);
        case 1: return launch_tube<float, float, true>(insts, items, nitems, fin, fout, health, grid, nt, ny, st);
        case 2: return launch_tube<float, double, false>(insts, items, nitems, fin, fout, health, grid, nt, ny, st);
        default: return hipErrorInvalidValue;
    }
}

// Variant step (scheme flags as in mrtlb.h: bit 0 collide-then-stream, bit 1
// nine-point Lax-Wendroff) from fin to fout; `tmp` holds the post-collision
// populations of the split form, whose reflecting ghosts are refilled
// between the two passes.
template <typename S, typename C, bool COMP>
hipError_t launch_variant(const Inst* P, int nx, int ny, int scheme, bool reflect, const void* fin,
                          void* fout, void* tmp, unsigned* health, hipStream_t st) {
    const dim3 grid((nx + 255) / 256, ny < 65535 ? ny : 65535);
    const S* in = static_cast<const S*>(fin);
    S* out = static_cast<S*>(fout);
    const bool split = scheme & 1, cross = scheme & 2;
    if (split) {
        S* h = static_cast<S*>(tmp);
        hipLaunchKernelGGL((collide_kernel<S, C, COMP>), grid, dim3(256), 0, st, P, in, h, health);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (reflect) {
            hipLaunchKernelGGL((ghost_kernel<S, C>), dim3((2 * (nx + ny) + 4 + 255) / 256, 1), dim3(256), 0, st,
                               P, h, 1);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (cross)
            hipLaunchKernelGGL((cell_step_kernel<S, C, COMP, false, true>), grid, dim3(256), 0, st, P, h, out, health);
        else
            hipLaunchKernelGGL((cell_step_kernel<S, C, COMP, false, false>), grid, dim3(256), 0, st, P, h, out, health);
    } else {
        hipLaunchKernelGGL((cell_step_kernel<S, C, COMP, true, true>), grid, dim3(256), 0, st, P, in, out, health);
    }
    return hipGetLastError();
}

hipError_t k_variant(int prec, const Inst* P, int nx, int ny, int scheme, bool reflect,
                     const void* fin, void* fout, void* tmp, unsigned* health, hipStream_t st) {
    switch (prec) {
        case 0: return launch_variant<double, double, false>(P, nx, ny, scheme, reflect, fin, fout, tmp, health, st);
        case 1: return launch_variant<float, float, true>(P, nx, ny, scheme, reflect, fin, fout, tmp, health, st);
        default: return launch_variant<float, double, false>(P, nx, ny, scheme, reflect, fin, fout, tmp, health, st);
    }
}

// One adjoint step; partial rows (one per item) are overwritten
// (accumulate = false) or added to (true); ds != NULL: then reduce the
// partial rows into ds (partial must hold nitems + kStageBlocks rows of 16
// doubles).  nt: non-temporal stores of lam^n.
template <typename S, typename C>
void launch_adjoint(const Inst* insts, const Item* items, int nitems, const void* lin,
                    const void* fn, void* lout, double* partial, int acc, bool nt, hipStream_t st) {
    const int blocks = 8 * ((nitems + 7) / 8);
    if (nt)
        hipLaunchKernelGGL((adjoint_kernel<S, C, true>), dim3(blocks), dim3(256), 0, st, insts, items,
                           nitems, static_cast<const S*>(lin), static_cast<const S*>(fn),
                           static_cast<S*>(lout), partial, acc);
    else
        hipLaunchKernelGGL((adjoint_kernel<S, C, false>), dim3(blocks), dim3(256), 0, st, insts, items,
                           nitems, static_cast<const S*>(lin), static_cast<const S*>(fn),
                           static_cast<S*>(lout), partial, acc);
}

hipError_t k_adjoint(int prec, const Inst* insts, const Item* items, int nitems, const void* lin,
                     const void* fn, void* lout, double* partial, bool accumulate, double* ds,
                     bool nt, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int acc = accumulate ? 1 : 0;
    switch (prec) {
        case 0: launch_adjoint<double, double>(insts, items, nitems, lin, fn, lout, partial, acc, nt, st); break;
        case 1: launch_adjoint<float, float>(insts, items, nitems, lin, fn, lout, partial, acc, nt, st); break;
        default: launch_adjoint<float, double>(insts, items, nitems, lin, fn, lout, partial, acc, nt, st); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ds) return e;
    // a few rows: one block sums them (one launch; small grids are
    // latency-bound); else two stages.  partial holds nitems rows, then
    // kStageBlocks rows of stage sums
    if (nitems <= kSingleStageRows) {
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kReduceThreads), 0, st, partial, nitems, ds);
        return hipGetLastError();
    }
    double* stage = partial + (long long)nitems * 16;
    const int per = (nitems + kStageBlocks - 1) / kStageBlocks;
    const int blocks = (nitems + per - 1) / per;
    hipLaunchKernelGGL(reduce_stripes, dim3(blocks), dim3(256), 0, st, partial, nitems, per, stage);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kReduceThreads), 0, st, stage, blocks, ds);
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
