// mrt_internal.h -- data shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mrt_transform.h"

namespace mrt {

enum { XLO = 0, XHI = 1, YLO = 2, YHI = 3 };
enum { BC_PERIODIC = 0, BC_EQ = 1, BC_OUTFLOW = 2, BC_REFLECT = 3 };

// One grid (instance) as the kernels see it.  Read by every lane of a wave
// at the same address, so it lives in scalar registers / the scalar cache.
struct Inst {
    long long off;      // element offset of the instance in the buffers
    long long plane;    // elements between populations (the sub-row length:
                        // a multiple of 256, >= nx + 3)
    int nx, ny, pitch;  // pitch: elements between grid rows (16 sub-rows + padding)
    int origin;         // population i of cell (x, y) is at
                        // off + i * plane + origin + y * pitch + x for
                        // -1 <= x <= nx, -1 <= y <= ny (x or y outside [0, n):
                        // the ghost ring; column nx + 1 is never read)
    // Where a neighbour outside the grid is read from: column col_lo for
    // x = -1 and col_hi for x >= nx, row row_lo for y = -1 and row_hi for
    // y = ny.  Periodic sides point at the wrapped cell, outflow sides at the
    // adjacent cell, fixed-equilibrium and reflecting sides at the ghost ring.
    int col_lo, col_hi, row_lo, row_hi;
    int item0;          // first work item of this instance (partial-sum rows)
    int pad0;
    int bc[4];
    double b;           // dof: gamma = (b + 2)/b
    double binv;        // 1/b
    double dt;
    double sdt[16];     // s_k dt; entries 0..3 unused (collision invariants)
    // Lax-Wendroff weights per axis (0: x, 1: y) and shell for a velocity
    // component +c, c = |v_a| dt / dx_a >= 0:
    //   [0] c^2/2 - c/2  weight of the downstream neighbour (x + 1)
    //   [1] c^2/2 + c/2  weight of the upstream neighbour (x - 1)
    // (for a component -c the two swap); they sum to c^2.
    double lw[2][4][2];
    float lwf[2][4][2];
    // mixed-derivative weight of the nine-point stencil per shell:
    // |c_x c_y| / 4 (zero on the axis shells)
    double lwc[4];
    float lwcf[4];
    // lw[a][k][0] + lw[a][k][1] (c^2), summed in each precision exactly as a
    // kernel would sum the two weights it reads
    double lws[2][4];
    float lwsf[2][4];
    double ghost[4][16];   // f^eq of each MRT_BC_EQ side
};

// Work item of the step kernel: one block of 4 waves advances 256 columns
// [x0, x0 + 256) of rows [y0, y1) of instance `inst`; the adjoint kernel
// splits the same item into four 64-column waves.
struct Item {
    int inst, x0, y0, y1;
};

// velocity component signs per population: +1, -1 or 0
MRT_HD int sgn_x(int i) {
    const int r = i & 3;
    if (i < 8) return r == 0 ? 1 : (r == 2 ? -1 : 0);
    return (r == 0 || r == 3) ? 1 : -1;
}
MRT_HD int sgn_y(int i) {
    const int r = i & 3;
    if (i < 8) return r == 1 ? 1 : (r == 3 ? -1 : 0);
    return (r == 0 || r == 1) ? 1 : -1;
}

}  // namespace mrt
