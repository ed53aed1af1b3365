// mrt_api.hip -- host side of the C ABI declared in include/mrtlb.h.
//
// Owns contexts and batches: parameter validation, population buffers, the
// per-instance constant block (Inst) and the work-item table read by the
// step kernel, the health flag, the tile autotuner and the captured HIP
// graphs of the batched form.  All compute is in mrt_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "mrt_dual.h"
#include "mrt_internal.h"
#include "mrt_tube.h"
#include "../../include/mrtlb.h"

namespace mrt {
hipError_t k_ghost(int prec, const Inst* insts, int count, int perim, void* f, int mode,
                   hipStream_t st);
hipError_t k_step(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                  void* fout, unsigned* health, int grid, bool nt, bool walls, hipStream_t st);
hipError_t k_step2(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                   void* fout, unsigned* health, int grid, bool nt, bool wrap4, hipStream_t st);
hipError_t k_tube(int prec, const Inst* insts, const Item* items, int nitems, const void* fin,
                  void* fout, unsigned* health, int grid, bool nt, int ny, hipStream_t st);
hipError_t k_variant(int prec, const Inst* P, int nx, int ny, int scheme, bool reflect,
                     const void* fin, void* fout, void* tmp, unsigned* health, hipStream_t st);
hipError_t k_adjoint(int prec, const Inst* insts, const Item* items, int nitems, const void* lin,
                     const void* fn, void* lout, double* partial, bool accumulate, double* ds,
                     bool nt, hipStream_t st);
hipError_t k_init(int prec, const Inst* P, long long cells, const double* rho, const double* ux,
                  const double* uy, const double* T, void* f, hipStream_t st);
hipError_t k_moments(int prec, const Inst* P, long long cells, const void* f, double* rho,
                     double* ux, double* uy, double* T, unsigned* health, hipStream_t st);
hipError_t k_density(int prec, const Inst* P, long long cells, const void* f, double* rho,
                     hipStream_t st);
hipError_t k_density_adjoint(int prec, const Inst* P, long long cells, const double* g_rho,
                             void* lam, hipStream_t st);
hipError_t k_init_adjoint(int prec, const Inst* P, long long cells, const void* lam,
                          const double* rho, const double* ux, const double* uy, const double* T,
                          double* g_rho, double* g_ux, double* g_uy, double* g_T, hipStream_t st);
hipError_t k_export(int prec, const Inst* P, long long cells, const void* f, double* out,
                    hipStream_t st);
hipError_t k_import(int prec, const Inst* P, long long cells, const double* in, void* f,
                    hipStream_t st);
}  // namespace mrt

using mrt::Inst;
using mrt::Item;
using mrt::kTubeSteps;
using mrt::kTubeWidth;

// Scratch of mrt_adjoint_step_noalloc: the rate-gradient partial rows of one
// adjoint step (one row of 16 doubles per work item, then the reduction's 64
// stage rows), in a fixed device array instead of a library allocation, so
// that the call allocates nothing.  1 MiB: grids of up to 8128 adjoint work
// items.  Each device holds its own copy until the process ends; host code
// uses only the per-device address resolved by scratch_address(), never the
// array's name.
constexpr int kScratchDoubles = 1 << 17;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per
// device (hipGetSymbolAddress with that device current); nullptr on error.
double* scratch_address(std::string& err) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        err = "no current HIP device (or device index >= 64) for the static scratch";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

namespace {

size_t elem_size(int prec) { return prec == MRT_FP64 ? 8 : 4; }

// Population layout: grid row j (-1..ny, the ghost rows included) is 16
// consecutive sub-rows, one per population, each `sub` elements long (sub a
// multiple of 256 >= nx + 3, so every sub-row starts 256-byte aligned, the
// ghost columns x = -1 / x = nx and the never-read column nx + 1 fit in its
// padding, and a 256-column work item never leaves it), followed by 256
// elements of padding.  Population i of cell (x, j) is at
// origin + j * pitch + i * plane + x with plane = sub and pitch = 16 sub + 256;
// 64 elements precede the first sub-row.  A block marching up a band then
// streams one contiguous 16-sub-row stretch per grid row, which the memory
// system serves faster than 16 streams a plane apart.  The padding makes the
// row stride an odd multiple of 1 KiB (FP32; 2 KiB FP64): with a stride of
// 2^14 times an integer, bands of 8 or 16 rows start at addresses that
// concentrate on a few memory channels (measured 10 % slower on 4096^2).
constexpr long long kRowPad = 256;
long long sub_for(int nx) { return ((long long)nx + 3 + 255) / 256 * 256; }
long long pitch_for(int nx) { return 16 * sub_for(nx) + kRowPad; }
long long plane_for(int nx) { return sub_for(nx); }
long long origin_for(int nx) { return pitch_for(nx) + 64; }
long long elems_for(int nx, int ny) { return (long long)(ny + 2) * pitch_for(nx) + 512; }

// The kernels index an instance with 32-bit element offsets (their row
// offsets and columns are unsigned 32-bit sums): an instance must stay below
// 2^32 elements (FP32 storage: 16 GiB per state, e.g. 16000 x 16000 cells).
bool size_ok(int nx, int ny) {
    return nx >= 1 && ny >= 1 && elems_for(nx, ny) < (1LL << 32);
}

bool bc_ok(const int bc[4]) {
    for (int k = 0; k < 4; ++k)
        if (bc[k] < MRT_BC_PERIODIC || bc[k] > MRT_BC_REFLECT) return false;
    if ((bc[0] == MRT_BC_PERIODIC) != (bc[1] == MRT_BC_PERIODIC)) return false;
    if ((bc[2] == MRT_BC_PERIODIC) != (bc[3] == MRT_BC_PERIODIC)) return false;
    return true;
}

// Validate parameters and fill the scheme constants of an instance.
int fill_inst(Inst& I, int nx, int ny, const int bc[4], const mrt_params* p, std::string& err) {
    if (!p) { err = "params is NULL"; return MRT_EINVAL; }
    if (!(p->gamma > 1.0 && p->gamma <= 2.0)) { err = "gamma must lie in (1, 2]"; return MRT_EINVAL; }
    if (!(p->dt > 0 && p->dx > 0 && p->dy > 0)) { err = "dt, dx, dy must be > 0"; return MRT_EINVAL; }
    if (!(p->eta0 == 0.0 || p->eta0 == 2.5)) { err = "eta0 must be 5/2 (0 selects it)"; return MRT_EINVAL; }
    double s[16];
    for (int k = 0; k < 16; ++k) s[k] = p->s[k];
    if (p->Pr > 0) {
        if (std::fabs(s[6] - s[5]) > 1e-12 * std::max(1.0, std::fabs(s[5]))) {
            err = "Pr > 0 needs s_7 == s_6";
            return MRT_EINVAL;
        }
        s[7] = s[8] = p->Pr * s[5];
    } else if (p->Pr < 0) {
        err = "Pr must be >= 0";
        return MRT_EINVAL;
    }
    for (int k = 4; k < 16; ++k) {
        const double sd = s[k] * p->dt;
        // [0, 1/dt] (text after Eq. 12d), with 1e-6 of slack for rates set to
        // exactly 1/dt and then perturbed (finite-difference checks)
        if (!(sd >= 0.0 && sd <= 1.0 + 1e-6)) {
            char buf[96];
            std::snprintf(buf, sizeof buf, "s_%d * dt = %g outside [0, 1]", k + 1, sd);
            err = buf;
            return MRT_EINVAL;
        }
    }
    I.b = 2.0 / (p->gamma - 1.0);
    I.binv = 1.0 / I.b;
    I.dt = p->dt;
    for (int k = 0; k < 16; ++k) I.sdt[k] = k < 4 ? 0.0 : s[k] * p->dt;
    const double h[2] = {p->dx, p->dy};
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 4; ++k) {
            const double c = mrt::shell_speed(k) * p->dt / h[a];
            I.lw[a][k][0] = 0.5 * c * c - 0.5 * c;
            I.lw[a][k][1] = 0.5 * c * c + 0.5 * c;
            I.lwf[a][k][0] = float(I.lw[a][k][0]);
            I.lwf[a][k][1] = float(I.lw[a][k][1]);
            I.lws[a][k] = I.lw[a][k][0] + I.lw[a][k][1];
            I.lwsf[a][k] = I.lwf[a][k][0] + I.lwf[a][k][1];
        }
    for (int k = 0; k < 4; ++k) {
        // diagonal shells: |v_x| = |v_y| = shell_speed(k)
        const double v = mrt::shell_speed(k);
        I.lwc[k] = k < 2 ? 0.0 : 0.25 * (v * p->dt / p->dx) * (v * p->dt / p->dy);
        I.lwcf[k] = float(I.lwc[k]);
    }
    for (int side = 0; side < 4; ++side) {
        I.bc[side] = bc[side];
        for (int i = 0; i < 16; ++i) I.ghost[side][i] = 0.0;
        if (bc[side] == MRT_BC_EQ) {
            const double* st = p->side_state[side];
            if (!(st[0] > 0 && st[3] > 0)) { err = "EQ side state needs rho > 0 and T > 0"; return MRT_EINVAL; }
            mrt::equilibrium_pops<double>(st[0], st[1], st[2], st[3], I.b, I.ghost[side]);
        }
    }
    // where out-of-grid neighbours are read (see Inst)
    auto lo = [](int kind, int n) { return kind == MRT_BC_PERIODIC ? n - 1 : (kind == MRT_BC_OUTFLOW ? 0 : -1); };
    auto hi = [](int kind, int n) { return kind == MRT_BC_PERIODIC ? 0 : (kind == MRT_BC_OUTFLOW ? n - 1 : n); };
    I.col_lo = lo(bc[0], nx);
    I.col_hi = hi(bc[1], nx);
    I.row_lo = lo(bc[2], ny);
    I.row_hi = hi(bc[3], ny);
    return MRT_OK;
}

bool has_kind(const int bc[4], int kind) {
    for (int k = 0; k < 4; ++k)
        if (bc[k] == kind) return true;
    return false;
}

// Captured step launches.  A graph of `steps` steps that starts from buffer
// `start` (0 or 1) replays the same launches on the same buffers, so n steps
// run as n / kGraphChunk replays of one kGraphChunk-step graph (an even
// count: each replay ends on the buffer it started from) and one graph of
// the n % kGraphChunk remaining steps; graphs are captured on first use and
// kept until the launch configuration changes.
constexpr int kGraphChunk = 64;

struct GraphCache {
    std::map<int, hipGraphExec_t> g;   // key: 2 * steps + start buffer
    void clear() {
        for (auto& kv : g) (void)hipGraphExecDestroy(kv.second);
        g.clear();
    }
};

// enqueue(cur, stream) launches one step reading buffer cur.  launch =
// false only captures the graphs n steps need (nothing runs, cur is kept).
template <typename Enqueue>
hipError_t run_graphs(GraphCache& cache, int& cur, int n, hipStream_t stream, Enqueue enqueue,
                      bool launch = true) {
    auto get = [&](int steps, int start, hipGraphExec_t* out) -> hipError_t {
        const int key = 2 * steps + start;
        auto it = cache.g.find(key);
        if (it != cache.g.end()) {
            *out = it->second;
            return hipSuccess;
        }
        hipStream_t cap = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return e;
        }
        int c = start;
        for (int k = 0; k < steps && e == hipSuccess; ++k) {
            if constexpr (std::is_invocable_v<Enqueue, int, hipStream_t, int>)
                e = enqueue(c, cap, k);
            else
                e = enqueue(c, cap);
            c ^= 1;
        }
        hipGraph_t graph = nullptr;
        const hipError_t e_end = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e_end;
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        // when only preparing (mrt_prepare_steps), upload the executable
        // graph to the device now, so that its first replay (inside a
        // caller's timed region or latency-critical loop) does not carry the
        // one-time upload; a graph made by a launching call is uploaded by
        // its launch (which also works while the caller captures the stream)
        if (e == hipSuccess && !launch) e = hipGraphUpload(exec, stream);
        if (e != hipSuccess) {
            if (exec) (void)hipGraphExecDestroy(exec);
            return e;
        }
        cache.g.emplace(key, exec);
        *out = exec;
        return hipSuccess;
    };
    hipGraphExec_t exec = nullptr;
    for (int q = 0; q < n / kGraphChunk; ++q) {
        hipError_t e = get(kGraphChunk, cur, &exec);
        if (e == hipSuccess && launch) e = hipGraphLaunch(exec, stream);
        if (e != hipSuccess) return e;
        if (!launch) break;      // every replay uses the same graph
    }
    const int r = n % kGraphChunk;
    if (r) {
        hipError_t e = get(r, cur, &exec);
        if (e == hipSuccess && launch) e = hipGraphLaunch(exec, stream);
        if (e != hipSuccess) return e;
        if (launch && (r & 1)) cur ^= 1;
    }
    return hipSuccess;
}

// Work items of one instance: 256-column chunks x ceil(ny / rows) bands of
// nearly equal height (at most `rows` rows, heights differ by at most 1).
void add_items(std::vector<Item>& items, int inst, int nx, int ny, int rows) {
    const long long nb = (ny + rows - 1) / rows;
    for (long long k = 0; k < nb; ++k) {
        const int y0 = int(k * ny / nb), y1 = int((k + 1) * ny / nb);
        for (int x0 = 0; x0 < nx; x0 += 256) items.push_back(Item{inst, x0, y0, y1});
    }
}

// Short bands (at most 6 rows) and many blocks: the step streams best with
// ~8-16k blocks of short marches (measured on the 4096^2 grid); small grids
// go down to one-row bands so that they still spread over the chip.
//
// The two-step kernel's blocks stay resident together: kTwoStepSlots[fp64]
// of them fill the chip (two per CU in FP32 storage, one in FP64).  A
// launch takes ceil(items / slots) rounds of blocks, and a block's time
// grows with the rows it stores plus about five rows' worth of fixed work
// (the two recomputed f^{n+1} halo rows and the halo-column prologue).
constexpr long long kTwoStepSlots[2] = {512, 256};
constexpr long long kTwoStepFixedRows = 5;

long long two_step_items(int nx, int ny, int rows) {
    return (long long)((nx + 255) / 256) * ((ny + rows - 1) / rows);
}

// Default band height of the two-step kernel: among 8, 16, 32 (and 64 in
// FP64 storage) rows, the one with the fewest rounds x (rows + 5) that
// still fills at least one round (8 rows when none does).  Measured on
// 2D Riemann grids and the shock-bubble grid, in both storage precisions:
// 1024^2 picks 8 / 16 rows (FP32 / FP64), 1536^2 8 / 16, 2048^2 32 / 64,
// 4096^2 32 / 64, each the fastest or within 7 % of it.
int default_rows2(int nx, int ny, int prec) {
    const bool fp64 = prec == MRT_FP64;
    const long long slots = kTwoStepSlots[fp64 ? 1 : 0];
    int best = 8;
    long long best_cost = -1;
    for (int r : {8, 16, 32, 64}) {
        if (r == 64 && !fp64) break;
        if (r > ny && r != 8) break;
        const long long items = two_step_items(nx, ny, r);
        if (items < slots && r != 8) continue;
        const long long cost = (items + slots - 1) / slots * (r + kTwoStepFixedRows);
        if (best_cost < 0 || cost < best_cost) {
            best = r;
            best_cost = cost;
        }
    }
    return std::min(best, ny);
}

// Whether a grid runs two steps per pass by default: larger than the
// last-level cache, or giving at least one full round of 8-row bands (from
// about 1024^2 on: there two steps per pass measured 1.2-1.9 x one, while
// 768^2 and smaller ran faster with one).
bool two_step_default(int nx, int ny, bool beyond_cache) {
    return beyond_cache || two_step_items(nx, ny, 8) >= kTwoStepSlots[0];
}

// Band height of the batch's two-step kernel when none is given.
constexpr int kBatchRows2 = 32;

int default_rows(int nx, int ny) {
    const long long chunks = (nx + 255) / 256;
    long long r = (chunks * ny + 8191) / 8192;
    r = std::max<long long>(1, std::min<long long>(r, 6));
    return int(std::min<long long>(r, ny));
}

}  // namespace

#define HIPTRY(call)                                                           \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            ctx_err = std::string(#call) + ": " + hipGetErrorString(e_);       \
            return MRT_EDEVICE;                                                \
        }                                                                      \
    } while (0)

struct mrt_ctx {
    int nx = 0, ny = 0, prec = 0;
    int bc[4] = {0, 0, 0, 0};
    hipStream_t stream = nullptr;
    void* f[2] = {nullptr, nullptr};
    bool own_f = false;
    int cur = 0;
    long long pitch = 0, plane = 0, origin = 0;
    Inst inst{};
    Inst* d_inst = nullptr;
    Item* d_items = nullptr;
    int nitems = 0, rows = 0, grid = 0;
    bool nt = false;                 // non-temporal population stores (large grids)
    bool walls = false;              // the step kernel writes the reflecting-wall ghosts
    GraphCache graphs;               // captured steps of mrt_step
    int per_pass = 1;                // time steps per pass of the marching kernel (1 or 2)
    Item* d_items2 = nullptr;        // work items of the two-step kernel
    int nitems2 = 0, rows2 = 0;
    bool wrap4 = false;              // a two-step band is a whole periodic height of 4 rows
    GraphCache graphs2;              // captured two-step passes
    Item* d_items4 = nullptr;        // work items of the tube march
    int nitems4 = 0;
    GraphCache graphs4;              // captured tube-march passes
    bool eager = false;              // launch step by step (the tile autotuner)
    int scheme = 0;                  // MRT_SCHEME_* flags
    void* f_tmp = nullptr;           // post-collision state of the split scheme
    Item* d_items_adj = nullptr;     // work items of the adjoint kernel
    int nitems_adj = 0;
    double* d_stage = nullptr;       // 4 * nx * ny doubles: field staging
    double* d_partial = nullptr;     // rate-gradient partial sums: 16 doubles per adjoint item,
                                     // then 64 rows for the reduction's first stage
    double* d_scratch = nullptr;     // the static scratch on this context's device
    std::string scratch_err;         // why d_scratch could not be resolved
    unsigned* d_health = nullptr;
    // second stream of the adjoint sweep (recomputation of the next segment
    // beside the adjoint steps of the current one) and its events, made on
    // first use
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
    bool params_set = false, fields_set = false;
    std::string err;
};

namespace {

int ctx_fail(mrt_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

// Ghost ring after the state was set from outside a step: the equilibrium
// ghosts of MRT_BC_EQ sides into every population buffer (no step overwrites
// them) and the reflecting-wall ghosts of the current state (from then on
// each step kernel writes those of its own output).
int fill_ghosts(mrt_ctx* c) {
    std::string& ctx_err = c->err;
    const int perim = 2 * (c->nx + c->ny);
    if (has_kind(c->bc, MRT_BC_EQ)) {
        for (int k = 0; k < 2; ++k) HIPTRY(mrt::k_ghost(c->prec, c->d_inst, 1, perim, c->f[k], 2, c->stream));
        if (c->f_tmp) HIPTRY(mrt::k_ghost(c->prec, c->d_inst, 1, perim, c->f_tmp, 2, c->stream));
    }
    if (has_kind(c->bc, MRT_BC_REFLECT))
        HIPTRY(mrt::k_ghost(c->prec, c->d_inst, 1, perim, c->f[c->cur], 1, c->stream));
    return MRT_OK;
}

int build_items(mrt_ctx* c, int rows) {
    std::string& ctx_err = c->err;
    std::vector<Item> items;
    add_items(items, 0, c->nx, c->ny, rows);
    if (c->d_items) HIPTRY(hipFree(c->d_items));
    c->d_items = nullptr;
    HIPTRY(hipMalloc(&c->d_items, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(c->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    c->nitems = int(items.size());
    c->rows = rows;
    c->graphs.clear();
    return MRT_OK;
}

// Work items of the two-step kernel: bands of `rows` <= 32 rows.
// Whether the two-step bands of an instance with band height `rows` are a
// whole periodic height of four rows (the march then reuses f^{n+1} of the
// wrapped rows; mrt_kernels.hip, step2_block).
bool wraps_four_rows(const Inst& I, int rows) {
    return I.ny == 4 && rows >= 4 && I.bc[2] == MRT_BC_PERIODIC && I.bc[3] == MRT_BC_PERIODIC;
}

int build_items2(mrt_ctx* c, int rows) {
    std::string& ctx_err = c->err;
    std::vector<Item> items;
    add_items(items, 0, c->nx, c->ny, rows);
    if (c->d_items2) HIPTRY(hipFree(c->d_items2));
    c->d_items2 = nullptr;
    HIPTRY(hipMalloc(&c->d_items2, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(c->d_items2, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    c->nitems2 = int(items.size());
    c->rows2 = rows;
    c->wrap4 = wraps_four_rows(c->inst, rows);
    c->graphs2.clear();
    return MRT_OK;
}

// Whether the tube march (kTubeSteps steps per pass, mrt_kernels.hip) can
// advance an instance: 1, 2 or 4 periodic rows, fixed-equilibrium x sides.
bool tube_inst_ok(const Inst& I) {
    return (I.ny == 1 || I.ny == 2 || I.ny == 4) && I.bc[2] == MRT_BC_PERIODIC &&
           I.bc[3] == MRT_BC_PERIODIC && I.bc[0] == MRT_BC_EQ && I.bc[1] == MRT_BC_EQ;
}

// Tube-march work items of an instance: kTubeWidth-column chunks.
void add_tube_items(std::vector<Item>& items, int inst, int nx, int ny) {
    for (int x0 = 0; x0 < nx; x0 += kTubeWidth) items.push_back(Item{inst, x0, 0, ny});
}

int build_items4(mrt_ctx* c) {
    std::string& ctx_err = c->err;
    std::vector<Item> items;
    add_tube_items(items, 0, c->nx, c->ny);
    if (c->d_items4) HIPTRY(hipFree(c->d_items4));
    c->d_items4 = nullptr;
    HIPTRY(hipMalloc(&c->d_items4, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(c->d_items4, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    c->nitems4 = int(items.size());
    c->graphs4.clear();
    return MRT_OK;
}

// Work items of the adjoint kernel: 256-column chunks of row bands, marched
// like the one-step kernel's.  Bands of up to 16 rows while the grid still
// gives ~2048 items (four blocks per block slot of the chip at two 4-wave
// blocks per CU), down to one row on small grids so that they still spread
// over the chip.
int adjoint_rows(int nx, int ny) {
    const long long chunks = (nx + 255) / 256;
    const long long r = std::max<long long>(1, std::min<long long>(16, chunks * ny / 2048));
    return int(std::min<long long>(r, ny));
}

int build_adjoint_items(mrt_ctx* c) {
    std::string& ctx_err = c->err;
    std::vector<Item> items;
    add_items(items, 0, c->nx, c->ny, adjoint_rows(c->nx, c->ny));
    HIPTRY(hipMalloc(&c->d_items_adj, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(c->d_items_adj, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    // one partial row per item, then the reduction's 64 stage rows
    HIPTRY(hipMalloc(&c->d_partial, (items.size() + 64) * 16 * sizeof(double)));
    c->nitems_adj = int(items.size());
    return MRT_OK;
}

// Stores bypass the caches (non-temporal) once one population buffer is
// larger than the 256 MB last-level cache: nothing of the new state can stay
// cached until the next step anyway.  Smaller grids keep it cached.
constexpr long long kNonTemporalBytes = 256LL << 20;

// Grids with reflecting walls up to this many cells have the step kernel
// write the wall ghosts of its output (one launch per step instead of two:
// the launch latency dominates there); larger ones refill them with the
// ghost kernel, which costs them less than the extra registers would.
constexpr long long kWallsInKernelCells = 1LL << 22;

int check_health(mrt_ctx* c) {
    std::string& ctx_err = c->err;
    unsigned h = 0;
    HIPTRY(hipMemcpyAsync(&h, c->d_health, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(hipStreamSynchronize(c->stream));
    if (h) {
        HIPTRY(hipMemsetAsync(c->d_health, 0, sizeof(unsigned), c->stream));
        HIPTRY(hipStreamSynchronize(c->stream));
        c->err = "non-finite value, rho <= 0 or T <= 0 detected";
        return MRT_EUNSTABLE;
    }
    return MRT_OK;
}

}  // namespace

extern "C" {

long long mrt_population_bytes(int nx, int ny, int precision) {
    if (!size_ok(nx, ny)) return 0;
    return elems_for(nx, ny) * (long long)elem_size(precision);
}

int mrt_init_grid(mrt_ctx** out, int nx, int ny, int precision, const int bc[4],
                  void* const f_dev[2], void* stream) {
    if (!out) return MRT_EINVAL;
    *out = nullptr;
    if (!size_ok(nx, ny) || precision < 0 || precision > 2 || !bc || !bc_ok(bc)) return MRT_EINVAL;
    mrt_ctx* c = new mrt_ctx();
    std::string& ctx_err = c->err;
    c->nx = nx;
    c->ny = ny;
    c->prec = precision;
    for (int k = 0; k < 4; ++k) c->bc[k] = bc[k];
    c->stream = static_cast<hipStream_t>(stream);
    c->pitch = pitch_for(nx);
    c->plane = plane_for(nx);
    c->origin = origin_for(nx);
    const size_t bytes = size_t(mrt_population_bytes(nx, ny, precision));
    auto fail = [&](int code) {
        mrt_destroy(c);
        return code;
    };
    if (f_dev && f_dev[0] && f_dev[1]) {
        c->f[0] = f_dev[0];
        c->f[1] = f_dev[1];
        c->own_f = false;
    } else {
        if (hipMalloc(&c->f[0], bytes) != hipSuccess || hipMalloc(&c->f[1], bytes) != hipSuccess)
            return fail(MRT_ENOMEM);
        c->own_f = true;
    }
    if (hipMalloc(&c->d_inst, sizeof(Inst)) != hipSuccess ||
        hipMalloc(&c->d_health, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&c->d_stage, 4 * sizeof(double) * size_t(nx) * ny) != hipSuccess)
        return fail(MRT_ENOMEM);
    if (hipMemset(c->d_health, 0, sizeof(unsigned)) != hipSuccess) return fail(MRT_EDEVICE);
    // zero both buffers: pitch padding and the plane gaps are never read, but
    // keep them defined
    if (hipMemset(c->f[0], 0, bytes) != hipSuccess || hipMemset(c->f[1], 0, bytes) != hipSuccess)
        return fail(MRT_EDEVICE);
    c->inst.off = 0;
    c->inst.plane = c->plane;
    c->inst.nx = nx;
    c->inst.ny = ny;
    c->inst.pitch = int(c->pitch);
    c->inst.origin = int(c->origin);
    c->inst.item0 = 0;
    for (int k = 0; k < 4; ++k) c->inst.bc[k] = bc[k];
    if (build_items(c, default_rows(nx, ny)) != MRT_OK) return fail(MRT_EDEVICE);
    if (build_adjoint_items(c) != MRT_OK) return fail(MRT_EDEVICE);
    // address of the static scratch on this device (mrt_adjoint_step_noalloc;
    // a failure here is reported by that call, the others do not need it)
    c->d_scratch = scratch_address(c->scratch_err);
    c->nt = (long long)bytes > kNonTemporalBytes;
    c->walls = has_kind(bc, MRT_BC_REFLECT) && (long long)nx * ny <= kWallsInKernelCells;
    // grids larger than the last-level cache (HBM-bound with one step per
    // pass: 4096^2 FP32 storage 0.65 -> 0.96, FP64 0.68 -> 0.93 of the
    // per-step roofline with two) and cache-resident ones from about 1024^2
    // on run two steps per pass by default
    if (two_step_default(nx, ny, c->nt)) {
        if (build_items2(c, default_rows2(nx, ny, precision)) != MRT_OK) return fail(MRT_EDEVICE);
        c->per_pass = 2;
    }
    // grids the tube march covers (1, 2 or 4 periodic rows, fixed-equilibrium
    // x sides: the shock tubes) run four steps per pass by default
    if (tube_inst_ok(c->inst)) {
        if (build_items4(c) != MRT_OK) return fail(MRT_EDEVICE);
        c->per_pass = kTubeSteps;
    }
    (void)ctx_err;
    *out = c;
    return MRT_OK;
}

int mrt_get_layout(const mrt_ctx* c, long long* pitch, long long* plane, long long* origin) {
    if (!c) return MRT_EINVAL;
    if (pitch) *pitch = c->pitch;
    if (plane) *plane = c->plane;
    if (origin) *origin = c->origin;
    return MRT_OK;
}

int mrt_set_params(mrt_ctx* c, const mrt_params* p) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    Inst I = c->inst;
    const int rc = fill_inst(I, c->nx, c->ny, c->bc, p, c->err);
    if (rc != MRT_OK) return rc;
    c->inst = I;
    HIPTRY(hipMemcpyAsync(c->d_inst, &c->inst, sizeof(Inst), hipMemcpyHostToDevice, c->stream));
    c->params_set = true;
    if (c->fields_set) {
        const int r = fill_ghosts(c);
        if (r != MRT_OK) return r;
    }
    HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

int mrt_set_fields(mrt_ctx* c, const double* rho, const double* ux, const double* uy,
                   const double* T, int on_device) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    if (!rho || !ux || !uy || !T) return ctx_fail(c, MRT_EINVAL, "NULL field");
    const long long n = (long long)c->nx * c->ny;
    if (on_device) {
        HIPTRY(mrt::k_init(c->prec, c->d_inst, n, rho, ux, uy, T, c->f[c->cur], c->stream));
    } else {
        for (long long k = 0; k < n; ++k)
            if (!(rho[k] > 0 && T[k] > 0)) return ctx_fail(c, MRT_EINVAL, "rho and T must be > 0");
        double* s = c->d_stage;
        const size_t b = sizeof(double) * size_t(n);
        HIPTRY(hipMemcpyAsync(s, rho, b, hipMemcpyHostToDevice, c->stream));
        HIPTRY(hipMemcpyAsync(s + n, ux, b, hipMemcpyHostToDevice, c->stream));
        HIPTRY(hipMemcpyAsync(s + 2 * n, uy, b, hipMemcpyHostToDevice, c->stream));
        HIPTRY(hipMemcpyAsync(s + 3 * n, T, b, hipMemcpyHostToDevice, c->stream));
        HIPTRY(mrt::k_init(c->prec, c->d_inst, n, s, s + n, s + 2 * n, s + 3 * n, c->f[c->cur], c->stream));
    }
    c->fields_set = true;
    const int r = fill_ghosts(c);
    if (r != MRT_OK) return r;
    if (!on_device) HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

static int step_impl(mrt_ctx* c, int n, bool launch);

int mrt_step(mrt_ctx* c, int n) { return step_impl(c, n, true); }

int mrt_prepare_steps(mrt_ctx* c, int n) { return step_impl(c, n, false); }

static int step_impl(mrt_ctx* c, int n, bool launch) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (n < 0) return ctx_fail(c, MRT_EINVAL, "n < 0");
    if (!c->params_set || !c->fields_set) return ctx_fail(c, MRT_ESTATE, "params and fields must be set");
    const int perim = 2 * (c->nx + c->ny);
    const bool reflect = has_kind(c->bc, MRT_BC_REFLECT);
    // one step reading buffer `cur`: reflecting-wall ghosts unless the step
    // kernel wrote them with the previous step's output (c->walls), then the
    // step.  The per-cell nine-point kernel writes none, so its ghosts
    // (corners too) are always refilled (the split scheme refills those of
    // its post-collision state itself)
    if (c->per_pass == kTubeSteps && c->scheme == 0) {
        // the tube march (no reflecting sides), the remaining steps one by one
        auto enqueue4 = [&](int cur, hipStream_t st) -> hipError_t {
            return mrt::k_tube(c->prec, c->d_inst, c->d_items4, c->nitems4, c->f[cur], c->f[1 - cur],
                               c->d_health, 0, c->nt, c->ny, st);
        };
        const int passes = n / kTubeSteps;
        if (c->eager || passes == 1) {
            if (launch)
                for (int k = 0; k < passes; ++k) {
                    HIPTRY(enqueue4(c->cur, c->stream));
                    c->cur ^= 1;
                }
        } else if (passes > 1) {
            HIPTRY(run_graphs(c->graphs4, c->cur, passes, c->stream, enqueue4, launch));
        }
        if (launch)
            for (int k = 0; k < n % kTubeSteps; ++k) {
                HIPTRY(mrt::k_step(c->prec, c->d_inst, c->d_items, c->nitems, c->f[c->cur], c->f[1 - c->cur],
                                   c->d_health, c->grid, c->nt, c->walls, c->stream));
                c->cur ^= 1;
            }
        return MRT_OK;
    }
    if (c->per_pass == 2 && c->scheme == 0) {
        // two steps per pass; an odd last step by the single-step kernel.
        // The two-step kernel writes the reflecting y-wall ghosts of its
        // output, so the ghost pass runs before the first pass of a call or
        // graph only, unless an x side reflects (then before every pass)
        const bool xwall = c->bc[0] == MRT_BC_REFLECT || c->bc[1] == MRT_BC_REFLECT;
        auto enqueue2 = [&](int cur, hipStream_t st, int k) -> hipError_t {
            if (reflect && (k == 0 || xwall)) {
                const hipError_t e = mrt::k_ghost(c->prec, c->d_inst, 1, perim, c->f[cur], 1, st);
                if (e != hipSuccess) return e;
            }
            return mrt::k_step2(c->prec, c->d_inst, c->d_items2, c->nitems2, c->f[cur], c->f[1 - cur],
                                c->d_health, 0, c->nt, c->wrap4, st);
        };
        auto enqueue1 = [&](int cur, hipStream_t st) -> hipError_t {
            if (reflect) {
                const hipError_t e = mrt::k_ghost(c->prec, c->d_inst, 1, perim, c->f[cur], 1, st);
                if (e != hipSuccess) return e;
            }
            return mrt::k_step(c->prec, c->d_inst, c->d_items, c->nitems, c->f[cur], c->f[1 - cur],
                               c->d_health, c->grid, c->nt, false, st);
        };
        const int pairs = n / 2;
        if (c->eager || pairs == 1) {
            // plain launches, one per pass (the autotuner times these)
            if (launch)
                for (int k = 0; k < pairs; ++k) {
                    HIPTRY(enqueue2(c->cur, c->stream, k));
                    c->cur ^= 1;
                }
        } else if (pairs > 1) {
            HIPTRY(run_graphs(c->graphs2, c->cur, pairs, c->stream, enqueue2, launch));
        }
        if ((n & 1) && launch) {
            HIPTRY(enqueue1(c->cur, c->stream));
            c->cur ^= 1;
        }
        return MRT_OK;
    }
    const bool ghost_pass = reflect && (c->scheme == MRT_SCHEME_LW_CROSS || (c->scheme == 0 && !c->walls));
    auto enqueue = [&](int cur, hipStream_t st) -> hipError_t {
        if (ghost_pass) {
            const hipError_t e = mrt::k_ghost(c->prec, c->d_inst, 1, perim, c->f[cur], 1, st);
            if (e != hipSuccess) return e;
        }
        if (c->scheme)
            return mrt::k_variant(c->prec, c->d_inst, c->nx, c->ny, c->scheme, reflect, c->f[cur],
                                  c->f[1 - cur], c->f_tmp, c->d_health, st);
        return mrt::k_step(c->prec, c->d_inst, c->d_items, c->nitems, c->f[cur], c->f[1 - cur],
                           c->d_health, c->grid, c->nt, c->walls, st);
    };
    if (n == 1 || c->eager) {
        if (!launch) return MRT_OK;
        for (int k = 0; k < n; ++k) {
            HIPTRY(enqueue(c->cur, c->stream));
            c->cur ^= 1;
        }
        return MRT_OK;
    }
    HIPTRY(run_graphs(c->graphs, c->cur, n, c->stream, enqueue, launch));
    return MRT_OK;
}

int mrt_step_buffers(mrt_ctx* c, const void* fin, void* fout) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    if (c->scheme) return ctx_fail(c, MRT_EINVAL, "explicit-buffer steps use the default scheme only");
    if (!fin || !fout || fin == fout) return ctx_fail(c, MRT_EINVAL, "need two distinct buffers");
    if (has_kind(c->bc, MRT_BC_EQ) || has_kind(c->bc, MRT_BC_REFLECT))
        HIPTRY(mrt::k_ghost(c->prec, c->d_inst, 1, 2 * (c->nx + c->ny), const_cast<void*>(fin), 3,
                            c->stream));
    HIPTRY(mrt::k_step(c->prec, c->d_inst, c->d_items, c->nitems, fin, fout, c->d_health, c->grid,
                       c->nt, c->walls, c->stream));
    return MRT_OK;
}

int mrt_read_moments(mrt_ctx* c, double* rho, double* ux, double* uy, double* T, int on_device) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set || !c->fields_set) return ctx_fail(c, MRT_ESTATE, "params and fields must be set");
    const long long n = (long long)c->nx * c->ny;
    if (on_device) {
        HIPTRY(mrt::k_moments(c->prec, c->d_inst, n, c->f[c->cur], rho, ux, uy, T, c->d_health, c->stream));
        return MRT_OK;
    }
    double* s = c->d_stage;
    HIPTRY(mrt::k_moments(c->prec, c->d_inst, n, c->f[c->cur], s, s + n, s + 2 * n, s + 3 * n,
                          c->d_health, c->stream));
    const size_t b = sizeof(double) * size_t(n);
    double* outs[4] = {rho, ux, uy, T};
    for (int k = 0; k < 4; ++k)
        if (outs[k]) HIPTRY(hipMemcpyAsync(outs[k], s + k * n, b, hipMemcpyDeviceToHost, c->stream));
    return check_health(c);
}

int mrt_get_populations(mrt_ctx* c, double* f, int on_device) {
    if (!c || !f) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    const long long n = (long long)c->nx * c->ny;
    if (on_device) {
        HIPTRY(mrt::k_export(c->prec, c->d_inst, n, c->f[c->cur], f, c->stream));
        return MRT_OK;
    }
    double* tmp = nullptr;
    HIPTRY(hipMallocAsync((void**)&tmp, sizeof(double) * 16 * size_t(n), c->stream));
    HIPTRY(mrt::k_export(c->prec, c->d_inst, n, c->f[c->cur], tmp, c->stream));
    HIPTRY(hipMemcpyAsync(f, tmp, sizeof(double) * 16 * size_t(n), hipMemcpyDeviceToHost, c->stream));
    HIPTRY(hipFreeAsync(tmp, c->stream));
    HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

int mrt_set_populations(mrt_ctx* c, const double* f, int on_device) {
    if (!c || !f) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    const long long n = (long long)c->nx * c->ny;
    if (on_device) {
        HIPTRY(mrt::k_import(c->prec, c->d_inst, n, f, c->f[c->cur], c->stream));
    } else {
        double* tmp = nullptr;
        HIPTRY(hipMallocAsync((void**)&tmp, sizeof(double) * 16 * size_t(n), c->stream));
        HIPTRY(hipMemcpyAsync(tmp, f, sizeof(double) * 16 * size_t(n), hipMemcpyHostToDevice, c->stream));
        HIPTRY(mrt::k_import(c->prec, c->d_inst, n, tmp, c->f[c->cur], c->stream));
        HIPTRY(hipFreeAsync(tmp, c->stream));
    }
    c->fields_set = true;
    const int r = fill_ghosts(c);
    if (r != MRT_OK) return r;
    if (!on_device) HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

int mrt_current_buffer(mrt_ctx* c, void** cur, void** other) {
    if (!c) return MRT_EINVAL;
    if (cur) *cur = c->f[c->cur];
    if (other) *other = c->f[1 - c->cur];
    return MRT_OK;
}

int mrt_sync(mrt_ctx* c) {
    if (!c) return MRT_EINVAL;
    return check_health(c);
}

int mrt_set_tile(mrt_ctx* c, int rows, int grid) {
    if (!c) return MRT_EINVAL;
    if (rows < 1 || grid < 0) return ctx_fail(c, MRT_EINVAL, "rows >= 1, grid >= 0");
    const int rc = build_items(c, std::min(rows, c->ny));
    if (rc != MRT_OK) return rc;
    c->grid = grid;
    return MRT_OK;
}

int mrt_set_steps_per_pass(mrt_ctx* c, int steps, int rows) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (steps != 1 && steps != 2 && steps != kTubeSteps)
        return ctx_fail(c, MRT_EINVAL, "steps per pass: 1, 2 or 4");
    if (rows < 0 || rows > MRT_MAX_BAND_ROWS_2) return ctx_fail(c, MRT_EINVAL, "rows: 0 (default) to 64");
    if (steps == kTubeSteps) {
        if (!tube_inst_ok(c->inst))
            return ctx_fail(c, MRT_EINVAL, "four steps per pass: 1, 2 or 4 periodic rows and "
                                           "fixed-equilibrium x sides");
        if (!c->d_items4) {
            const int rc = build_items4(c);
            if (rc != MRT_OK) return rc;
        }
    }
    if (steps == 2) {
        const int r = std::min(rows > 0 ? rows : default_rows2(c->nx, c->ny, c->prec), c->ny);
        if (r != c->rows2 || !c->d_items2) {
            const int rc = build_items2(c, r);
            if (rc != MRT_OK) return rc;
        }
    }
    c->per_pass = steps;
    c->graphs.clear();
    c->graphs2.clear();
    c->graphs4.clear();
    // the two-step path can leave the reflecting ghosts of the current state
    // stale; the single-step kernel expects them current
    if (c->params_set && c->fields_set) {
        const int rc = fill_ghosts(c);
        if (rc != MRT_OK) return rc;
    }
    HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

int mrt_set_scheme(mrt_ctx* c, int flags) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (flags < 0 || flags > (MRT_SCHEME_SPLIT | MRT_SCHEME_LW_CROSS))
        return ctx_fail(c, MRT_EINVAL, "unknown scheme flags");
    if ((flags & MRT_SCHEME_SPLIT) && !c->f_tmp) {
        const size_t bytes = size_t(mrt_population_bytes(c->nx, c->ny, c->prec));
        if (hipMalloc(&c->f_tmp, bytes) != hipSuccess) return ctx_fail(c, MRT_ENOMEM, "no memory for the split state");
        HIPTRY(hipMemsetAsync(c->f_tmp, 0, bytes, c->stream));
    }
    c->scheme = flags;
    c->graphs.clear();
    // the variants do not write the reflecting ghosts of their output: make
    // the ring current for whichever scheme runs next
    if (c->params_set && c->fields_set) {
        const int rc = fill_ghosts(c);
        if (rc != MRT_OK) return rc;
    }
    HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

int mrt_get_steps_per_pass(const mrt_ctx* c, int* steps, int* rows) {
    if (!c) return MRT_EINVAL;
    if (steps) *steps = c->per_pass;
    if (rows) *rows = c->per_pass == kTubeSteps ? c->ny : (c->per_pass == 2 ? c->rows2 : c->rows);
    return MRT_OK;
}

int mrt_get_tile(const mrt_ctx* c, int* rows, int* grid) {
    if (!c) return MRT_EINVAL;
    if (rows) *rows = c->rows;
    if (grid) *grid = c->grid;
    return MRT_OK;
}

int mrt_autotune(mrt_ctx* c, int steps) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set || !c->fields_set) return ctx_fail(c, MRT_ESTATE, "params and fields must be set");
    if (steps < 1) steps = 4;
    // the saved state must carry current reflecting-wall ghosts (after
    // two-step passes they can be stale), whichever kernel is chosen
    {
        const int rc = fill_ghosts(c);
        if (rc != MRT_OK) return rc;
    }
    const size_t bytes = size_t(mrt_population_bytes(c->nx, c->ny, c->prec));
    void* save = nullptr;
    HIPTRY(hipMalloc(&save, bytes));
    HIPTRY(hipMemcpyAsync(save, c->f[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream));
    hipEvent_t e0, e1;
    HIPTRY(hipEventCreate(&e0));
    HIPTRY(hipEventCreate(&e1));
    int dev = 0, cus = 0;
    HIPTRY(hipGetDevice(&dev));
    HIPTRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int row_opts[] = {1, 2, 3, 4, 5, 6, 8, 12, 16, 32, 64, 128};
    const int grid_mult[] = {0, 2, 4, 8};
    c->per_pass = 1;
    float best = 1e30f;
    int best_rows = c->rows, best_grid = c->grid;
    for (int r : row_opts) {
        if (r > c->ny && r != row_opts[0]) break;
        if (build_items(c, std::min(r, c->ny)) != MRT_OK) return MRT_EDEVICE;
        for (int gm : grid_mult) {
            const int g = gm == 0 ? 0 : gm * cus;
            if (g != 0 && g * 4 >= c->nitems) continue;
            c->grid = g;
            // warm-up, then timed (plain launches: no graph per trial)
            c->eager = true;
            mrt_step(c, 1);
            HIPTRY(hipEventRecord(e0, c->stream));
            mrt_step(c, steps);
            HIPTRY(hipEventRecord(e1, c->stream));
            c->eager = false;
            HIPTRY(hipEventSynchronize(e1));
            float ms = 0;
            HIPTRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_rows = c->rows;
                best_grid = g;
            }
            HIPTRY(hipMemcpyAsync(c->f[c->cur], save, bytes, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    // two steps per pass, per step
    int best_pass = 1, best_rows2 = 0;
    {
        best /= float(steps);
        const int steps2 = steps + (steps & 1);
        const int rows2_opts[] = {8, 16, 32, 64};
        for (int r : rows2_opts) {
            if (r > c->ny && r != rows2_opts[0]) break;
            if (build_items2(c, std::min(r, c->ny)) != MRT_OK) return MRT_EDEVICE;
            c->per_pass = 2;
            c->eager = true;
            mrt_step(c, 2);
            HIPTRY(hipEventRecord(e0, c->stream));
            mrt_step(c, steps2);
            HIPTRY(hipEventRecord(e1, c->stream));
            c->eager = false;
            HIPTRY(hipEventSynchronize(e1));
            float ms = 0;
            HIPTRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms / float(steps2) < best) {
                best = ms / float(steps2);
                best_pass = 2;
                best_rows2 = c->rows2;
            }
            HIPTRY(hipMemcpyAsync(c->f[c->cur], save, bytes, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    // the tube march, per step
    if (tube_inst_ok(c->inst) && c->scheme == 0) {
        if (build_items4(c) != MRT_OK) return MRT_EDEVICE;
        c->per_pass = kTubeSteps;
        const int steps4 = kTubeSteps * std::max(1, (steps + kTubeSteps - 1) / kTubeSteps);
        c->eager = true;
        mrt_step(c, kTubeSteps);
        HIPTRY(hipEventRecord(e0, c->stream));
        mrt_step(c, steps4);
        HIPTRY(hipEventRecord(e1, c->stream));
        c->eager = false;
        HIPTRY(hipEventSynchronize(e1));
        float ms = 0;
        HIPTRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms / float(steps4) < best) {
            best = ms / float(steps4);
            best_pass = kTubeSteps;
        }
        HIPTRY(hipMemcpyAsync(c->f[c->cur], save, bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPTRY(hipStreamSynchronize(c->stream));
    HIPTRY(hipEventDestroy(e0));
    HIPTRY(hipEventDestroy(e1));
    HIPTRY(hipFree(save));
    HIPTRY(hipMemsetAsync(c->d_health, 0, sizeof(unsigned), c->stream));
    if (build_items(c, best_rows) != MRT_OK) return MRT_EDEVICE;
    c->grid = best_grid;
    c->per_pass = best_pass;
    if (best_pass == 2 && build_items2(c, best_rows2) != MRT_OK) return MRT_EDEVICE;
    c->graphs.clear();
    c->graphs2.clear();
    c->graphs4.clear();
    HIPTRY(hipStreamSynchronize(c->stream));
    return MRT_OK;
}

void mrt_destroy(mrt_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->own_f) {
        if (c->f[0]) (void)hipFree(c->f[0]);
        if (c->f[1]) (void)hipFree(c->f[1]);
    }
    if (c->d_inst) (void)hipFree(c->d_inst);
    if (c->d_items) (void)hipFree(c->d_items);
    if (c->d_items_adj) (void)hipFree(c->d_items_adj);
    if (c->d_items2) (void)hipFree(c->d_items2);
    if (c->d_items4) (void)hipFree(c->d_items4);
    if (c->f_tmp) (void)hipFree(c->f_tmp);
    c->graphs.clear();
    c->graphs2.clear();
    c->graphs4.clear();
    if (c->d_stage) (void)hipFree(c->d_stage);
    if (c->d_partial) (void)hipFree(c->d_partial);
    if (c->d_health) (void)hipFree(c->d_health);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    for (hipEvent_t e : {c->ev_fork, c->ev_rec[0], c->ev_rec[1], c->ev_adj[0], c->ev_adj[1]})
        if (e) (void)hipEventDestroy(e);
    delete c;
}

const char* mrt_last_error(const mrt_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

// ---------------------------------------------------------------- adjoint

static bool all_periodic(const mrt_ctx* c) {
    for (int k = 0; k < 4; ++k)
        if (c->bc[k] != MRT_BC_PERIODIC) return false;
    return true;
}

int mrt_adjoint_step(mrt_ctx* c, const void* lam_next, const void* f_n, void* lam_n, double* ds) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    if (!all_periodic(c)) return ctx_fail(c, MRT_EINVAL, "adjoint needs periodic boundaries");
    if (c->scheme) return ctx_fail(c, MRT_EINVAL, "the adjoint is of the default scheme only");
    if (!lam_next || !f_n || !lam_n || !ds || lam_n == lam_next)
        return ctx_fail(c, MRT_EINVAL, "bad adjoint buffers");
    HIPTRY(mrt::k_adjoint(c->prec, c->d_inst, c->d_items_adj, c->nitems_adj, lam_next, f_n, lam_n,
                          c->d_partial, false, ds, c->nt, c->stream));
    return MRT_OK;
}

int mrt_adjoint_step_noalloc(mrt_ctx* c, const void* lam_next, const void* f_n, void* lam_n,
                             double* ds) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    if (!all_periodic(c)) return ctx_fail(c, MRT_EINVAL, "adjoint needs periodic boundaries");
    if (c->scheme) return ctx_fail(c, MRT_EINVAL, "the adjoint is of the default scheme only");
    if (!lam_next || !f_n || !lam_n || !ds || lam_n == lam_next)
        return ctx_fail(c, MRT_EINVAL, "bad adjoint buffers");
    if (!c->d_scratch) return ctx_fail(c, MRT_EDEVICE, c->scratch_err);
    const long long need = ((long long)c->nitems_adj + 64) * 16;
    if (need > kScratchDoubles) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "grid too large for the static scratch: %d adjoint work items, at most %d",
                      c->nitems_adj, kScratchDoubles / 16 - 64);
        return ctx_fail(c, MRT_EINVAL, buf);
    }
    // the kernel overwrites every partial row it reduces (no accumulation),
    // so nothing has to be cleared first
    HIPTRY(mrt::k_adjoint(c->prec, c->d_inst, c->d_items_adj, c->nitems_adj, lam_next, f_n, lam_n,
                          c->d_scratch, false, ds, c->nt, c->stream));
    return MRT_OK;
}

int mrt_step_checkpointed(mrt_ctx* c, void* f, void* f_tmp, int segment, int nsteps,
                          void* const* checkpoints) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    if (!f || !f_tmp || f == f_tmp || segment < 1 || nsteps < 0 || (nsteps > 0 && !checkpoints))
        return ctx_fail(c, MRT_EINVAL, "bad checkpointed-step arguments");
    const int nck = (nsteps + segment - 1) / segment;
    for (int k = 0; k < nck; ++k)
        if (!checkpoints[k] || checkpoints[k] == f || checkpoints[k] == f_tmp)
            return ctx_fail(c, MRT_EINVAL, "checkpoint buffers must be distinct from f and f_tmp");
    const size_t bytes = size_t(mrt_population_bytes(c->nx, c->ny, c->prec));
    if (nsteps == 0) return MRT_OK;
    // f^0 is copied into the first checkpoint; every later checkpointed
    // state is written there by its step directly (no copy), the others go
    // to whichever of f / f_tmp the step does not read
    HIPTRY(hipMemcpyAsync(checkpoints[0], f, bytes, hipMemcpyDeviceToDevice, c->stream));
    void* a = f;
    for (int n = 0; n < nsteps; ++n) {
        void* dst;
        if ((n + 1) % segment == 0 && n + 1 < nsteps)
            dst = checkpoints[(n + 1) / segment];
        else
            dst = a == f ? f_tmp : f;
        const int rc = mrt_step_buffers(c, a, dst);
        if (rc != MRT_OK) return rc;
        a = dst;
    }
    if (a != f) HIPTRY(hipMemcpyAsync(f, a, bytes, hipMemcpyDeviceToDevice, c->stream));
    return MRT_OK;
}

// The sweep's second stream (default priority, like every stream here) and
// its events.
static int ensure_aux_stream(mrt_ctx* c) {
    std::string& ctx_err = c->err;
    if (c->aux) return MRT_OK;
    // the events first: the stream is the flag that all of them exist (the
    // ones made before a failure are kept and reused by the next attempt)
    for (hipEvent_t* e : {&c->ev_fork, &c->ev_rec[0], &c->ev_rec[1], &c->ev_adj[0], &c->ev_adj[1]})
        if (!*e) HIPTRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    hipStream_t st = nullptr;
    HIPTRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    c->aux = st;
    return MRT_OK;
}

int mrt_adjoint_sweep(mrt_ctx* c, const void* const* checkpoints, int segment, int nsteps,
                      void* const* work, int nwork, void* lam, void* lam_tmp, double* ds) {
    if (!c) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    if (!all_periodic(c)) return ctx_fail(c, MRT_EINVAL, "adjoint needs periodic boundaries");
    if (c->scheme) return ctx_fail(c, MRT_EINVAL, "the adjoint is of the default scheme only");
    if (!lam || !lam_tmp || lam == lam_tmp || !ds || segment < 1 || nsteps < 0 || nwork < 0 ||
        (nsteps > 0 && !checkpoints))
        return ctx_fail(c, MRT_EINVAL, "bad adjoint-sweep arguments");
    const int nck = (nsteps + segment - 1) / segment;
    for (int k = 0; k < nck; ++k)
        if (!checkpoints[k]) return ctx_fail(c, MRT_EINVAL, "missing checkpoint");
    // w recomputed states per segment; two sets of them let the next
    // segment's recomputation run beside the current segment's adjoint steps
    const int w = std::max(0, std::min(segment, nsteps) - 1);
    if (nwork < w) return ctx_fail(c, MRT_EINVAL, "fewer work buffers than min(segment, nsteps) - 1");
    const int sets = (w > 0 && nck > 1 && nwork >= 2 * w) ? 2 : 1;
    if (w > 0 && !work) return ctx_fail(c, MRT_EINVAL, "bad adjoint-sweep arguments");
    for (int j = 0; j < sets * w; ++j)
        if (!work[j] || work[j] == lam || work[j] == lam_tmp)
            return ctx_fail(c, MRT_EINVAL, "work buffers must be distinct from lam and lam_tmp");
    if (sets == 2) {
        const int rc = ensure_aux_stream(c);
        if (rc != MRT_OK) return rc;
    }
    auto set_of = [&](int seg) { return sets == 2 ? (seg & 1) : 0; };
    // f^{start + j} of segment seg: its checkpoint for j = 0, else a work buffer
    auto state = [&](int seg, int j) -> const void* {
        return j == 0 ? checkpoints[seg] : work[set_of(seg) * w + j - 1];
    };
    // f^{start + 1} .. f^{stop - 1} of segment seg, one step each as
    // mrt_step_buffers takes it on a periodic grid (no ghost ring to refill)
    auto recompute = [&](int seg, hipStream_t st) -> hipError_t {
        const int start = seg * segment, stop = std::min(nsteps, start + segment);
        for (int j = 1; j < stop - start; ++j) {
            const hipError_t e = mrt::k_step(c->prec, c->d_inst, c->d_items, c->nitems, state(seg, j - 1),
                                             const_cast<void*>(state(seg, j)), c->d_health, c->grid, c->nt,
                                             c->walls, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    void* cur = lam;
    void* nxt = lam_tmp;
    // the rate-gradient partial rows of all steps are summed in place and
    // reduced into ds once, after the last step
    bool first = true;
    auto adjoint_steps = [&](int seg) -> hipError_t {
        const int start = seg * segment, stop = std::min(nsteps, start + segment);
        for (int n = stop - 1; n >= start; --n) {
            const hipError_t e = mrt::k_adjoint(c->prec, c->d_inst, c->d_items_adj, c->nitems_adj, cur,
                                                state(seg, n - start), nxt, c->d_partial, !first,
                                                n == 0 ? ds : nullptr, c->nt, c->stream);
            if (e != hipSuccess) return e;
            first = false;
            std::swap(cur, nxt);
        }
        return hipSuccess;
    };
    if (sets == 1) {
        for (int seg = nck - 1; seg >= 0; --seg) {
            HIPTRY(recompute(seg, c->stream));
            HIPTRY(adjoint_steps(seg));
        }
    } else {
        // segment seg's states are recomputed on the second stream into set
        // seg & 1 while the adjoint steps of segment seg + 1 read the other
        // set on the context's stream.  ev_rec[s]: set s holds its segment's
        // states; ev_adj[s]: the adjoint steps reading set s are done, so it
        // may be overwritten.  The adjoint steps themselves stay in order on
        // one stream: lam and ds are those of the one-stream sweep.
        HIPTRY(hipEventRecord(c->ev_fork, c->stream));
        HIPTRY(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
        bool read_issued[2] = {false, false};
        HIPTRY(recompute(nck - 1, c->aux));
        HIPTRY(hipEventRecord(c->ev_rec[set_of(nck - 1)], c->aux));
        for (int seg = nck - 1; seg >= 0; --seg) {
            if (seg >= 1) {
                const int s2 = set_of(seg - 1);
                if (read_issued[s2]) HIPTRY(hipStreamWaitEvent(c->aux, c->ev_adj[s2], 0));
                HIPTRY(recompute(seg - 1, c->aux));
                HIPTRY(hipEventRecord(c->ev_rec[s2], c->aux));
            }
            const int s1 = set_of(seg);
            HIPTRY(hipStreamWaitEvent(c->stream, c->ev_rec[s1], 0));
            HIPTRY(adjoint_steps(seg));
            HIPTRY(hipEventRecord(c->ev_adj[s1], c->stream));
            read_issued[s1] = true;
        }
        // the context's stream waited for the last recomputation (segment 0)
        // before its adjoint steps: nothing of the sweep is left on aux
    }
    if (cur != lam) {
        const size_t bytes = size_t(mrt_population_bytes(c->nx, c->ny, c->prec));
        HIPTRY(hipMemcpyAsync(lam, cur, bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    return MRT_OK;
}

int mrt_density(mrt_ctx* c, const void* f, double* rho) {
    if (!c || !f || !rho) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    HIPTRY(mrt::k_density(c->prec, c->d_inst, (long long)c->nx * c->ny, f, rho, c->stream));
    return MRT_OK;
}

int mrt_density_adjoint(mrt_ctx* c, const double* g_rho, void* lam) {
    if (!c || !g_rho || !lam) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    HIPTRY(mrt::k_density_adjoint(c->prec, c->d_inst, (long long)c->nx * c->ny, g_rho, lam, c->stream));
    return MRT_OK;
}

int mrt_init_adjoint(mrt_ctx* c, const void* lam0, const double* rho, const double* ux,
                     const double* uy, const double* T, double* g_rho, double* g_ux, double* g_uy,
                     double* g_T) {
    if (!c || !lam0 || !rho || !ux || !uy || !T) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    HIPTRY(mrt::k_init_adjoint(c->prec, c->d_inst, (long long)c->nx * c->ny, lam0, rho, ux, uy, T,
                               g_rho, g_ux, g_uy, g_T, c->stream));
    return MRT_OK;
}

int mrt_init_buffer(mrt_ctx* c, const double* rho, const double* ux, const double* uy,
                    const double* T, void* f) {
    if (!c || !rho || !ux || !uy || !T || !f) return MRT_EINVAL;
    std::string& ctx_err = c->err;
    if (!c->params_set) return ctx_fail(c, MRT_ESTATE, "set_params first");
    HIPTRY(mrt::k_init(c->prec, c->d_inst, (long long)c->nx * c->ny, rho, ux, uy, T, f, c->stream));
    if (has_kind(c->bc, MRT_BC_EQ))
        HIPTRY(mrt::k_ghost(c->prec, c->d_inst, 1, 2 * (c->nx + c->ny), f, 2, c->stream));
    return MRT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch

struct mrt_batch {
    int count = 0, prec = 0;
    hipStream_t stream = nullptr;
    std::vector<Inst> insts;
    std::vector<long long> cells;
    long long total_cells = 0, total_elems = 0, max_cells = 0;
    int max_perim = 0;
    bool any_reflect = false;
    bool any_xwall = false;                 // some instance has a reflecting x side
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    Inst* d_insts = nullptr;
    Item* d_items = nullptr;
    int nitems = 0, rows = 0, grid = 0;
    bool nt = false;                        // non-temporal population stores
    bool walls = false;                     // the step kernel writes the reflecting-wall ghosts
    double* d_stage = nullptr;
    unsigned* d_health = nullptr;
    GraphCache graphs;                      // captured steps
    int per_pass = 1;                       // time steps per pass (1 or 2)
    Item* d_items2 = nullptr;               // work items of the two-step kernel
    int nitems2 = 0, rows2 = 0;
    bool wrap4 = false;                     // some band is a whole periodic height of 4 rows
    GraphCache graphs2;                     // captured two-step passes
    Item* d_items4 = nullptr;               // work items of the tube march
    int nitems4 = 0, tube_ny = 0;           // tube_ny: the rows of every instance
    GraphCache graphs4;                     // captured tube-march passes
    std::string err;
};

namespace {

int batch_items(mrt_batch* b, int rows) {
    std::string& ctx_err = b->err;
    std::vector<Item> items;
    for (int i = 0; i < b->count; ++i) {
        b->insts[i].item0 = int(items.size());
        add_items(items, i, b->insts[i].nx, b->insts[i].ny, std::min(rows, b->insts[i].ny));
    }
    if (b->d_items) HIPTRY(hipFree(b->d_items));
    b->d_items = nullptr;
    HIPTRY(hipMalloc(&b->d_items, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    b->nitems = int(items.size());
    b->rows = rows;
    b->graphs.clear();
    return MRT_OK;
}

// Work items of the two-step kernel: bands of at most `rows` <= 32 rows per
// instance (the instance table is not touched).
int batch_items2(mrt_batch* b, int rows) {
    std::string& ctx_err = b->err;
    std::vector<Item> items;
    for (int i = 0; i < b->count; ++i)
        add_items(items, i, b->insts[i].nx, b->insts[i].ny, std::min(rows, b->insts[i].ny));
    if (b->d_items2) HIPTRY(hipFree(b->d_items2));
    b->d_items2 = nullptr;
    HIPTRY(hipMalloc(&b->d_items2, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(b->d_items2, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    b->nitems2 = int(items.size());
    b->rows2 = rows;
    b->wrap4 = false;
    for (int i = 0; i < b->count; ++i) b->wrap4 = b->wrap4 || wraps_four_rows(b->insts[i], rows);
    b->graphs2.clear();
    return MRT_OK;
}

// Whether the tube march (kTubeSteps steps per pass) can advance the
// batch: every instance the same height of 1, 2 or 4 periodic rows with
// fixed-equilibrium x sides.
bool tube_march_ok(const mrt_batch* b) {
    for (const Inst& I : b->insts)
        if (!tube_inst_ok(I) || I.ny != b->insts[0].ny) return false;
    return true;
}

// Work items of the tube march: kTubeWidth-column chunks of each instance.
int batch_items4(mrt_batch* b) {
    std::string& ctx_err = b->err;
    std::vector<Item> items;
    for (int i = 0; i < b->count; ++i) add_tube_items(items, i, b->insts[i].nx, b->insts[i].ny);
    b->tube_ny = b->insts[0].ny;
    if (b->d_items4) HIPTRY(hipFree(b->d_items4));
    b->d_items4 = nullptr;
    HIPTRY(hipMalloc(&b->d_items4, items.size() * sizeof(Item)));
    HIPTRY(hipMemcpy(b->d_items4, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    b->nitems4 = int(items.size());
    b->graphs4.clear();
    return MRT_OK;
}

}  // namespace

extern "C" {

int mrt_batch_create(mrt_batch** out, int count, const mrt_instance* desc, int precision,
                     void* stream) {
    if (!out) return MRT_EINVAL;
    *out = nullptr;
    if (count < 1 || !desc || precision < 0 || precision > 2) return MRT_EINVAL;
    mrt_batch* b = new mrt_batch();
    std::string& ctx_err = b->err;
    b->count = count;
    b->prec = precision;
    b->stream = static_cast<hipStream_t>(stream);
    b->insts.resize(count);
    b->cells.resize(count);
    long long off = 0;
    int maxny = 1;
    for (int i = 0; i < count; ++i) {
        const mrt_instance& d = desc[i];
        if (!size_ok(d.nx, d.ny) || !bc_ok(d.bc)) {
            delete b;
            return MRT_EINVAL;
        }
        Inst& I = b->insts[i];
        I = Inst{};
        I.nx = d.nx;
        I.ny = d.ny;
        I.pitch = int(pitch_for(d.nx));
        I.origin = int(origin_for(d.nx));
        I.plane = plane_for(d.nx);
        b->max_perim = std::max(b->max_perim, 2 * (d.nx + d.ny));
        b->any_reflect = b->any_reflect || has_kind(d.bc, MRT_BC_REFLECT);
        b->any_xwall = b->any_xwall || d.bc[0] == MRT_BC_REFLECT || d.bc[1] == MRT_BC_REFLECT;
        I.off = off;
        std::string e;
        if (fill_inst(I, d.nx, d.ny, d.bc, &d.params, e) != MRT_OK) {
            delete b;
            return MRT_EINVAL;
        }
        off += elems_for(d.nx, d.ny);
        b->cells[i] = (long long)d.nx * d.ny;
        b->total_cells += b->cells[i];
        b->max_cells = std::max(b->max_cells, b->cells[i]);
        maxny = std::max(maxny, d.ny);
    }
    b->total_elems = off;
    const size_t bytes = size_t(off) * elem_size(precision);
    b->nt = (long long)bytes > kNonTemporalBytes;
    b->walls = b->any_reflect && b->total_cells <= kWallsInKernelCells;
    auto fail = [&](int code) {
        mrt_batch_destroy(b);
        return code;
    };
    if (hipMalloc(&b->f[0], bytes) != hipSuccess || hipMalloc(&b->f[1], bytes) != hipSuccess ||
        hipMalloc(&b->d_insts, sizeof(Inst) * count) != hipSuccess ||
        hipMalloc(&b->d_stage, 4 * sizeof(double) * size_t(b->max_cells)) != hipSuccess ||
        hipMalloc(&b->d_health, sizeof(unsigned)) != hipSuccess)
        return fail(MRT_ENOMEM);
    if (hipMemset(b->f[0], 0, bytes) != hipSuccess || hipMemset(b->f[1], 0, bytes) != hipSuccess ||
        hipMemset(b->d_health, 0, sizeof(unsigned)) != hipSuccess)
        return fail(MRT_EDEVICE);
    if (batch_items(b, std::min(maxny, 64)) != MRT_OK) return fail(MRT_EDEVICE);
    // a batch of tubes the tube march covers (all of one height of 1, 2 or 4
    // periodic rows, fixed-equilibrium x sides) runs four steps per pass by
    // default
    if (tube_march_ok(b)) {
        if (batch_items4(b) != MRT_OK) return fail(MRT_EDEVICE);
        b->per_pass = kTubeSteps;
    }
    if (hipMemcpy(b->d_insts, b->insts.data(), sizeof(Inst) * count, hipMemcpyHostToDevice) != hipSuccess)
        return fail(MRT_EDEVICE);
    (void)ctx_err;
    *out = b;
    return MRT_OK;
}

int mrt_batch_set_fields(mrt_batch* b, int i, const double* rho, const double* ux,
                         const double* uy, const double* T) {
    if (!b || i < 0 || i >= b->count || !rho || !ux || !uy || !T) return MRT_EINVAL;
    std::string& ctx_err = b->err;
    const long long n = b->cells[i];
    for (long long k = 0; k < n; ++k)
        if (!(rho[k] > 0 && T[k] > 0)) {
            b->err = "rho and T must be > 0";
            return MRT_EINVAL;
        }
    double* s = b->d_stage;
    const size_t by = sizeof(double) * size_t(n);
    HIPTRY(hipMemcpyAsync(s, rho, by, hipMemcpyHostToDevice, b->stream));
    HIPTRY(hipMemcpyAsync(s + n, ux, by, hipMemcpyHostToDevice, b->stream));
    HIPTRY(hipMemcpyAsync(s + 2 * n, uy, by, hipMemcpyHostToDevice, b->stream));
    HIPTRY(hipMemcpyAsync(s + 3 * n, T, by, hipMemcpyHostToDevice, b->stream));
    HIPTRY(mrt::k_init(b->prec, b->d_insts + i, n, s, s + n, s + 2 * n, s + 3 * n, b->f[b->cur], b->stream));
    // equilibrium ghosts of this instance in both buffers, reflecting ones
    // of its current state
    const int perim = 2 * (b->insts[i].nx + b->insts[i].ny);
    for (int k = 0; k < 2; ++k)
        HIPTRY(mrt::k_ghost(b->prec, b->d_insts + i, 1, perim, b->f[k], 2, b->stream));
    HIPTRY(mrt::k_ghost(b->prec, b->d_insts + i, 1, perim, b->f[b->cur], 1, b->stream));
    HIPTRY(hipStreamSynchronize(b->stream));
    return MRT_OK;
}

static int batch_step_impl(mrt_batch* b, int n, bool launch);

int mrt_batch_step(mrt_batch* b, int n) { return batch_step_impl(b, n, true); }

int mrt_batch_prepare_steps(mrt_batch* b, int n) { return batch_step_impl(b, n, false); }

static int batch_step_impl(mrt_batch* b, int n, bool launch) {
    if (!b || n < 0) return MRT_EINVAL;
    std::string& ctx_err = b->err;
    if (n == 0) return MRT_OK;
    if (b->per_pass == kTubeSteps) {
        // the tube march (no reflecting sides: its x sides are fixed
        // equilibria, its y sides periodic), the remaining steps one by one
        auto enqueue4 = [&](int cur, hipStream_t st) -> hipError_t {
            return mrt::k_tube(b->prec, b->d_insts, b->d_items4, b->nitems4, b->f[cur], b->f[1 - cur],
                               b->d_health, 0, b->nt, b->tube_ny, st);
        };
        const int passes = n / kTubeSteps;
        if (passes > 0) HIPTRY(run_graphs(b->graphs4, b->cur, passes, b->stream, enqueue4, launch));
        if (launch) {
            for (int k = 0; k < n % kTubeSteps; ++k) {
                HIPTRY(mrt::k_step(b->prec, b->d_insts, b->d_items, b->nitems, b->f[b->cur],
                                   b->f[1 - b->cur], b->d_health, b->grid, b->nt, false, b->stream));
                b->cur ^= 1;
            }
        }
        return MRT_OK;
    }
    if (b->per_pass == 2) {
        // two steps per pass, an odd last step by the single-step kernel.
        // The two-step kernel writes the reflecting y-wall ghosts of its
        // output: the ghost pass runs before the first pass of a graph, and
        // before every pass only when some instance has a reflecting x side
        auto ghosts = [&](int cur, hipStream_t st) -> hipError_t {
            return b->any_reflect ? mrt::k_ghost(b->prec, b->d_insts, b->count, b->max_perim, b->f[cur], 1, st)
                                  : hipSuccess;
        };
        auto enqueue2 = [&](int cur, hipStream_t st, int k) -> hipError_t {
            const hipError_t e = k == 0 || b->any_xwall ? ghosts(cur, st) : hipSuccess;
            if (e != hipSuccess) return e;
            return mrt::k_step2(b->prec, b->d_insts, b->d_items2, b->nitems2, b->f[cur], b->f[1 - cur],
                                b->d_health, 0, b->nt, b->wrap4, st);
        };
        const int pairs = n / 2;
        if (pairs > 0) HIPTRY(run_graphs(b->graphs2, b->cur, pairs, b->stream, enqueue2, launch));
        if ((n & 1) && launch) {
            HIPTRY(ghosts(b->cur, b->stream));
            HIPTRY(mrt::k_step(b->prec, b->d_insts, b->d_items, b->nitems, b->f[b->cur], b->f[1 - b->cur],
                               b->d_health, b->grid, b->nt, false, b->stream));
            b->cur ^= 1;
        }
        return MRT_OK;
    }
    // reflecting-wall ghosts: written by the step kernel with its output
    // (b->walls), else refilled before each step
    auto enqueue = [&](int cur, hipStream_t st) -> hipError_t {
        if (b->any_reflect && !b->walls) {
            const hipError_t e = mrt::k_ghost(b->prec, b->d_insts, b->count, b->max_perim, b->f[cur], 1, st);
            if (e != hipSuccess) return e;
        }
        return mrt::k_step(b->prec, b->d_insts, b->d_items, b->nitems, b->f[cur], b->f[1 - cur],
                           b->d_health, b->grid, b->nt, b->walls, st);
    };
    HIPTRY(run_graphs(b->graphs, b->cur, n, b->stream, enqueue, launch));
    return MRT_OK;
}

int mrt_batch_read_moments(mrt_batch* b, int i, double* rho, double* ux, double* uy, double* T) {
    if (!b || i < 0 || i >= b->count) return MRT_EINVAL;
    std::string& ctx_err = b->err;
    const long long n = b->cells[i];
    double* s = b->d_stage;
    HIPTRY(mrt::k_moments(b->prec, b->d_insts + i, n, b->f[b->cur], s, s + n, s + 2 * n, s + 3 * n,
                          b->d_health, b->stream));
    double* outs[4] = {rho, ux, uy, T};
    for (int k = 0; k < 4; ++k)
        if (outs[k])
            HIPTRY(hipMemcpyAsync(outs[k], s + k * n, sizeof(double) * size_t(n), hipMemcpyDeviceToHost, b->stream));
    unsigned h = 0;
    HIPTRY(hipMemcpyAsync(&h, b->d_health, sizeof h, hipMemcpyDeviceToHost, b->stream));
    HIPTRY(hipStreamSynchronize(b->stream));
    if (h) {
        HIPTRY(hipMemsetAsync(b->d_health, 0, sizeof(unsigned), b->stream));
        HIPTRY(hipStreamSynchronize(b->stream));
        b->err = "non-finite value, rho <= 0 or T <= 0 detected";
        return MRT_EUNSTABLE;
    }
    return MRT_OK;
}

int mrt_batch_get_populations(mrt_batch* b, int i, double* f) {
    if (!b || i < 0 || i >= b->count || !f) return MRT_EINVAL;
    std::string& ctx_err = b->err;
    const long long n = b->cells[i];
    double* tmp = nullptr;
    HIPTRY(hipMallocAsync((void**)&tmp, sizeof(double) * 16 * size_t(n), b->stream));
    HIPTRY(mrt::k_export(b->prec, b->d_insts + i, n, b->f[b->cur], tmp, b->stream));
    HIPTRY(hipMemcpyAsync(f, tmp, sizeof(double) * 16 * size_t(n), hipMemcpyDeviceToHost, b->stream));
    HIPTRY(hipFreeAsync(tmp, b->stream));
    HIPTRY(hipStreamSynchronize(b->stream));
    return MRT_OK;
}

int mrt_batch_set_tile(mrt_batch* b, int rows, int grid) {
    if (!b || rows < 1 || grid < 0) return MRT_EINVAL;
    const int rc = batch_items(b, rows);
    if (rc != MRT_OK) return rc;
    std::string& ctx_err = b->err;
    HIPTRY(hipMemcpy(b->d_insts, b->insts.data(), sizeof(Inst) * b->count, hipMemcpyHostToDevice));
    b->grid = grid;
    return MRT_OK;
}

int mrt_batch_set_steps_per_pass(mrt_batch* b, int steps, int rows) {
    if (!b) return MRT_EINVAL;
    std::string& ctx_err = b->err;
    if (steps != 1 && steps != 2 && steps != kTubeSteps)
        return (b->err = "steps per pass: 1, 2 or 4", MRT_EINVAL);
    if (rows < 0 || rows > MRT_MAX_BAND_ROWS_2) return (b->err = "rows: 0 (default) to 64", MRT_EINVAL);
    if (steps == kTubeSteps) {
        if (!tube_march_ok(b))
            return (b->err = "four steps per pass: every instance 1, 2 or 4 periodic rows (the same "
                             "for all) with fixed-equilibrium x sides", MRT_EINVAL);
        if (!b->d_items4) {
            const int rc = batch_items4(b);
            if (rc != MRT_OK) return rc;
        }
    }
    if (steps == 2) {
        const int r = rows > 0 ? rows : kBatchRows2;
        if (r != b->rows2 || !b->d_items2) {
            const int rc = batch_items2(b, r);
            if (rc != MRT_OK) return rc;
        }
    }
    b->per_pass = steps;
    b->graphs.clear();
    b->graphs2.clear();
    b->graphs4.clear();
    // the two-step path can leave the reflecting ghosts of the current state
    // stale; the single-step kernel with in-kernel walls expects them current
    if (b->any_reflect)
        HIPTRY(mrt::k_ghost(b->prec, b->d_insts, b->count, b->max_perim, b->f[b->cur], 1, b->stream));
    HIPTRY(hipStreamSynchronize(b->stream));
    return MRT_OK;
}

int mrt_batch_get_steps_per_pass(const mrt_batch* b, int* steps, int* rows) {
    if (!b) return MRT_EINVAL;
    if (steps) *steps = b->per_pass;
    if (rows) *rows = b->per_pass == kTubeSteps ? b->tube_ny : (b->per_pass == 2 ? b->rows2 : b->rows);
    return MRT_OK;
}

int mrt_batch_get_tile(const mrt_batch* b, int* rows, int* grid) {
    if (!b) return MRT_EINVAL;
    if (rows) *rows = b->rows;
    if (grid) *grid = b->grid;
    return MRT_OK;
}

int mrt_batch_autotune(mrt_batch* b, int steps) {
    if (!b) return MRT_EINVAL;
    std::string& ctx_err = b->err;
    if (steps < 1) steps = 8;
    // the saved state must carry current reflecting-wall ghosts (after
    // two-step passes they can be stale), whichever kernel is chosen
    if (b->any_reflect)
        HIPTRY(mrt::k_ghost(b->prec, b->d_insts, b->count, b->max_perim, b->f[b->cur], 1, b->stream));
    const size_t bytes = size_t(b->total_elems) * elem_size(b->prec);
    void* save = nullptr;
    HIPTRY(hipMalloc(&save, bytes));
    HIPTRY(hipMemcpyAsync(save, b->f[b->cur], bytes, hipMemcpyDeviceToDevice, b->stream));
    hipEvent_t e0, e1;
    HIPTRY(hipEventCreate(&e0));
    HIPTRY(hipEventCreate(&e1));
    int dev = 0, cus = 0;
    HIPTRY(hipGetDevice(&dev));
    HIPTRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int maxny = 1;
    for (const auto& I : b->insts) maxny = std::max(maxny, I.ny);
    const int row_opts[] = {1, 2, 4, 8, 16, 32, 64};
    const int grid_mult[] = {0, 2, 4, 8};
    float best = 1e30f;
    int best_rows = b->rows, best_grid = b->grid;
    const int cur0 = b->cur;
    b->per_pass = 1;
    for (int r : row_opts) {
        if (r > maxny) break;
        for (int gm : grid_mult) {
            if (mrt_batch_set_tile(b, r, gm * cus) != MRT_OK) return MRT_EDEVICE;
            if (gm != 0 && gm * cus * 4 >= b->nitems) continue;
            mrt_batch_step(b, steps);    // capture + warm-up
            HIPTRY(hipEventRecord(e0, b->stream));
            mrt_batch_step(b, steps);
            HIPTRY(hipEventRecord(e1, b->stream));
            HIPTRY(hipEventSynchronize(e1));
            float ms = 0;
            HIPTRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_rows = r;
                best_grid = gm * cus;
            }
            b->cur = cur0;
            HIPTRY(hipMemcpyAsync(b->f[b->cur], save, bytes, hipMemcpyDeviceToDevice, b->stream));
        }
    }
    // two steps per pass, per step
    int best_pass = 1, best_rows2 = 0;
    {
        best /= float(steps);
        const int steps2 = steps + (steps & 1);
        const int rows2_opts[] = {4, 8, 16, 32, 64};
        for (int r : rows2_opts) {
            if (r > maxny && r != rows2_opts[0]) break;
            if (batch_items2(b, r) != MRT_OK) return MRT_EDEVICE;
            b->per_pass = 2;
            mrt_batch_step(b, steps2);    // capture + warm-up
            HIPTRY(hipEventRecord(e0, b->stream));
            mrt_batch_step(b, steps2);
            HIPTRY(hipEventRecord(e1, b->stream));
            HIPTRY(hipEventSynchronize(e1));
            float ms = 0;
            HIPTRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms / float(steps2) < best) {
                best = ms / float(steps2);
                best_pass = 2;
                best_rows2 = r;
            }
            b->cur = cur0;
            HIPTRY(hipMemcpyAsync(b->f[b->cur], save, bytes, hipMemcpyDeviceToDevice, b->stream));
        }
    }
    // the tube march, per step
    if (tube_march_ok(b)) {
        if (batch_items4(b) != MRT_OK) return MRT_EDEVICE;
        b->per_pass = kTubeSteps;
        const int steps4 = kTubeSteps * std::max(1, (steps + kTubeSteps - 1) / kTubeSteps);
        mrt_batch_step(b, steps4);    // capture + warm-up
        HIPTRY(hipEventRecord(e0, b->stream));
        mrt_batch_step(b, steps4);
        HIPTRY(hipEventRecord(e1, b->stream));
        HIPTRY(hipEventSynchronize(e1));
        float ms = 0;
        HIPTRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms / float(steps4) < best) {
            best = ms / float(steps4);
            best_pass = kTubeSteps;
        }
        b->cur = cur0;
        HIPTRY(hipMemcpyAsync(b->f[b->cur], save, bytes, hipMemcpyDeviceToDevice, b->stream));
    }
    HIPTRY(hipStreamSynchronize(b->stream));
    HIPTRY(hipEventDestroy(e0));
    HIPTRY(hipEventDestroy(e1));
    HIPTRY(hipFree(save));
    HIPTRY(hipMemsetAsync(b->d_health, 0, sizeof(unsigned), b->stream));
    b->per_pass = 1;
    int rc = mrt_batch_set_tile(b, best_rows, best_grid);
    if (rc == MRT_OK && best_pass == 2) rc = mrt_batch_set_steps_per_pass(b, 2, best_rows2);
    if (rc == MRT_OK && best_pass == kTubeSteps) rc = mrt_batch_set_steps_per_pass(b, kTubeSteps, 0);
    HIPTRY(hipStreamSynchronize(b->stream));
    return rc;
}

long long mrt_batch_cells(const mrt_batch* b) { return b ? b->total_cells : 0; }

void mrt_batch_destroy(mrt_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    b->graphs.clear();
    b->graphs2.clear();
    b->graphs4.clear();
    if (b->d_items2) (void)hipFree(b->d_items2);
    if (b->d_items4) (void)hipFree(b->d_items4);
    if (b->f[0]) (void)hipFree(b->f[0]);
    if (b->f[1]) (void)hipFree(b->f[1]);
    if (b->d_insts) (void)hipFree(b->d_insts);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_stage) (void)hipFree(b->d_stage);
    if (b->d_health) (void)hipFree(b->d_health);
    delete b;
}

const char* mrt_batch_last_error(const mrt_batch* b) { return b ? b->err.c_str() : "NULL batch"; }

// --------------------------------------------------------- host utilities
// The same templated transform code the kernels run, evaluated on the host
// in FP64.  Used by the library for boundary equilibria and exported for
// CPU-side checks of the factored transforms.

int mrt_host_transform(int which, const double* in, double* out) {
    if (!in || !out) return MRT_EINVAL;
    switch (which) {
        case 0: mrt::pops_to_moments(in, out); return MRT_OK;
        case 1: mrt::moments_to_pops(in, out); return MRT_OK;
        case 2: mrt::moments_T(in, out); return MRT_OK;
        case 3: mrt::inverse_T(in, out); return MRT_OK;
        default: return MRT_EINVAL;
    }
}

int mrt_host_equilibrium(double gamma, double rho, double ux, double uy, double T, double* f) {
    if (!f || !(gamma > 1.0)) return MRT_EINVAL;
    mrt::equilibrium_pops<double>(rho, ux, uy, T, 2.0 / (gamma - 1.0), f);
    return MRT_OK;
}

int mrt_host_collision(double gamma, const double* s, double dt, const double* f, double* out) {
    if (!s || !f || !out || !(gamma > 1.0)) return MRT_EINVAL;
    double sdt[16];
    for (int k = 0; k < 16; ++k) sdt[k] = s[k] * dt;
    double rho, P;
    mrt::collision_dt<double>(f, 2.0 / (gamma - 1.0), sdt, out, rho, P);
    return MRT_OK;
}

int mrt_host_cell_adjoint(double gamma, const double* s, double dt, const double* f,
                          const double* lam, double* coll, double* dsk) {
    if (!s || !f || !lam || !coll || !dsk || !(gamma > 1.0)) return MRT_EINVAL;
    double sdt[16];
    for (int k = 0; k < 16; ++k) sdt[k] = k < 4 ? 0.0 : s[k] * dt;
    const double b = 2.0 / (gamma - 1.0);
    mrt::cell_adjoint<double>(f, lam, b, 1.0 / b, sdt, dt, coll, dsk);
    return MRT_OK;
}

int mrt_host_conserved_fp32(const float* f, float* q) {
    if (!f || !q) return MRT_EINVAL;
    mrt::conserved_compensated(f, q);
    return MRT_OK;
}

}  // extern "C"
