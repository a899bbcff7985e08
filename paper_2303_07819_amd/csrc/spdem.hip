// spdem: superparameterised sea-ice floe DEM for MI355X (gfx950, CDNA4).
//
// Host side: the C ABI of include/spdem.h over the kernels of dem_kernels.h.
//
// Layout: floe state SoA in HBM, sorted by cell, updated in place (xi, yi u32
// cell fractions; u, v, w, th, r, h f32).  Statistics are double-buffered per
// time level (ncells x 16 f64) and so is the continuum Q (4 x ncells f64).
//
// Scheduling: cells are grouped by floe count into buckets (<= 64, <= 128,
// <= 256, <= 512, <= 1024 floes).  Each non-empty bucket is one launch per step
// over its cell list, sorted costliest first, run with W wavefronts per cell
// (one wavefront for small cells, a tile of up to 8 for large ones), either in
// grid order or by persistent workgroups that pull cells from a counter.  W and
// the persistent flag per bucket come from defaults or from sp_autotune, which
// times every variant on a scratch copy of the state.  The continuum update of
// step k runs inside the DEM launch of step k + 1, and chunks of steady-state
// steps are replayed as one captured HIP graph.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/spdem.h"
#include "dem_kernels.h"
#include "block_kernels.h"

using namespace spdem;

namespace {

constexpr int kNumBuckets = 5;
constexpr double kSkinFrac = 0.3;   // smallest candidate-list skin, in units of the largest radius
constexpr int kBucketHi[kNumBuckets] = {64, 128, 256, 512, SP_MAX_CELL_FLOES};
constexpr int kDefaultWaves[kNumBuckets] = {1, 2, 4, 4, 8};
constexpr int kDefaultGraphChunk = 16;
constexpr int kDefaultStepBlock = 32;   // steps per blocked DEM launch

struct Bucket {
    int waves = 4;
    int persist = 0;                    // resident workgroups stride over the cells
    int bwaves = 0;                     // wavefronts per cell of blocked launches (0: derived from waves)
    int cap = 0;                        // LDS floe capacity per group
    int resident = 1;                   // workgroups resident at once (persistent grid size)
    std::vector<int32_t> cells_h;       // costliest first
    int4* work_d = nullptr;             // (cell, first floe, count, -) per entry of cells_h
    size_t work_cap = 0;                // entries work_d holds
};

}  // namespace

struct sp_ctx {
    sp_params p;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int device = 0;
    int num_cus = 256;

    // ocean
    double u0 = 0, v0 = 0;
    int nmodes = 0;
    double kx[SP_MAX_MODES], ky[SP_MAX_MODES], au[SP_MAX_MODES], av[SP_MAX_MODES],
        ph[SP_MAX_MODES];
    bool phase_dirty = true;

    // floes
    int64_t n = 0;
    int32_t ncells = 0;
    int32_t nbx = 1, nby = 1;
    int32_t sched = SP_SCHED_ALLPAIRS;
    bool have_floes = false;
    std::vector<int32_t> start_h;
    std::vector<int32_t> counts_h;
    std::vector<int32_t> order_h;       // cells by floe count, largest first (stable)
    int32_t* empty_d = nullptr;         // cells without floes: no DEM work, continuum update only
    int nempty = 0;
    Bucket bk[kNumBuckets];
    float r_bin = 0.0f;         // largest radius the sub-bins are sized for
    float skin = 0.0f;          // candidate-list skin (m)
    float skin_set = 0.0f;      // the skin planned for the floes as set (re-plans stay below it)
    struct HybridState* hyb = nullptr;

    // device buffers
    uint32_t *xi = nullptr, *yi = nullptr;
    float *u = nullptr, *v = nullptr, *w = nullptr, *th = nullptr, *r = nullptr, *h = nullptr;
    int32_t* cell_start = nullptr;
    double2* phase = nullptr;
    double* ocen = nullptr;                 // [ncells][4]: ocean u, v and curl at each cell centre, 0
    double* momb[2] = {nullptr, nullptr};   // statistics of time level k in momb[k & 1]
    double* mom2 = nullptr;                 // statistics of the current state (read_moments)
    double* Q[2] = {nullptr, nullptr};      // continuum of time level k in Q[k & 1]
    uint32_t* err_d = nullptr;
    unsigned long long* contacts_d = nullptr;
    unsigned long long* cands_d = nullptr;  // candidate tests per cell (blocked steps)
    unsigned long long* cfl_bits_d = nullptr;
    float* desc = nullptr;                  // closure descriptors [ncells][6] (lazy)
    bool desc_stale = false;                // radii changed since desc and mf were computed
    double* mf = nullptr;                   // mean-field drag coefficients [ncells][4] (with desc)
    double* red = nullptr;                  // reduced DEM of every cell [ncells][4]
    double t_now = 0.0;                     // time of the current state since the floes were set
    double* qprev = nullptr;                // continuum snapshot for tendencies
    uint16_t* vlist = nullptr;              // candidate lists [n][kListCap], entry-major per cell
    uint8_t* vcount = nullptr;              // candidates per floe [n]
    uint4* tsp_j = nullptr;                 // tangential spring history (SP_TANGENTIAL_SPRING): partners [n]
    double* tsp_x = nullptr;                //   and displacements [n][SP_SPRING_CAP]
    float* vdisp = nullptr;                 // per-cell displacement bound since the lists were built

    // time stepping
    int64_t kstep = 0;          // DEM steps since the floes were set
    bool lf_pending = false;    // the continuum update of level kstep - 1 is still to run
    double lf_dt = 0.0;         // step size of that update
    int64_t steps = 0;

    // coupling cadence (Algorithm 1): coarse step of N0 fine steps in N1
    // sub-steps, coarse-to-fine updates every n_t fine steps
    int32_t N0 = 1, N1 = 1, n_t = 1;
    int64_t cpl_j = 0;                      // fine steps since the cadence was set
    int64_t cpl_nudges = 0;                 // coarse-to-fine update passes since then
    double* cpl_ring = nullptr;             // [N0][ncells][kMomStride] window statistics
    int32_t cpl_ring_slots = 0;
    double* cpl_mean = nullptr;             // [ncells][kMomStride] mean of the window
    double* cpl_x0 = nullptr;               // [ncells][kMomStride] statistics at the coarse-step start
    int32_t* cpl_cells = nullptr;           // cells with floes
    int32_t cpl_ncl = 0;
    unsigned long long* cpl_count = nullptr;   // clamped, invalid cell updates
    unsigned int* cpl_rreq = nullptr;       // radius the next coarse step's updates may reach (float bits)
    int64_t cpl_replans = 0;                // contact-search re-plans at coarse steps

    // temporal blocking of the plain step: K steps per DEM launch (1: per step)
    int32_t block_k = kDefaultStepBlock;
    double* blk_ring = nullptr;             // [2][block_k][ncells][kMomStride] statistics of two blocks' steps
    int32_t blk_ring_slots = 0;
    int blk_parity = 0;                     // ring half of the next block
    hipStream_t lf_stream = nullptr;        // continuum updates of blocks (default priority)
    hipStream_t bk_stream = nullptr;        // blocked launches of the smaller buckets (default priority)
    hipEvent_t bk_fork = nullptr, bk_join = nullptr;
    hipEvent_t dem_done[2] = {nullptr, nullptr};
    hipEvent_t lf_done[2] = {nullptr, nullptr};
    bool lf_used[2] = {false, false};       // lf_done[i] was recorded
    int lf_last = -1;                       // ring half whose updates were enqueued last, not yet joined
    int64_t blk_steps = 0;                  // steps taken in blocks since the floes were set

    // graph replay
    int graph_chunk = kDefaultGraphChunk;
    bool graph_ok = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double graph_dt = 0.0;
};

// Scratch of sp_read_moments_noalloc: the statistics rows of up to
// kNoAllocMaxCells cells (8 MiB), one copy per device for the life of the
// process.  Host code never names it: it uses the device address taken by
// hipGetSymbolAddress when a context is created on that device.
constexpr int kNoAllocMaxCells = 65536;
static __device__ __align__(256) double scratch[(size_t)kNoAllocMaxCells * kMomStride];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, the current device (taken once
// per device).
hipError_t scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
    return hipSuccess;
}

double* scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// Continuum rows: out[c][f] = Q[f][c].
__global__ __launch_bounds__(256) void q_rows_kernel(const double* Q, int nc, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc * 4) out[i] = Q[(size_t)(i & 3) * nc + (i >> 2)];
}
}  // namespace

void hybrid_free(sp_ctx* c);   // hybrid_host.h
sp_status coupled_steps(sp_ctx* c, const StepArgs& base, int64_t nsteps);   // coupling_host.h

namespace {
sp_status init_reduced_all(sp_ctx* c, const double* mom);   // closure_host.h
sp_status refresh_reduced_all(sp_ctx* c);
void coupling_free(sp_ctx* c);                              // coupling_host.h
}  // namespace

namespace {

// Dirichlet boundary in x of the coarse model (SP_WALL_X).
int wall_x(const sp_ctx* c) { return (c->p.flags & SP_WALL_X) ? 1 : 0; }

sp_status fail(sp_ctx* ctx, sp_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

// A failing HIP call also leaves its code as the thread's last error; clear it
// so that a later launch check does not report it again.
#define HIP_TRY(ctx, expr)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return fail((ctx), SP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));            \
        }                                                                                      \
    } while (0)

#define SP_TRY(expr)                 \
    do {                             \
        sp_status s_ = (expr);       \
        if (s_ != SP_OK) return s_;  \
    } while (0)

template <class T>
sp_status dalloc(sp_ctx* ctx, T** p, size_t count)
{
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, SP_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
    }
    return SP_OK;
}

void drop_graph(sp_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

void free_all(sp_ctx* c)
{
    drop_graph(c);
    hybrid_free(c);
    coupling_free(c);
    void* ps[] = {c->xi, c->yi, c->u, c->v, c->w, c->th, c->r, c->h, c->cell_start, c->phase, c->ocen,
                  c->momb[0], c->momb[1], c->mom2, c->Q[0], c->Q[1], c->err_d, c->contacts_d,
                  c->cfl_bits_d, c->desc, c->mf, c->red, c->qprev, c->vlist, c->vcount, c->vdisp, c->empty_d,
                  c->blk_ring, c->cands_d, c->tsp_j, c->tsp_x};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    for (auto& b : c->bk) {
        if (b.work_d) (void)hipFree(b.work_d);
        b.work_d = nullptr;
    }
    c->xi = c->yi = nullptr;
    c->u = c->v = c->w = c->th = c->r = c->h = nullptr;
    c->cell_start = nullptr;
    c->phase = nullptr;
    c->ocen = nullptr;
    c->momb[0] = c->momb[1] = c->mom2 = nullptr;
    c->Q[0] = c->Q[1] = nullptr;
    c->err_d = nullptr;
    c->contacts_d = c->cfl_bits_d = nullptr;
    c->desc = nullptr;
    c->mf = nullptr;
    c->red = nullptr;
    c->qprev = nullptr;
    c->vlist = nullptr;
    c->vcount = nullptr;
    c->tsp_j = nullptr;
    c->tsp_x = nullptr;
    c->vdisp = nullptr;
    c->empty_d = nullptr;
    c->nempty = 0;
    c->blk_ring = nullptr;
    c->blk_ring_slots = 0;
    c->cands_d = nullptr;
}

// LDS bytes of one group (one cell) for a schedule, capacity and W.
size_t group_bytes(int sched, int cap, int nb, int waves)
{
    size_t b = (size_t)cap * (16 + 16 + 2 * kListCap + 4);
    if (sched == SP_SCHED_BINNED) b += (size_t)cap * 16 + (size_t)(2 * nb + 1) * 4;   // sorted copy, bins
    b = std::max(b, (size_t)kDyn * 64 * waves * sizeof(double));   // reduction buffer
    return (b + 15) & ~(size_t)15;
}

// LDS a multi-group workgroup may use (one group per workgroup may use more).
constexpr size_t kLdsBudget = 65536;

// Cells per workgroup: up to 4 / W for W < 4, fewer when their LDS would not fit.
int groups_per_block(int waves, size_t gbytes)
{
    if (waves >= 4) return 1;
    const int mx = 4 / waves;
    return std::max(1, std::min(mx, (int)(kLdsBudget / std::max<size_t>(gbytes, 1))));
}

StepArgs make_args(const sp_ctx* c, double dt)
{
    StepArgs a;
    memset(&a, 0, sizeof a);
    a.xi = c->xi;
    a.yi = c->yi;
    a.u = c->u;
    a.v = c->v;
    a.w = c->w;
    a.th = c->th;
    a.r = c->r;
    a.h = c->h;
    a.cell_start = c->cell_start;
    a.phase = c->phase;
    a.vlist = c->vlist;
    a.vcount = c->vcount;
    a.tsp_j = c->tsp_j;
    a.tsp_x = c->tsp_x;
    a.vdisp = c->vdisp;
    a.skin = c->skin;
    a.err = c->err_d;
    a.contacts = c->contacts_d;
    a.cands = c->cands_d;
    a.max_cfl_bits = c->cfl_bits_d;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.dX = c->p.cell_lx;
    a.dY = c->p.cell_ly;
    a.inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    a.ncells = c->ncells;
    a.nmodes = c->nmodes;
    a.nbx = c->nbx;
    a.nby = c->nby;
    a.flags = c->p.flags;
    a.qxd = c->p.cell_lx * 0x1.0p-32;
    a.qyd = c->p.cell_ly * 0x1.0p-32;
    a.qx = (float)a.qxd;
    a.qy = (float)a.qyd;
    a.inv_qxd = 0x1.0p32 / c->p.cell_lx;
    a.inv_qyd = 0x1.0p32 / c->p.cell_ly;
    a.dtd = dt;
    a.Ed = c->p.E;
    a.Gd = c->p.G;
    a.mud = c->p.mu;
    a.rho_ice_d = c->p.rho_ice;
    a.cdrho = c->p.cd * c->p.rho_ocean;
    a.u0 = c->u0;
    a.v0 = c->v0;
    for (int m = 0; m < c->nmodes; ++m) {
        a.modes.kxL[m] = (float)(c->kx[m] * c->p.cell_lx);
        a.modes.kyL[m] = (float)(c->ky[m] * c->p.cell_ly);
        a.modes.au[m] = c->au[m];
        a.modes.av[m] = c->av[m];
        a.modes.cz[m] = c->av[m] * c->kx[m] - c->au[m] * c->ky[m];
    }
    // phase offsets within a cell stay inside [-1.6, 1.6]: sin and cos
    // straight from their polynomials (no range reduction)
    float reach = 0.0f;
    for (int m = 0; m < c->nmodes; ++m)
        reach = std::max(reach, 0.5f * (fabsf(a.modes.kxL[m]) + fabsf(a.modes.kyL[m])));
    a.modes.direct = reach <= 1.6f ? 1 : 0;
    return a;
}

sp_status upload_ocean_centres(sp_ctx* c);

sp_status upload_phase(sp_ctx* c)
{
    if (!c->phase_dirty || c->ncells == 0) return SP_OK;
    const int nm = c->nmodes > 0 ? c->nmodes : 1;
    std::vector<double2> tab((size_t)c->ncells * nm, make_double2(0.0, 1.0));
    for (int cell = 0; cell < c->ncells; ++cell) {
        const double Xc = ((double)(cell % c->p.nx) + 0.5) * c->p.cell_lx;
        const double Yc = ((double)(cell / c->p.nx) + 0.5) * c->p.cell_ly;
        for (int m = 0; m < c->nmodes; ++m) {
            const double t = c->kx[m] * Xc + c->ky[m] * Yc + c->ph[m];
            tab[(size_t)cell * nm + m] = make_double2(sin(t), cos(t));
        }
    }
    SP_TRY(dalloc(c, &c->phase, tab.size()));
    HIP_TRY(c, hipMemcpyAsync(c->phase, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice,
                              c->stream));
    SP_TRY(upload_ocean_centres(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->phase_dirty = false;
    drop_graph(c);
    return SP_OK;
}

// Mark the candidate lists of every cell (cells == null) or of the listed
// cells stale: their next step rebuilds them.
__global__ void invalidate_lists_kernel(float* vdisp, const int32_t* cells, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) vdisp[cells ? cells[i] : i] = __int_as_float(0x7f800000);   // +inf
}

sp_status invalidate_lists(sp_ctx* c, const int32_t* cells_d, int n)
{
    if (!c->vdisp || n <= 0) return SP_OK;
    hipLaunchKernelGGL(invalidate_lists_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->vdisp, cells_d, n);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

sp_status check_device_err(sp_ctx* c)
{
    uint32_t e = 0;
    HIP_TRY(c, hipMemcpyAsync(&e, c->err_d, sizeof e, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!e) return SP_OK;
    if (e & kErrOverlap) return fail(c, SP_EOVERLAP, "coincident floe centres in contact");
    if (e & kErrNaN) return fail(c, SP_ENAN, "non-finite floe state");
    if (e & kErrCapacity) return fail(c, SP_ECAPACITY, "more than %d contacts on one floe", kListCap);
    if (e & kErrWall) return fail(c, SP_EWALL, "a floe crossed a wall");
    return fail(c, SP_ECFL, "continuum CFL number exceeded 1");
}

// --------------------------------------------------------- kernel launches
template <int SCHED, int W, bool PERSIST>
sp_status launch_t(sp_ctx* c, const StepArgs& a, int grid, int threads, size_t lds)
{
    if (a.flags & SP_TANGENTIAL_SPRING) {   // one workgroup per cell group (launch_bucket's grid)
        if (a.cap <= 64 * W)
            hipLaunchKernelGGL((dem_step_kernel<SCHED, W, false, true, true>), dim3(grid), dim3(threads), lds,
                               c->stream, a);
        else
            hipLaunchKernelGGL((dem_step_kernel<SCHED, W, false, false, true>), dim3(grid), dim3(threads), lds,
                               c->stream, a);
    } else if (a.cap <= 64 * W)   // one floe per lane
        hipLaunchKernelGGL((dem_step_kernel<SCHED, W, PERSIST, true>), dim3(grid), dim3(threads), lds, c->stream, a);
    else
        hipLaunchKernelGGL((dem_step_kernel<SCHED, W, PERSIST, false>), dim3(grid), dim3(threads), lds, c->stream, a);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

template <int SCHED, int W, bool PERSIST>
sp_status prepare_t(sp_ctx* c, int threads, size_t lds, int cap, int* resident)
{
    const int BT = threads;
    const void* k = cap <= 64 * W ? (const void*)dem_step_kernel<SCHED, W, PERSIST, true>
                                  : (const void*)dem_step_kernel<SCHED, W, PERSIST, false>;
    if (lds > 65536) HIP_TRY(c, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, BT, lds));
    if (resident) *resident = std::max(1, per_cu) * c->num_cus;
    return SP_OK;
}

#define SP_DISPATCH(FN, ...)                                                                  \
    switch ((sched == SP_SCHED_BINNED ? 100 : 0) + waves * 2 + (persist ? 1 : 0)) {              \
    case 2: return FN<1, 1, false>(__VA_ARGS__);                                               \
    case 3: return FN<1, 1, true>(__VA_ARGS__);                                                \
    case 4: return FN<1, 2, false>(__VA_ARGS__);                                               \
    case 5: return FN<1, 2, true>(__VA_ARGS__);                                                \
    case 8: return FN<1, 4, false>(__VA_ARGS__);                                               \
    case 9: return FN<1, 4, true>(__VA_ARGS__);                                                \
    case 16: return FN<1, 8, false>(__VA_ARGS__);                                              \
    case 17: return FN<1, 8, true>(__VA_ARGS__);                                               \
    case 102: return FN<2, 1, false>(__VA_ARGS__);                                             \
    case 103: return FN<2, 1, true>(__VA_ARGS__);                                              \
    case 104: return FN<2, 2, false>(__VA_ARGS__);                                             \
    case 105: return FN<2, 2, true>(__VA_ARGS__);                                              \
    case 108: return FN<2, 4, false>(__VA_ARGS__);                                             \
    case 109: return FN<2, 4, true>(__VA_ARGS__);                                              \
    case 116: return FN<2, 8, false>(__VA_ARGS__);                                             \
    case 117: return FN<2, 8, true>(__VA_ARGS__);                                              \
    default: return fail(c, SP_EINVAL, "no kernel for waves=%d", waves);                      \
    }

sp_status launch_sel(sp_ctx* c, int sched, int waves, int persist, const StepArgs& a, int grid, int threads,
                     size_t lds)
{
    SP_DISPATCH(launch_t, c, a, grid, threads, lds)
}

sp_status prepare_sel(sp_ctx* c, int sched, int waves, int persist, int threads, size_t lds, int cap,
                      int* resident)
{
    SP_DISPATCH(prepare_t, c, threads, lds, cap, resident)
}

template <int SCHED, int W, bool TSP>
sp_status launch_block_tt(sp_ctx* c, hipStream_t st, const StepArgs& a, int grid, int threads, size_t lds, int K,
                          const BlockNudge& nd)
{
    if (lds > 65536)
        HIP_TRY(c, hipFuncSetAttribute((const void*)dem_block_kernel<SCHED, W, TSP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((dem_block_kernel<SCHED, W, TSP>), dim3(grid), dim3(threads), lds, st, a, K, nd);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

template <int SCHED, int W>
sp_status launch_block_t(sp_ctx* c, hipStream_t st, const StepArgs& a, int grid, int threads, size_t lds, int K,
                         const BlockNudge& nd)
{
    if (a.flags & SP_TANGENTIAL_SPRING) return launch_block_tt<SCHED, W, true>(c, st, a, grid, threads, lds, K, nd);
    return launch_block_tt<SCHED, W, false>(c, st, a, grid, threads, lds, K, nd);
}

sp_status launch_block_sel(sp_ctx* c, hipStream_t st, int sched, int waves, const StepArgs& a, int grid,
                           int threads, size_t lds, int K, const BlockNudge& nd)
{
    const bool binned = sched == SP_SCHED_BINNED;
    switch (waves) {
    case 1: return binned ? launch_block_t<2, 1>(c, st, a, grid, threads, lds, K, nd) : launch_block_t<1, 1>(c, st, a, grid, threads, lds, K, nd);
    case 2: return binned ? launch_block_t<2, 2>(c, st, a, grid, threads, lds, K, nd) : launch_block_t<1, 2>(c, st, a, grid, threads, lds, K, nd);
    case 4: return binned ? launch_block_t<2, 4>(c, st, a, grid, threads, lds, K, nd) : launch_block_t<1, 4>(c, st, a, grid, threads, lds, K, nd);
    case 8: return binned ? launch_block_t<2, 8>(c, st, a, grid, threads, lds, K, nd) : launch_block_t<1, 8>(c, st, a, grid, threads, lds, K, nd);
    case 16: return binned ? launch_block_t<2, 16>(c, st, a, grid, threads, lds, K, nd) : launch_block_t<1, 16>(c, st, a, grid, threads, lds, K, nd);
    default: return fail(c, SP_EINVAL, "no blocked kernel for waves=%d", waves);
    }
}

size_t bucket_group_bytes(const sp_ctx* c, const Bucket& b)
{
    return group_bytes(c->sched, b.cap, c->nbx * c->nby, b.waves);
}

int bucket_gpb(const sp_ctx* c, const Bucket& b) { return groups_per_block(b.waves, bucket_group_bytes(c, b)); }

size_t bucket_lds(const sp_ctx* c, const Bucket& b) { return (size_t)bucket_gpb(c, b) * bucket_group_bytes(c, b); }

int bucket_threads(const sp_ctx* c, const Bucket& b) { return bucket_gpb(c, b) * 64 * b.waves; }

sp_status prepare_bucket(sp_ctx* c, Bucket& b)
{
    return prepare_sel(c, c->sched, b.waves, b.persist, bucket_threads(c, b), bucket_lds(c, b), b.cap, &b.resident);
}

// One DEM launch for bucket b at time level k (writes the statistics of level
// k); with lf, the continuum update of level k - 1 runs in the same launch.
// `fixed` (autotuning) supplies every buffer pointer itself; mom_to (coupled
// cadence) takes the statistics instead, with no continuum update.
sp_status launch_bucket(sp_ctx* c, const Bucket& b, const StepArgs& base, int64_t k, bool lf,
                        bool fixed = false, double* mom_to = nullptr)
{
    if (b.cells_h.empty()) return SP_OK;
    StepArgs a = base;
    a.work = b.work_d;
    a.ncl = (int32_t)b.cells_h.size();
    a.cap = b.cap;
    a.group_bytes = (int32_t)bucket_group_bytes(c, b);
    if (!fixed) {
        a.mom = c->momb[k & 1];
        a.lf = lf ? 1 : 0;
        a.mom_prev = c->momb[(k + 1) & 1];
        a.Qp = c->Q[(k + 1) & 1];
        a.Qn = c->Q[k & 1];
        if (mom_to) {
            a.mom = mom_to;
            a.lf = 0;
        }
    }
    const int gpb = bucket_gpb(c, b);
    const int groups = (int)((b.cells_h.size() + gpb - 1) / gpb);
    // the tangential spring's kernels take one workgroup per cell group
    const bool persist = b.persist && !(c->p.flags & SP_TANGENTIAL_SPRING);
    const int grid = persist ? std::min(groups, b.resident) : groups;
    return launch_sel(c, c->sched, b.waves, persist, a, grid, bucket_threads(c, b), bucket_lds(c, b));
}

// Wavefronts per cell of a bucket's blocked launches: the autotuner's choice
// where it made one, else the bucket's own W when its cells have at most 64 W
// floes, else the smallest of 8 and 16 that holds one floe per lane (up to the
// 1024-floe cell limit).
int block_waves(const Bucket& b)
{
    if (b.bwaves > 0 && b.cap <= 64 * b.bwaves) return b.bwaves;
    if (b.cap <= 64 * b.waves) return b.waves;
    return b.cap <= 512 ? 8 : 16;
}

// LDS of one cell of a blocked launch: the per-step layout, 1 / m and
// 1 / (m r^2) per floe beside the state, and with the tangential spring the
// floes' contact history.
constexpr size_t kBlockLdsMax = 160 * 1024;

size_t block_group_bytes(const sp_ctx* c, int cap, int waves)
{
    size_t b = group_bytes(c->sched, cap, c->nbx * c->nby, waves) + (size_t)cap * 16;
    if (c->p.flags & SP_TANGENTIAL_SPRING) b += (size_t)cap * kSpringBytes;
    return b;
}

// K steps from level kstep as one blocked launch per bucket (of bk, default the
// context's buckets), the statistics of step t into mom + t * (ncells x
// kMomStride) (work entries flagged for mom_alt: there); with an active nd, the
// coarse-to-fine update of every launched cell at the end.
sp_status launch_blocks(sp_ctx* c, const StepArgs& base, double* mom, int K, const BlockNudge& nd,
                        const Bucket* bk = nullptr, hipStream_t on = nullptr)
{
    if (!bk) bk = c->bk;
    const hipStream_t s0 = on ? on : c->stream;   // the stream the launches follow and that waits for them
    // with several buckets, the one of most floes on the library stream and
    // the others beside it on a second stream (their cells are disjoint; the
    // library stream waits for both)
    int main_q = -1, nb = 0;
    int64_t most = -1;
    for (int q = 0; q < kNumBuckets; ++q) {   // every bucket checked before any launch
        const Bucket& b = bk[q];
        if (b.cells_h.empty()) continue;
        const int w = block_waves(b);
        if (b.cap > 64 * w) return fail(c, SP_EINVAL, "%d floes per cell exceed a blocked launch", b.cap);
        if (block_group_bytes(c, b.cap, w) > kBlockLdsMax)
            return fail(c, SP_ECAPACITY, "%d floes per cell exceed the LDS of a blocked launch", b.cap);
        ++nb;
        const int64_t f = (int64_t)bk[q].cells_h.size() * bk[q].cap;
        if (f > most) {
            most = f;
            main_q = q;
        }
    }
    if (nb > 1) {
        if (!c->bk_stream) {
            HIP_TRY(c, hipStreamCreateWithFlags(&c->bk_stream, hipStreamNonBlocking));
            HIP_TRY(c, hipEventCreateWithFlags(&c->bk_fork, hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->bk_join, hipEventDisableTiming));
        }
        HIP_TRY(c, hipEventRecord(c->bk_fork, s0));
        HIP_TRY(c, hipStreamWaitEvent(c->bk_stream, c->bk_fork, 0));
    }
    sp_status status = SP_OK;
    for (int q = 0; q < kNumBuckets; ++q) {
        const Bucket& b = bk[q];
        if (b.cells_h.empty()) continue;
        const hipStream_t st = (nb > 1 && q != main_q) ? c->bk_stream : s0;
        const int w = block_waves(b);
        const size_t gbytes = block_group_bytes(c, b.cap, w);
        const int gpb = groups_per_block(w, gbytes);
        StepArgs a = base;
        a.work = b.work_d;
        a.ncl = (int32_t)b.cells_h.size();
        a.cap = b.cap;
        a.group_bytes = (int32_t)gbytes;
        a.mom = mom;
        a.lf = 0;
        const int grid = (int)((b.cells_h.size() + gpb - 1) / gpb);
        status = launch_block_sel(c, st, c->sched, w, a, grid, gpb * 64 * w, (size_t)gpb * gbytes, K, nd);
        if (status) break;
    }
    if (nb > 1) {   // joined also after a failed launch: nothing stays behind on the second stream
        HIP_TRY(c, hipEventRecord(c->bk_join, c->bk_stream));
        HIP_TRY(c, hipStreamWaitEvent(s0, c->bk_join, 0));
    }
    return status;
}

sp_status launch_empty_lf(sp_ctx* c, const StepArgs& base, int64_t k);

sp_status step_once(sp_ctx* c, const StepArgs& base)
{
    const bool lf = c->lf_pending;
    for (auto& b : c->bk) SP_TRY(launch_bucket(c, b, base, c->kstep, lf));
    if (lf) SP_TRY(launch_empty_lf(c, base, c->kstep));
    c->kstep++;
    c->lf_pending = !(c->p.flags & SP_NO_CONTINUUM);
    c->lf_dt = base.dtd;
    c->steps++;
    return SP_OK;
}

// Continuum update of level kstep - 1 if it is still pending.
sp_status flush_lf(sp_ctx* c)
{
    if (!c->lf_pending) return SP_OK;
    const int64_t k = c->kstep - 1;
    hipLaunchKernelGGL(lf_kernel, dim3((c->ncells + 63) / 64), dim3(64), 0, c->stream, c->momb[k & 1],
                       c->Q[k & 1], c->Q[(k + 1) & 1], c->p.nx, c->p.ny, c->lf_dt, c->p.cell_lx,
                       c->p.cell_ly, 1.0 / (c->p.cell_lx * c->p.cell_ly), c->cfl_bits_d, c->err_d, wall_x(c));
    HIP_TRY(c, hipGetLastError());
    c->lf_pending = false;
    return SP_OK;
}

// Blocked plain steps apply with a block length above one, the plain cadence
// and no hybrid (the coupled cadence and the hybrid block on their own terms).
bool block_eligible(const sp_ctx* c)
{
    if (!(c->block_k > 1 && c->N0 == 1 && !c->hyb)) return false;
    // with the tangential spring, while every bucket's cells fit a blocked launch's LDS
    if (c->p.flags & SP_TANGENTIAL_SPRING)
        for (const auto& b : c->bk)
            if (!b.cells_h.empty() && block_group_bytes(c, b.cap, block_waves(b)) > kBlockLdsMax) return false;
    return true;
}

// Make the library stream wait for the continuum updates of the last block
// (they run on a stream of their own, beside the next block's DEM launch).
sp_status join_block_lf(sp_ctx* c)
{
    if (c->lf_last < 0) return SP_OK;
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->lf_done[c->lf_last], 0));
    c->lf_last = -1;
    return SP_OK;
}

// Statistics ring (two halves of block_k slots, zero rows for cells without
// floes), update stream and events of blocked steps; allocated before the
// first block (sp_set_floes, sp_set_step_block), so that no timed step pays it.
sp_status block_prepare(sp_ctx* c)
{
    const int K = c->block_k;
    const size_t slot = (size_t)c->ncells * kMomStride;
    if (!c->blk_ring || c->blk_ring_slots != K) {
        SP_TRY(join_block_lf(c));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        SP_TRY(dalloc(c, &c->blk_ring, 2 * slot * (size_t)K));
        HIP_TRY(c, hipMemsetAsync(c->blk_ring, 0, 2 * slot * (size_t)K * 8, c->stream));
        c->blk_ring_slots = K;
        c->lf_used[0] = c->lf_used[1] = false;
    }
    if (!c->lf_stream) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->lf_stream, hipStreamNonBlocking));
        for (int i = 0; i < 2; ++i) {
            HIP_TRY(c, hipEventCreateWithFlags(&c->dem_done[i], hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->lf_done[i], hipEventDisableTiming));
        }
    }
    return SP_OK;
}

// One blocked launch per bucket: K steps (1 <= K <= block_k) of the plain
// path from level kstep, statistics of step t into slot t of one half of the
// ring; then the K continuum updates on the update stream, which overlap the
// next block's DEM launch (that launch writes the other half; a half is
// written again only after its updates are done).  A run shorter than a block
// is one launch of its own length, so every plain step of an eligible context
// is blocked.
sp_status block_chunk(sp_ctx* c, const StepArgs& base, int K, bool time_dem = false, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr)
{
    const size_t slot = (size_t)c->ncells * kMomStride;
    SP_TRY(block_prepare(c));
    if (K < 1 || K > c->blk_ring_slots) return fail(c, SP_EINVAL, "block of %d steps outside [1, %d]", K, c->blk_ring_slots);
    SP_TRY(flush_lf(c));
    const int r = c->blk_parity;
    double* const ring = c->blk_ring + (size_t)r * c->blk_ring_slots * slot;
    if (c->lf_used[r]) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->lf_done[r], 0));
    if (time_dem) HIP_TRY(c, hipEventRecord(e0, c->stream));
    BlockNudge none;
    memset(&none, 0, sizeof none);
    SP_TRY(launch_blocks(c, base, ring, K, none));
    if (time_dem) HIP_TRY(c, hipEventRecord(e1, c->stream));
    if (!(c->p.flags & SP_NO_CONTINUUM)) {
        // everything enqueued on the library stream so far (this block's
        // statistics, earlier continuum work) precedes the updates
        HIP_TRY(c, hipEventRecord(c->dem_done[r], c->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->lf_stream, c->dem_done[r], 0));
        for (int t = 0; t < K; ++t) {
            const int64_t k = c->kstep + t;
            hipLaunchKernelGGL(lf_kernel, dim3((c->ncells + 63) / 64), dim3(64), 0, c->lf_stream, ring + t * slot,
                               c->Q[k & 1], c->Q[(k + 1) & 1], c->p.nx, c->p.ny, base.dtd, c->p.cell_lx,
                               c->p.cell_ly, base.inv_area, c->cfl_bits_d, c->err_d, wall_x(c));
            HIP_TRY(c, hipGetLastError());
        }
        HIP_TRY(c, hipEventRecord(c->lf_done[r], c->lf_stream));
        c->lf_used[r] = true;
        c->lf_last = r;
    }
    c->blk_parity = r ^ 1;
    c->kstep += K;
    c->steps += K;
    c->blk_steps += K;
    c->lf_pending = false;
    return SP_OK;
}

sp_status prepare_buckets(sp_ctx* c)
{
    for (auto& b : c->bk) {
        if (b.cells_h.empty()) continue;
        SP_TRY(prepare_bucket(c, b));
    }
    return SP_OK;
}

// Count buckets over the cells with include[cell] != 0 (all cells if null),
// costliest first (the order fixed when the floes were set); counts must be
// the context's counts.  alt (per cell, may be null): 1 sends a cell's
// statistics to mom_alt.  Work lists keep their device buffers while they fit.
sp_status build_buckets_into(sp_ctx* c, Bucket* bk, const int32_t* counts, const uint8_t* include,
                             const uint8_t* alt = nullptr)
{
    for (int q = 0; q < kNumBuckets; ++q) bk[q].cells_h.clear();
    for (int32_t cell : c->order_h) {
        if (include && !include[cell]) continue;
        int q = 0;
        while (counts[cell] > kBucketHi[q]) ++q;
        bk[q].cells_h.push_back(cell);
    }
    std::vector<int4> work[kNumBuckets];
    for (int q = 0; q < kNumBuckets; ++q) {
        Bucket& b = bk[q];
        int mx = 0;
        for (int32_t cell : b.cells_h) mx = std::max(mx, counts[cell]);
        b.cap = std::max(16, (mx + 15) / 16 * 16);
        work[q].resize(b.cells_h.size());
        for (size_t i = 0; i < work[q].size(); ++i) {
            const int32_t cell = b.cells_h[i];
            work[q][i] = make_int4(cell, c->start_h[cell], counts[cell], alt ? (int)alt[cell] : 0);
        }
        if (!b.work_d || work[q].size() > b.work_cap) {
            b.work_cap = std::max<size_t>(1, work[q].size());
            SP_TRY(dalloc(c, &b.work_d, b.work_cap));
        }
        if (!work[q].empty())
            HIP_TRY(c, hipMemcpyAsync(b.work_d, work[q].data(), work[q].size() * sizeof(int4),
                                      hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));   // `work` is a host temporary
    return SP_OK;
}

// Buckets of the cells with floes, and the list of the others.
sp_status build_buckets(sp_ctx* c, const int32_t* counts)
{
    std::vector<uint8_t> has(c->ncells);
    std::vector<int32_t> empty;
    for (int i = 0; i < c->ncells; ++i) {
        has[i] = counts[i] > 0;
        if (!has[i]) empty.push_back(i);
    }
    c->nempty = (int)empty.size();
    SP_TRY(dalloc(c, &c->empty_d, std::max<size_t>(1, empty.size())));
    if (!empty.empty())
        HIP_TRY(c, hipMemcpyAsync(c->empty_d, empty.data(), empty.size() * 4, hipMemcpyHostToDevice, c->stream));
    SP_TRY(build_buckets_into(c, c->bk, counts, has.data()));   // synchronises
    return SP_OK;
}

// The continuum update of level k - 1 for the cells without floes (the DEM
// launches of step k do it for the others).
sp_status launch_empty_lf(sp_ctx* c, const StepArgs& base, int64_t k)
{
    if (c->nempty == 0) return SP_OK;
    hipLaunchKernelGGL(lf_list_kernel, dim3((c->nempty + 63) / 64), dim3(64), 0, c->stream, c->empty_d, c->nempty,
                       c->momb[(k + 1) & 1], c->Q[(k + 1) & 1], c->Q[k & 1], c->p.nx, c->p.ny, base.dtd,
                       c->p.cell_lx, c->p.cell_ly, base.inv_area, c->cfl_bits_d, c->err_d, wall_x(c));
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

sp_status reset_continuum(sp_ctx* c)
{
    StepArgs a = make_args(c, 0.0);
    a.mom = c->momb[0];
    if (c->ncells > 0) {
        hipLaunchKernelGGL(stats_kernel, dim3(c->ncells), dim3(256), 0, c->stream, a, nullptr, 0);
        HIP_TRY(c, hipGetLastError());
        // the static statistics (n, M, A_ice) must be present at both levels
        HIP_TRY(c, hipMemcpyAsync(c->momb[1], c->momb[0], (size_t)c->ncells * kMomStride * 8,
                                  hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(q_from_moments_kernel, dim3((c->ncells + 255) / 256), dim3(256), 0, c->stream,
                           c->momb[0], c->Q[0], c->ncells, 1.0 / (c->p.cell_lx * c->p.cell_ly));
        HIP_TRY(c, hipGetLastError());
        // both buffers: the coupled cadence keeps the coarse state in each
        HIP_TRY(c, hipMemcpyAsync(c->Q[1], c->Q[0], (size_t)c->ncells * 4 * 8, hipMemcpyDeviceToDevice,
                                  c->stream));
    }
    c->kstep = 0;
    c->lf_pending = false;
    c->cpl_j = 0;
    return SP_OK;
}

// Capture `graph_chunk` steady-state steps (entry: kstep even, continuum
// pending unless disabled) as one graph.
sp_status capture_graph(sp_ctx* c, double dt)
{
    drop_graph(c);
    const StepArgs base = make_args(c, dt);
    const bool cont = !(c->p.flags & SP_NO_CONTINUUM);
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        c->graph_ok = false;
        return SP_OK;
    }
    sp_status st = SP_OK;
    for (int i = 0; i < c->graph_chunk && !st; ++i) {
        for (auto& b : c->bk) {
            st = launch_bucket(c, b, base, i, cont);
            if (st) break;
        }
        if (!st && cont) st = launch_empty_lf(c, base, i);
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st) {
        // a launch the graph cannot hold (e.g. a workgroup above the graph's LDS
        // limit): keep stepping eagerly
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->graph_ok = false;
        c->err.clear();
        return SP_OK;
    }
    if (e != hipSuccess || !g) {
        (void)hipGetLastError();
        c->graph_ok = false;
        return SP_OK;
    }
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->gexec = nullptr;
        c->graph_ok = false;
        return SP_OK;
    }
    c->graph = g;
    c->graph_dt = dt;
    return SP_OK;
}

// Autotuning of blocked steps on a scratch copy of the state (`a` points at
// it): every non-empty bucket alone, over the wavefronts per cell that hold one
// floe per lane (W = 1 .. 16), then the block length over the whole step
// (16, 32, 64 steps); each variant one warm-up launch and the minimum of reps
// timed launches, per step.  Sets each bucket's bwaves and the block length.
constexpr int kTuneBlocks[3] = {16, 32, 64};

sp_status tune_blocked(sp_ctx* c, StepArgs a, int reps, hipEvent_t e0, hipEvent_t e1, double* total)
{
    double* smom = nullptr;
    unsigned long long* scands = nullptr;
    sp_status st = dalloc(c, &smom, (size_t)kTuneBlocks[2] * c->ncells * kMomStride);
    if (!st) st = dalloc(c, &scands, std::max<size_t>(1, (size_t)c->ncells));
    a.cands = scands;
    BlockNudge none;
    memset(&none, 0, sizeof none);
    auto time_blocks = [&](const Bucket* bk, int K, double* per_step) -> sp_status {
        SP_TRY(launch_blocks(c, a, smom, K, none, bk));   // warm-up (and list rebuilds)
        double best = 1e30;
        for (int r = 0; r < reps; ++r) {
            HIP_TRY(c, hipEventRecord(e0, c->stream));
            SP_TRY(launch_blocks(c, a, smom, K, none, bk));
            HIP_TRY(c, hipEventRecord(e1, c->stream));
            HIP_TRY(c, hipEventSynchronize(e1));
            float ms = 0.0f;
            HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, (double)ms / K);
        }
        *per_step = best;
        return SP_OK;
    };
    const int wv[5] = {1, 2, 4, 8, 16};
    double sum = 0.0;
    for (int q = 0; q < kNumBuckets && !st; ++q) {
        Bucket& b = c->bk[q];
        if (b.cells_h.empty()) continue;
        Bucket trial[kNumBuckets];
        trial[q].cap = b.cap;
        trial[q].waves = b.waves;
        trial[q].cells_h = b.cells_h;
        trial[q].work_d = b.work_d;
        double best = 1e30;
        int bw = block_waves(b);
        for (int wi = 0; wi < 5 && !st; ++wi) {
            if (b.cap > 64 * wv[wi]) continue;        // one floe per lane
            trial[q].bwaves = wv[wi];
            double t = 0.0;
            st = time_blocks(trial, c->block_k, &t);
            if (!st && t < best) {
                best = t;
                bw = wv[wi];
            }
        }
        trial[q].work_d = nullptr;    // owned by the real bucket
        if (!st) {
            b.bwaves = bw;
            sum += best;
        }
    }
    int bestK = c->block_k;
    double bestT = 1e30;
    for (int i = 0; i < 3 && !st; ++i) {
        double t = 0.0;
        st = time_blocks(c->bk, kTuneBlocks[i], &t);
        if (!st && t < bestT) {
            bestT = t;
            bestK = kTuneBlocks[i];
        }
    }
    (void)hipStreamSynchronize(c->stream);
    if (smom) (void)hipFree(smom);
    if (scands) (void)hipFree(scands);
    if (st) return st;
    c->block_k = bestK;
    *total = bestT < 1e30 ? bestT : sum;
    return SP_OK;
}

}  // namespace

extern "C" {

sp_status sp_create(const sp_params* params, void* stream, sp_ctx** out)
{
    if (!out) return SP_EINVAL;
    *out = nullptr;
    if (!params) return SP_EINVAL;
    const sp_params& p = *params;
    if (p.nx < 1 || p.ny < 1 || !(p.cell_lx > 0) || !(p.cell_ly > 0) || !(p.rho_ice > 0) ||
        !(p.rho_ocean >= 0) || !(p.cd >= 0) || !(p.E >= 0) || !(p.G >= 0) || !(p.mu >= 0) ||
        p.schedule < 0 || p.schedule > 2 || (int64_t)p.nx * p.ny > (1 << 30))
        return SP_EINVAL;
    sp_ctx* c = new sp_ctx();
    c->p = p;
    c->ncells = p.nx * p.ny;
    for (int q = 0; q < kNumBuckets; ++q) c->bk[q].waves = kDefaultWaves[q];
    (void)hipGetDevice(&c->device);
    {
        const hipError_t e = scratch_setup(c->device);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete c;
            return SP_EDEVICE;
        }
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
        c->num_cus = cus;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return SP_EDEVICE;
        }
        c->own_stream = true;
    }
    sp_status st = SP_OK;
    if (!st) st = dalloc(c, &c->err_d, 1);
    if (!st) st = dalloc(c, &c->contacts_d, std::max<size_t>(1, (size_t)c->ncells));
    if (!st) st = dalloc(c, &c->cands_d, std::max<size_t>(1, (size_t)c->ncells));
    if (!st) st = dalloc(c, &c->cfl_bits_d, 1);
    if (!st) st = dalloc(c, &c->momb[0], (size_t)c->ncells * kMomStride);
    if (!st) st = dalloc(c, &c->momb[1], (size_t)c->ncells * kMomStride);
    if (!st) st = dalloc(c, &c->mom2, (size_t)c->ncells * kMomStride);
    if (!st) st = dalloc(c, &c->Q[0], (size_t)c->ncells * 4);
    if (!st) st = dalloc(c, &c->Q[1], (size_t)c->ncells * 4);
    if (!st && hipMemsetAsync(c->err_d, 0, sizeof(uint32_t), c->stream) != hipSuccess) st = SP_EDEVICE;
    if (!st && hipMemsetAsync(c->contacts_d, 0, (size_t)c->ncells * 8, c->stream) != hipSuccess) st = SP_EDEVICE;
    if (!st && hipMemsetAsync(c->cands_d, 0, (size_t)c->ncells * 8, c->stream) != hipSuccess) st = SP_EDEVICE;
    if (!st && hipMemsetAsync(c->cfl_bits_d, 0, 8, c->stream) != hipSuccess) st = SP_EDEVICE;
    if (st) {
        sp_destroy(c);
        return st;
    }
    *out = c;
    return SP_OK;
}

void sp_destroy(sp_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->lf_stream) (void)hipStreamSynchronize(c->lf_stream);
    for (int i = 0; i < 2; ++i) {
        if (c->dem_done[i]) (void)hipEventDestroy(c->dem_done[i]);
        if (c->lf_done[i]) (void)hipEventDestroy(c->lf_done[i]);
    }
    if (c->lf_stream) (void)hipStreamDestroy(c->lf_stream);
    if (c->bk_stream) (void)hipStreamSynchronize(c->bk_stream);
    if (c->bk_fork) (void)hipEventDestroy(c->bk_fork);
    if (c->bk_join) (void)hipEventDestroy(c->bk_join);
    if (c->bk_stream) (void)hipStreamDestroy(c->bk_stream);
    free_all(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* sp_last_error(const sp_ctx* c)
{
    return c ? c->err.c_str() : "null context";
}

sp_status sp_set_ocean(sp_ctx* c, double u0, double v0, int32_t nmodes, const double* kx,
                       const double* ky, const double* au, const double* av, const double* phase)
{
    if (!c) return SP_EINVAL;
    if (nmodes < 0 || nmodes > SP_MAX_MODES)
        return fail(c, SP_EINVAL, "nmodes %d outside [0, %d]", nmodes, SP_MAX_MODES);
    if (nmodes > 0 && (!kx || !ky || !au || !av || !phase))
        return fail(c, SP_EINVAL, "null mode array");
    if (!std::isfinite(u0) || !std::isfinite(v0)) return fail(c, SP_EINVAL, "non-finite current");
    for (int m = 0; m < nmodes; ++m)
        if (!std::isfinite(kx[m]) || !std::isfinite(ky[m]) || !std::isfinite(au[m]) ||
            !std::isfinite(av[m]) || !std::isfinite(phase[m]))
            return fail(c, SP_EINVAL, "non-finite mode %d", m);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->u0 = u0;
    c->v0 = v0;
    c->nmodes = nmodes;
    for (int m = 0; m < nmodes; ++m) {
        c->kx[m] = kx[m];
        c->ky[m] = ky[m];
        c->au[m] = au[m];
        c->av[m] = av[m];
        c->ph[m] = phase[m];
    }
    c->phase_dirty = true;
    drop_graph(c);
    SP_TRY(upload_phase(c));
    if (c->have_floes) {
        // the reduced DEM is relative to the current: take it again from the floes
        SP_TRY(flush_lf(c));
        SP_TRY(refresh_reduced_all(c));
    }
    return SP_OK;
}

// Contact-search geometry for radii up to rmax: sub-bins, schedule, skin (at
// most skin_cap) and the radius limit of re-synchronisation; every cell's
// candidate lists are invalidated.
static sp_status plan_bins(sp_ctx* c, float rmax, bool any, double skin_cap = INFINITY)
{
    c->r_bin = rmax;
    // candidate lists are kept while the floes move less than half a skin of
    // at least kSkinFrac r_max; sub-bins of side >= 2 r_max + skin, and any
    // slack of the sub-bins goes to the skin
    const double skin0 = kSkinFrac * (double)rmax;
    int bx = any ? (int)floor(c->p.cell_lx / (2.0 * (double)rmax + skin0)) : 1;
    int by = any ? (int)floor(c->p.cell_ly / (2.0 * (double)rmax + skin0)) : 1;
    bx = std::min(bx, kMaxBinsSide);
    by = std::min(by, kMaxBinsSide);
    if (bx < 3) bx = 1;
    if (by < 3) by = 1;
    int sched = c->p.schedule;
    if (sched == SP_SCHED_AUTO) sched = (bx >= 3 || by >= 3) ? SP_SCHED_BINNED : SP_SCHED_ALLPAIRS;
    c->sched = sched;
    if (sched == SP_SCHED_BINNED) {
        c->nbx = bx;
        c->nby = by;
    } else {
        c->nbx = c->nby = 1;
    }
    // binned axes: all the slack of the sub-bins (at least skin0); an axis
    // searched whole sets no limit
    double skin = INFINITY;
    if (c->nbx >= 3) skin = std::min(skin, c->p.cell_lx / c->nbx - 2.0 * (double)rmax);
    if (c->nby >= 3) skin = std::min(skin, c->p.cell_ly / c->nby - 2.0 * (double)rmax);
    if (!std::isfinite(skin)) skin = skin0;
    skin = std::min(skin, skin_cap);
    // float rounding must not let a pair at the bin side escape the sweep
    c->skin = any ? (float)(skin * (1.0 - 1e-6)) : 0.0f;
    SP_TRY(invalidate_lists(c, nullptr, c->ncells));
    return SP_OK;
}

static sp_status set_floes_common(sp_ctx* c, int64_t n, const int32_t* counts, const void* const* src,
                                  hipMemcpyKind kind)
{
    if (!c) return SP_EINVAL;
    if (n < 0 || n > INT32_MAX || !counts) return fail(c, SP_EINVAL, "bad floe count or counts");
    int64_t tot = 0;
    int32_t mx = 0;
    for (int i = 0; i < c->ncells; ++i) {
        if (counts[i] < 0) return fail(c, SP_EINVAL, "negative count in cell %d", i);
        tot += counts[i];
        mx = std::max(mx, counts[i]);
    }
    if (tot != n) return fail(c, SP_EINVAL, "sum of counts %lld != n %lld", (long long)tot, (long long)n);
    if (mx > SP_MAX_CELL_FLOES)
        return fail(c, SP_ECAPACITY, "%d floes in one cell (max %d)", mx, SP_MAX_CELL_FLOES);
    for (int k = 0; k < 8; ++k)
        if (n > 0 && !src[k] && k != 4 && k != 5) return fail(c, SP_EINVAL, "null floe array %d", k);

    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    hybrid_free(c);   // its cell lists follow the floes
    coupling_free(c);   // so do the coupled cadence's
    c->cpl_nudges = 0;
    SP_TRY(join_block_lf(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->blk_ring) (void)hipFree(c->blk_ring);   // and the blocked steps' statistics
    c->blk_ring = nullptr;
    c->blk_ring_slots = 0;
    c->lf_used[0] = c->lf_used[1] = false;
    c->have_floes = false;
    if (c->desc) (void)hipFree(c->desc);   // descriptors follow the floes
    if (c->mf) (void)hipFree(c->mf);
    c->desc = nullptr;
    c->mf = nullptr;
    c->t_now = 0.0;
    const size_t N = (size_t)n;
    SP_TRY(dalloc(c, &c->xi, N));
    SP_TRY(dalloc(c, &c->yi, N));
    SP_TRY(dalloc(c, &c->u, N));
    SP_TRY(dalloc(c, &c->v, N));
    SP_TRY(dalloc(c, &c->w, N));
    SP_TRY(dalloc(c, &c->th, N));
    SP_TRY(dalloc(c, &c->r, N));
    SP_TRY(dalloc(c, &c->h, N));
    SP_TRY(dalloc(c, &c->cell_start, (size_t)c->ncells + 1));
    SP_TRY(dalloc(c, &c->vlist, std::max<size_t>(1, N) * kListCap));
    SP_TRY(dalloc(c, &c->vcount, std::max<size_t>(1, N)));
    if (c->p.flags & SP_TANGENTIAL_SPRING) {   // no contacts remembered yet
        SP_TRY(dalloc(c, &c->tsp_j, std::max<size_t>(1, N)));
        SP_TRY(dalloc(c, &c->tsp_x, std::max<size_t>(1, N) * SP_SPRING_CAP));
        HIP_TRY(c, hipMemsetAsync(c->tsp_j, 0xff, std::max<size_t>(1, N) * sizeof(uint4), c->stream));
        HIP_TRY(c, hipMemsetAsync(c->tsp_x, 0, std::max<size_t>(1, N) * SP_SPRING_CAP * 8, c->stream));
    }
    SP_TRY(dalloc(c, &c->vdisp, (size_t)c->ncells));
    void* dst[8] = {c->xi, c->yi, c->u, c->v, c->w, c->th, c->r, c->h};
    if (n > 0) {
        for (int k = 0; k < 8; ++k) {
            if (src[k]) {
                HIP_TRY(c, hipMemcpyAsync(dst[k], src[k], N * 4, kind, c->stream));
            } else {
                HIP_TRY(c, hipMemsetAsync(dst[k], 0, N * 4, c->stream));
            }
        }
    }
    // radius and thickness validation on a host copy
    std::vector<float> rh(N), hh(N);
    if (n > 0) {
        HIP_TRY(c, hipMemcpyAsync(rh.data(), c->r, N * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(hh.data(), c->h, N * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    float rmax = 0.0f;
    for (size_t i = 0; i < N; ++i) {
        if (!(rh[i] > 0.0f) || !std::isfinite(rh[i])) return fail(c, SP_EINVAL, "radius %zu not positive", i);
        if (!(hh[i] > 0.0f) || !std::isfinite(hh[i])) return fail(c, SP_EINVAL, "thickness %zu not positive", i);
        rmax = std::max(rmax, rh[i]);
    }
    const double Lmin = std::min(c->p.cell_lx, c->p.cell_ly);
    if (n > 0 && !((double)rmax < 0.25 * Lmin))
        return fail(c, SP_EINVAL, "r_max %g must stay below a quarter of the cell (%g)", rmax, 0.25 * Lmin);

    c->start_h.assign((size_t)c->ncells + 1, 0);
    for (int i = 0; i < c->ncells; ++i) c->start_h[i + 1] = c->start_h[i] + counts[i];
    c->counts_h.assign(counts, counts + c->ncells);
    c->order_h.resize(c->ncells);
    for (int32_t i = 0; i < c->ncells; ++i) c->order_h[i] = i;
    std::stable_sort(c->order_h.begin(), c->order_h.end(),
                     [&](int32_t x, int32_t y) { return c->counts_h[x] > c->counts_h[y]; });
    HIP_TRY(c, hipMemcpyAsync(c->cell_start, c->start_h.data(), ((size_t)c->ncells + 1) * 4,
                              hipMemcpyHostToDevice, c->stream));
    SP_TRY(plan_bins(c, rmax, n > 0));
    c->skin_set = c->skin;
    c->n = n;
    SP_TRY(build_buckets(c, counts));
    SP_TRY(prepare_buckets(c));
    if (block_eligible(c)) SP_TRY(block_prepare(c));
    HIP_TRY(c, hipMemsetAsync(c->err_d, 0, 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->contacts_d, 0, (size_t)c->ncells * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->cands_d, 0, (size_t)c->ncells * 8, c->stream));
    c->blk_steps = 0;
    HIP_TRY(c, hipMemsetAsync(c->cfl_bits_d, 0, 8, c->stream));
    c->steps = 0;
    SP_TRY(upload_phase(c));
    SP_TRY(reset_continuum(c));
    SP_TRY(init_reduced_all(c, c->momb[0]));   // statistics of the initial state
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->have_floes = true;
    return SP_OK;
}

sp_status sp_set_floes(sp_ctx* c, int64_t n, const int32_t* counts, const uint32_t* xi,
                       const uint32_t* yi, const float* u, const float* v, const float* omega,
                       const float* theta, const float* r, const float* h)
{
    const void* src[8] = {xi, yi, u, v, omega, theta, r, h};
    return set_floes_common(c, n, counts, src, hipMemcpyHostToDevice);
}

sp_status sp_set_floes_device(sp_ctx* c, int64_t n, const int32_t* counts, const void* xi,
                              const void* yi, const void* u, const void* v, const void* omega,
                              const void* theta, const void* r, const void* h)
{
    const void* src[8] = {xi, yi, u, v, omega, theta, r, h};
    return set_floes_common(c, n, counts, src, hipMemcpyDeviceToDevice);
}

// A call's continuum updates follow its last blocked launch (each earlier
// block's run beside the next block's DEM launch).  Ending the call in a short
// launch of kTailSteps steps lets the updates of the steps before it run
// beside that launch, and leaves only its own after it; the extra launch costs
// its staging and write-back.  Measured on MI355X: a continuum launch on a grid
// of up to kTailMaxCells cells takes about kLfLaunchPs (launch and memory
// latency, not bandwidth), one more blocked launch about kStagePsPerFloe
// picoseconds per floe (plain64, 1,048,576 floes in 4096 cells: 27 us, and a
// 20-step call 3-4 % faster; uneven128, 4.17 M floes in 16,384 cells: 108 us
// against 30 updates of 2.8 us, slower split, so not split).
constexpr int kTailSteps = 2;
constexpr int kTailMaxCells = 16384;
constexpr double kLfLaunchPs = 2.8e6;
constexpr double kStagePsPerFloe = 26.0;

static bool tail_split_pays(const sp_ctx* c, int K)
{
    if (K < 6 * kTailSteps || c->ncells > kTailMaxCells) return false;
    return (double)(K - kTailSteps) * kLfLaunchPs > kStagePsPerFloe * (double)c->n;
}

sp_status sp_step(sp_ctx* c, double dt, int64_t nsteps)
{
    if (!c) return SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_step before sp_set_floes");
    if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0)
        return fail(c, SP_EINVAL, "dt must be positive and nsteps non-negative");
    SP_TRY(upload_phase(c));
    if (c->lf_pending && c->lf_dt != dt) SP_TRY(flush_lf(c));   // pending update of another dt
    const bool cont = !(c->p.flags & SP_NO_CONTINUUM);
    const StepArgs base = make_args(c, dt);
    c->t_now += dt * (double)nsteps;
    if (c->N0 > 1) return coupled_steps(c, base, nsteps);
    int64_t left = nsteps;
    if (block_eligible(c)) {
        // whole blocks, then the remainder as one shorter block: no step of
        // this path runs the per-step kernel or captures a graph
        while (left > 0) {
            int K = (int)std::min<int64_t>(left, c->block_k);
            if (K == left && cont && tail_split_pays(c, K)) K -= kTailSteps;
            SP_TRY(block_chunk(c, base, K));
            left -= K;
        }
        SP_TRY(join_block_lf(c));   // later work on the stream sees the continuum
        return SP_OK;
    }
    while (left > 0) {
        const bool steady = (c->kstep % 2 == 0) && (c->lf_pending == cont);
        if (c->graph_chunk > 0 && c->graph_ok && steady && left >= c->graph_chunk) {
            if (!c->gexec || c->graph_dt != dt) SP_TRY(capture_graph(c, dt));
            if (c->gexec) {
                HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
                c->kstep += c->graph_chunk;
                c->steps += c->graph_chunk;
                c->lf_pending = cont;
                c->lf_dt = dt;
                left -= c->graph_chunk;
                continue;
            }
        }
        SP_TRY(step_once(c, base));
        --left;
    }
    return SP_OK;
}

sp_status sp_profile_steps(sp_ctx* c, double dt, int64_t nsteps, double* dem_ms, double* lf_ms)
{
    if (!c) return SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_profile_steps before sp_set_floes");
    if (!(dt > 0.0) || nsteps < 1) return fail(c, SP_EINVAL, "dt must be positive and nsteps >= 1");
    if (c->N0 > 1) return fail(c, SP_ESTATE, "sp_profile_steps times the cadence N0 = 1");
    SP_TRY(upload_phase(c));
    if (c->lf_pending && c->lf_dt != dt) SP_TRY(flush_lf(c));
    if (block_eligible(c)) {
        // blocked steps: events around each chunk's DEM launches and around the
        // whole run; the DEM time per step, and the rest (continuum updates) per step
        const int64_t chunks = (nsteps + c->block_k - 1) / c->block_k;
        std::vector<hipEvent_t> ev((size_t)chunks * 2 + 2);
        for (auto& e : ev) HIP_TRY(c, hipEventCreate(&e));
        const StepArgs base = make_args(c, dt);
        c->t_now += dt * (double)(chunks * c->block_k);
        sp_status st = SP_OK;
        HIP_TRY(c, hipEventRecord(ev[2 * chunks], c->stream));
        for (int64_t q = 0; q < chunks && !st; ++q) st = block_chunk(c, base, c->block_k, true, ev[2 * q], ev[2 * q + 1]);
        if (!st) st = join_block_lf(c);
        HIP_TRY(c, hipEventRecord(ev[2 * chunks + 1], c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        double sd = 0.0;
        float all = 0.0f;
        for (int64_t q = 0; q < chunks && !st; ++q) {
            float x = 0.0f;
            if (hipEventElapsedTime(&x, ev[2 * q], ev[2 * q + 1]) != hipSuccess) st = fail(c, SP_EDEVICE, "event timing");
            sd += x;
        }
        if (!st && hipEventElapsedTime(&all, ev[2 * chunks], ev[2 * chunks + 1]) != hipSuccess)
            st = fail(c, SP_EDEVICE, "event timing");
        for (auto& e : ev) (void)hipEventDestroy(e);
        if (st) return st;
        const double per = (double)(chunks * c->block_k);
        if (dem_ms) *dem_ms = sd / per;
        if (lf_ms) *lf_ms = ((double)all - sd) / per;
        return check_device_err(c);
    }
    // One event pair around the whole run of back-to-back launches: an event
    // recorded between two launches costs a few microseconds of its own.
    hipEvent_t ev[2] = {nullptr, nullptr};
    HIP_TRY(c, hipEventCreate(&ev[0]));
    HIP_TRY(c, hipEventCreate(&ev[1]));
    const StepArgs base = make_args(c, dt);
    sp_status st = SP_OK;
    c->t_now += dt * (double)nsteps;
    HIP_TRY(c, hipEventRecord(ev[0], c->stream));
    for (int64_t k = 0; k < nsteps && !st; ++k) st = step_once(c, base);
    HIP_TRY(c, hipEventRecord(ev[1], c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float total = 0;
    const hipError_t te = hipEventElapsedTime(&total, ev[0], ev[1]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st) return st;
    HIP_TRY(c, te);
    const double sd = total;
    if (dem_ms) *dem_ms = sd / (double)nsteps;
    if (lf_ms) *lf_ms = 0.0;   // the continuum update runs inside the DEM launches
    return check_device_err(c);
}

sp_status sp_synchronize(sp_ctx* c)
{
    if (!c) return SP_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return check_device_err(c);
}

sp_status sp_read_moments(sp_ctx* c, int32_t which, double* out)
{
    if (!c || !out) return c ? fail(c, SP_EINVAL, "null output") : SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    const int nc = c->ncells;
    if (which == SP_MOMENTS_DEM) {
        StepArgs a = make_args(c, 0.0);
        a.mom = c->mom2;
        if (nc > 0) {
            hipLaunchKernelGGL(stats_kernel, dim3(nc), dim3(256), 0, c->stream, a, nullptr, 0);
            HIP_TRY(c, hipGetLastError());
        }
        std::vector<double> buf((size_t)nc * kMomStride);
        HIP_TRY(c, hipMemcpyAsync(buf.data(), c->mom2, buf.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < nc; ++i)
            for (int k = 0; k < SP_NMOM; ++k) out[(size_t)i * SP_NMOM + k] = buf[(size_t)i * kMomStride + k];
    } else if (which == SP_MOMENTS_CONTINUUM) {
        SP_TRY(flush_lf(c));
        std::vector<double> buf((size_t)nc * 4);
        HIP_TRY(c, hipMemcpyAsync(buf.data(), c->Q[c->kstep & 1], buf.size() * 8, hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < nc; ++i)
            for (int f = 0; f < 4; ++f) out[(size_t)i * 4 + f] = buf[(size_t)f * nc + i];
    } else {
        return fail(c, SP_EINVAL, "unknown moments selector %d", which);
    }
    return check_device_err(c);
}

sp_status sp_read_moments_noalloc(sp_ctx* c, int32_t which, double* out)
{
    if (!c || !out) return c ? fail(c, SP_EINVAL, "null output") : SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    if (which != SP_MOMENTS_DEM && which != SP_MOMENTS_CONTINUUM)
        return fail(c, SP_EINVAL, "unknown moments selector %d", which);
    if (c->ncells > kNoAllocMaxCells)
        return fail(c, SP_ECAPACITY, "%d cells exceed the %d of sp_read_moments_noalloc's static scratch",
                    c->ncells, kNoAllocMaxCells);
    double* const sc = scratch_of(c->device);
    if (!sc) return fail(c, SP_EDEVICE, "no static scratch on device %d", c->device);
    const int nc = c->ncells;
    if (which == SP_MOMENTS_DEM) {
        StepArgs a = make_args(c, 0.0);
        a.mom = sc;   // every row of the call is written before it is read
        if (nc > 0) {
            hipLaunchKernelGGL(stats_kernel, dim3(nc), dim3(256), 0, c->stream, a, nullptr, 0);
            HIP_TRY(c, hipGetLastError());
            HIP_TRY(c, hipMemcpy2DAsync(out, SP_NMOM * sizeof(double), sc, kMomStride * sizeof(double),
                                        SP_NMOM * sizeof(double), (size_t)nc, hipMemcpyDeviceToHost, c->stream));
        }
    } else {
        SP_TRY(flush_lf(c));
        if (nc > 0) {
            hipLaunchKernelGGL(q_rows_kernel, dim3((nc * 4 + 255) / 256), dim3(256), 0, c->stream, c->Q[c->kstep & 1],
                               nc, sc);
            HIP_TRY(c, hipGetLastError());
            HIP_TRY(c, hipMemcpyAsync(out, sc, (size_t)nc * 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        }
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return check_device_err(c);
}

sp_status sp_read_floes(sp_ctx* c, uint32_t* xi, uint32_t* yi, float* u, float* v, float* omega,
                        float* theta, float* r)
{
    if (!c) return SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    const size_t N = (size_t)c->n * 4;
    void* dst[7] = {xi, yi, u, v, omega, theta, r};
    const void* src[7] = {c->xi, c->yi, c->u, c->v, c->w, c->th, c->r};
    for (int k = 0; k < 7; ++k)
        if (dst[k] && N) HIP_TRY(c, hipMemcpyAsync(dst[k], src[k], N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return check_device_err(c);
}

sp_status sp_read_pairs(sp_ctx* c, int64_t cap, int32_t* l, int32_t* j, int64_t* count)
{
    if (!c || !count || cap < 0 || (cap > 0 && (!l || !j)))
        return c ? fail(c, SP_EINVAL, "bad pair buffers") : SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    // first pass counts, second pass stores everything, host sorts
    unsigned long long* cnt_d = nullptr;
    SP_TRY(dalloc(c, &cnt_d, 1));
    StepArgs a = make_args(c, 0.0);
    HIP_TRY(c, hipMemsetAsync(cnt_d, 0, 8, c->stream));
    if (c->ncells > 0)
        hipLaunchKernelGGL(pairs_kernel, dim3(c->ncells), dim3(256), 0, c->stream, a, (int32_t*)nullptr,
                           (int32_t*)nullptr, cnt_d, 0ll);
    unsigned long long tot = 0;
    HIP_TRY(c, hipMemcpyAsync(&tot, cnt_d, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (tot > 0) {
        int32_t *pl = nullptr, *pj = nullptr;
        sp_status st = dalloc(c, &pl, tot);
        if (!st) st = dalloc(c, &pj, tot);
        if (st) {
            (void)hipFree(cnt_d);
            if (pl) (void)hipFree(pl);
            return st;
        }
        HIP_TRY(c, hipMemsetAsync(cnt_d, 0, 8, c->stream));
        hipLaunchKernelGGL(pairs_kernel, dim3(c->ncells), dim3(256), 0, c->stream, a, pl, pj, cnt_d,
                           (long long)tot);
        std::vector<int32_t> hl(tot), hj(tot);
        HIP_TRY(c, hipMemcpyAsync(hl.data(), pl, tot * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(hj.data(), pj, tot * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        std::vector<int64_t> key(tot);
        for (size_t i = 0; i < tot; ++i) key[i] = ((int64_t)hl[i] << 32) | (uint32_t)hj[i];
        std::sort(key.begin(), key.end());
        for (size_t i = 0; i < tot && (int64_t)i < cap; ++i) {
            l[i] = (int32_t)(key[i] >> 32);
            j[i] = (int32_t)(key[i] & 0xffffffff);
        }
        (void)hipFree(pl);
        (void)hipFree(pj);
    }
    (void)hipFree(cnt_d);
    *count = (int64_t)tot;
    return check_device_err(c);
}

sp_status sp_get_stats(sp_ctx* c, int64_t* contacts, int64_t* steps, double* max_cfl)
{
    if (!c) return SP_EINVAL;
    if (c->have_floes) SP_TRY(flush_lf(c));
    unsigned long long cnt = 0, bits = 0;
    std::vector<unsigned long long> per_cell((size_t)c->ncells);
    HIP_TRY(c, hipMemcpyAsync(per_cell.data(), c->contacts_d, per_cell.size() * 8, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(&bits, c->cfl_bits_d, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (unsigned long long x : per_cell) cnt += x;
    if (contacts) *contacts = (int64_t)cnt;
    if (steps) *steps = c->steps;
    if (max_cfl) {
        double d;
        memcpy(&d, &bits, 8);
        *max_cfl = d;
    }
    return SP_OK;
}

sp_status sp_get_schedule(sp_ctx* c, int32_t* schedule, int32_t* bins_x, int32_t* bins_y)
{
    if (!c) return SP_EINVAL;
    if (schedule) *schedule = c->sched;
    if (bins_x) *bins_x = c->nbx;
    if (bins_y) *bins_y = c->nby;
    return SP_OK;
}

sp_status sp_get_batching(sp_ctx* c, int32_t* cells, int32_t* waves, int32_t* persistent)
{
    if (!c) return SP_EINVAL;
    for (int q = 0; q < kNumBuckets; ++q) {
        if (cells) cells[q] = (int32_t)c->bk[q].cells_h.size();
        if (waves) waves[q] = c->bk[q].waves;
        if (persistent) persistent[q] = c->bk[q].persist;
    }
    return SP_OK;
}

sp_status sp_set_batching(sp_ctx* c, const int32_t* waves, const int32_t* persistent)
{
    if (!c || !waves || !persistent) return c ? fail(c, SP_EINVAL, "null batching arrays") : SP_EINVAL;
    for (int q = 0; q < kNumBuckets; ++q)
        if (!(waves[q] == 1 || waves[q] == 2 || waves[q] == 4 || waves[q] == 8) ||
            (persistent[q] != 0 && persistent[q] != 1))
            return fail(c, SP_EINVAL, "bucket %d: waves must be 1, 2, 4 or 8, persistent 0 or 1", q);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    for (int q = 0; q < kNumBuckets; ++q) {
        c->bk[q].waves = waves[q];
        c->bk[q].persist = persistent[q];
        c->bk[q].bwaves = 0;   // blocked launches follow the new W
    }
    if (c->have_floes) SP_TRY(prepare_buckets(c));
    return SP_OK;
}

sp_status sp_set_step_block(sp_ctx* c, int32_t k)
{
    if (!c) return SP_EINVAL;
    if (k < 1 || k > SP_MAX_STEP_BLOCK) return fail(c, SP_EINVAL, "step block must be in [1, %d]", SP_MAX_STEP_BLOCK);
    SP_TRY(flush_lf(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->block_k = k;
    if (c->have_floes && block_eligible(c)) SP_TRY(block_prepare(c));
    return SP_OK;
}

sp_status sp_get_work(sp_ctx* c, int64_t* candidate_tests, int64_t* blocked_steps)
{
    if (!c) return SP_EINVAL;
    std::vector<unsigned long long> per_cell((size_t)c->ncells);
    HIP_TRY(c, hipMemcpyAsync(per_cell.data(), c->cands_d, per_cell.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned long long t = 0;
    for (unsigned long long x : per_cell) t += x;
    if (candidate_tests) *candidate_tests = (int64_t)t;
    if (blocked_steps) *blocked_steps = c->blk_steps;
    return SP_OK;
}

sp_status sp_get_step_block(sp_ctx* c, int32_t* k, int32_t* active)
{
    if (!c) return SP_EINVAL;
    if (k) *k = c->block_k;
    if (active) *active = block_eligible(c) ? 1 : 0;
    return SP_OK;
}

sp_status sp_set_graph_chunk(sp_ctx* c, int32_t chunk)
{
    if (!c) return SP_EINVAL;
    if (chunk < 0 || (chunk % 2) != 0) return fail(c, SP_EINVAL, "graph chunk must be even and >= 0");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->graph_chunk = chunk;
    c->graph_ok = true;
    return SP_OK;
}

sp_status sp_autotune(sp_ctx* c, double dt, int32_t reps, double* best_ms)
{
    if (!c) return SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_autotune before sp_set_floes");
    if (!(dt > 0.0) || reps < 1) return fail(c, SP_EINVAL, "dt must be positive and reps >= 1");
    if (c->p.flags & SP_TANGENTIAL_SPRING) return fail(c, SP_ESTATE, "the autotuner does not run the tangential spring");
    SP_TRY(upload_phase(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    // scratch copies of the mutable state: the trials do not advance the simulation
    const size_t N = (size_t)std::max<int64_t>(1, c->n);
    uint32_t *sx = nullptr, *sy = nullptr, *serr = nullptr;
    float *su = nullptr, *sv = nullptr, *sw = nullptr, *sth = nullptr;
    double* smom = nullptr;
    unsigned long long* scnt = nullptr;
    sp_status st = SP_OK;
    if (!st) st = dalloc(c, &sx, N);
    if (!st) st = dalloc(c, &sy, N);
    if (!st) st = dalloc(c, &su, N);
    if (!st) st = dalloc(c, &sv, N);
    if (!st) st = dalloc(c, &sw, N);
    if (!st) st = dalloc(c, &sth, N);
    if (!st) st = dalloc(c, &serr, 1);
    if (!st) st = dalloc(c, &scnt, std::max<size_t>(1, (size_t)c->ncells));
    if (!st) st = dalloc(c, &smom, (size_t)c->ncells * kMomStride);
    auto cleanup = [&]() {
        void* ps[] = {sx, sy, su, sv, sw, sth, serr, scnt, smom};
        for (void* p : ps)
            if (p) (void)hipFree(p);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = SP_EDEVICE;
    const size_t B = (size_t)c->n * 4;
    if (!st && c->n > 0) {
        void* dsts[6] = {sx, sy, su, sv, sw, sth};
        const void* srcs[6] = {c->xi, c->yi, c->u, c->v, c->w, c->th};
        for (int k = 0; k < 6 && !st; ++k)
            if (hipMemcpyAsync(dsts[k], srcs[k], B, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
                st = SP_EDEVICE;
    }
    if (!st && hipMemsetAsync(serr, 0, 4, c->stream) != hipSuccess) st = SP_EDEVICE;
    StepArgs a = make_args(c, dt);
    a.xi = sx;
    a.yi = sy;
    a.u = su;
    a.v = sv;
    a.w = sw;
    a.th = sth;
    a.err = serr;
    a.contacts = scnt;
    a.mom = smom;
    a.lf = 0;
    double total = 0.0;
    const bool blocked = block_eligible(c);
    if (!st && blocked) st = tune_blocked(c, a, reps, e0, e1, &total);
    const int wv[4] = {1, 2, 4, 8};
    for (int q = 0; q < kNumBuckets && !st && !blocked; ++q) {
        Bucket& b = c->bk[q];
        if (b.cells_h.empty()) continue;
        Bucket trial;
        trial.cap = b.cap;
        trial.cells_h = b.cells_h;
        trial.work_d = b.work_d;
        double best = 1e30;
        int bw = b.waves, bq = b.persist;
        for (int wi = 0; wi < 4 && !st; ++wi)
            for (int pq = 0; pq < 2 && !st; ++pq) {
                trial.waves = wv[wi];
                trial.persist = pq;
                if (prepare_bucket(c, trial) != SP_OK) continue;   // variant does not fit this device
                for (int k = 0; k < 2 && !st; ++k) st = launch_bucket(c, trial, a, k, false, true);   // warm-up
                double t_best = 1e30;
                for (int r = 0; r < reps && !st; ++r) {
                    if (hipEventRecord(e0, c->stream) != hipSuccess) st = SP_EDEVICE;
                    for (int k = 0; k < 2 && !st; ++k) st = launch_bucket(c, trial, a, k, false, true);
                    if (!st && hipEventRecord(e1, c->stream) != hipSuccess) st = SP_EDEVICE;
                    if (!st && hipEventSynchronize(e1) != hipSuccess) st = SP_EDEVICE;
                    float ms = 0;
                    if (!st && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = SP_EDEVICE;
                    if (!st) t_best = std::min(t_best, 0.5 * (double)ms);
                }
                if (!st && t_best < best) {
                    best = t_best;
                    bw = trial.waves;
                    bq = pq;
                }
            }
        trial.work_d = nullptr;    // owned by the real bucket
        b.waves = bw;
        b.persist = bq;
        total += best;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    cleanup();
    if (st) return st == SP_EDEVICE ? fail(c, st, "autotune timing failed") : st;
    SP_TRY(prepare_buckets(c));
    SP_TRY(invalidate_lists(c, nullptr, c->ncells));   // the trials stepped a scratch state with them
    if (blocked) SP_TRY(block_prepare(c));              // the ring for the chosen block length
    drop_graph(c);
    if (best_ms) *best_ms = total;
    return SP_OK;
}

sp_status sp_get_block_waves(sp_ctx* c, int32_t* waves)
{
    if (!c || !waves) return c ? fail(c, SP_EINVAL, "null waves") : SP_EINVAL;
    for (int q = 0; q < kNumBuckets; ++q) waves[q] = c->bk[q].cells_h.empty() ? 0 : block_waves(c->bk[q]);
    return SP_OK;
}

}  // extern "C"

#include "closure_host.h"
#include "hybrid_host.h"
#include "coupling_host.h"
#include "global_dem.h"
#include "checkpoint_host.h"
