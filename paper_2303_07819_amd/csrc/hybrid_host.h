// Coarse-to-fine re-synchronisation and the DEM + closure hybrid step
// (included at the end of spdem.hip, after closure_host.h).
//
// Re-synchronisation (Sec. 3.3, all nudging sub-steps taken at once): a cell's
// floes are moved to target coarse values (rho, P_x, P_y, P_w).  Radii are
// scaled by the common factor that makes the cell mass rho A (an increment
// proportional to each radius), then every floe gets the same velocity shift
// A dP / M and the same spin shift A dP_w / sum I, which puts P and P_w exactly
// on their targets.
//
// Hybrid step: cells flagged as closure cells skip the DEM.  Their continuum
// state takes the base update (the Lax-Friedrichs step with every cell's
// statistics from its reduced DEM, closure_host.h) plus the network's residual
// tendency for the features of the base-updated state Q_b:
// Q <- Q_b + dt T(features(Q_b)).  The other cells run the DEM step and the
// Lax-Friedrichs update, which reads the coefficient of a neighbouring closure
// cell from its reduced DEM.  A closure cell's floes stay frozen.  Every
// check_every steps a rotating sample of closure cells is checked: their floes
// catch up with the DEM steps they missed (cells do not interact in the DEM,
// so this is exactly the plain method's fine state), their statistics give the
// residual tendency the plain method applies, and a cell whose closure misses
// it by more than the tolerance runs the DEM for the next fallback_steps
// steps; every checked cell's reduced DEM restarts from its true floes.
#pragma once

namespace spdem {

enum { RS_OK = 0, RS_CLAMPED = 1, RS_INVALID = 2 };

// Sum / max over one wavefront, taken from lane 0 so that every lane uses the
// same value (xor butterflies leave each lane a sum in its own order).
__device__ __forceinline__ double wave_sum_d(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return __shfl(x, 0, 64);
}

__device__ __forceinline__ float wave_max_f(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    return __shfl(x, 0, 64);
}

// One wavefront (64 threads) per listed cell.  Targets: targets[ncl][4], or
// with x0m the coarse-to-fine update X0 + frac (Q - X0) of the cell (X0 =
// (M, P_x, P_y, L) / area from the statistics x0m, Q [4][nc]).  The radius
// scale is limited so that no radius exceeds r_lim (the contact-search bin
// radius); such a cell reports RS_CLAMPED and keeps a smaller mass than its
// target.  A target that cannot be met (rho <= 0 or not finite for a cell with
// floes, anything nonzero for an empty cell) leaves the cell unchanged and
// reports RS_INVALID.  status may be null.  With vdisp, the cell's candidate
// lists stay valid: the largest radius growth of its floes (rounded up) is
// added to its displacement bound, since a radius that grows by g moves every
// contact threshold of the floe as a displacement by g would.  With counters,
// clamped and invalid cells are also counted into counters[0] and counters[1].
__global__ __launch_bounds__(64) void resync_kernel(const int32_t* cells, const int32_t* cell_start, float* r,
                                                    const float* h, float* u, float* v, float* w,
                                                    const double* targets, const double* x0m, const double* Qc,
                                                    double frac, int nc, double rho_ice, double area, float r_lim,
                                                    int32_t* status, float* vdisp, unsigned long long* counters)
{
    const int c = cells[blockIdx.x];
    const int s = cell_start[c], n = cell_start[c + 1] - s;
    const int lane = threadIdx.x;
    double tg[4];
    if (x0m) {
        const double* st = x0m + (size_t)c * kMomStride;
        const double inv_area = 1.0 / area;
        const double x0[4] = {st[M_MASS] * inv_area, st[M_PX] * inv_area, st[M_PY] * inv_area, st[M_L] * inv_area};
#pragma unroll
        for (int f = 0; f < 4; ++f) tg[f] = x0[f] + frac * (Qc[(size_t)f * nc + c] - x0[f]);
    } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) tg[f] = targets[(size_t)blockIdx.x * 4 + f];
    }
    if (n == 0) {
        if (lane == 0 && status)
            status[blockIdx.x] = (tg[0] != 0.0 || tg[1] != 0.0 || tg[2] != 0.0 || tg[3] != 0.0) ? RS_INVALID : RS_OK;
        return;
    }
    bool finite = true;
#pragma unroll
    for (int f = 0; f < 4; ++f) finite = finite && isfinite(tg[f]);
    if (!finite || !(tg[0] > 0.0)) {
        if (lane == 0) {
            if (status) status[blockIdx.x] = RS_INVALID;
            if (counters) atomicAdd(&counters[1], 1ull);
        }
        return;
    }
    // mass and largest radius of the cell
    double m0 = 0.0;
    float r0 = 0.0f;
    for (int l = lane; l < n; l += 64) {
        const float rf = r[s + l];
        const double rl = rf;
        m0 += rho_ice * (double)h[s + l] * kPi * rl * rl;
        r0 = fmaxf(r0, rf);
    }
    const double mass = wave_sum_d(m0);
    const float rmax = wave_max_f(r0);
    double sc = sqrt(tg[0] * area / mass);
    const double lim = (double)r_lim / (double)rmax;
    const bool clamped = sc > lim;
    if (clamped) sc = lim;
    // rescale the radii, then the sums of the rescaled cell
    double acc[5] = {0, 0, 0, 0, 0};   // M, sum m u, sum m v, L, sum I
    float grow = 0.0f;
    for (int l = lane; l < n; l += 64) {
        const float ro = r[s + l];
        const float rn = fminf((float)((double)ro * sc), r_lim);
        grow = fmaxf(grow, rn - ro);   // rounded to nearest; rounded up below
        r[s + l] = rn;
        const double rl = rn;
        const double m = rho_ice * (double)h[s + l] * kPi * rl * rl;
        acc[0] += m;
        acc[1] += m * (double)u[s + l];
        acc[2] += m * (double)v[s + l];
        acc[3] += m * rl * rl * (double)w[s + l];
        acc[4] += m * rl * rl;
    }
    double tot[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) tot[k] = wave_sum_d(acc[k]);
    const float gmax = wave_max_f(grow);
    if (lane == 0 && vdisp && gmax > 0.0f) {
        // rn - ro is exact or one rounding off; two ulps of margin on the
        // difference and on the sum keep the bound an upper bound
        const float g = gmax * (1.0f + 0x1p-22f);
        vdisp[c] = (vdisp[c] + g) * (1.0f + 0x1p-22f);
    }
    if (lane == 0 && counters && clamped) atomicAdd(&counters[0], 1ull);
    const double dvx = (tg[1] * area - tot[1]) / tot[0];
    const double dvy = (tg[2] * area - tot[2]) / tot[0];
    const double dw = (tg[3] * area - tot[3]) / tot[4];
    for (int l = lane; l < n; l += 64) {
        u[s + l] = (float)((double)u[s + l] + dvx);
        v[s + l] = (float)((double)v[s + l] + dvy);
        w[s + l] = (float)((double)w[s + l] + dw);
    }
    if (lane == 0 && status) status[blockIdx.x] = clamped ? RS_CLAMPED : RS_OK;
}

// Continuum step of the hybrid: closure cells Qb + dT T (Qb: the base-updated
// state, T: the network's residual tendency, applied while the cell's reduced
// DEM is younger than `window`, always if window <= 0), the others the LF
// step of their statistics.
__global__ void hybrid_continuum_kernel(const double* mom, const double* Q, const double* Qb, double* Qn,
                                        const int32_t* row, const float* T, const double* red, double t,
                                        double window, int nx, int ny, double dT, double dX, double dY,
                                        double inv_area, unsigned long long* max_cfl_bits, uint32_t* err)
{
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = nx * ny;
    if (C >= nc) return;
    const int q = row[C];
    if (q >= 0) {
        const double w = (window <= 0.0 || t - red[(size_t)C * 4 + 3] < window) ? dT : 0.0;
#pragma unroll
        for (int f = 0; f < 4; ++f) Qn[(size_t)f * nc + C] = Qb[(size_t)f * nc + C] + w * (double)T[(size_t)q * 4 + f];
    } else {
        lf_cell(C, mom, Q, Qn, nx, ny, dT, dX, dY, inv_area, max_cfl_bits, err, false);   // the hybrid has no walls
    }
}

// Plain-method residual tendency (LF(Q) - Qb) / dT of the listed cells: their
// own coefficients and sources from the statistics `fresh`, the neighbours'
// coefficients from `mom`.
__global__ void check_tendency_kernel(const int32_t* cells, int ncl, const double* fresh, const double* mom,
                                      const double* Q, const double* Qb, int nx, int ny, double dT, double dX,
                                      double dY, double inv_area, float* T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    const int C = cells[i];
    const int nc = nx * ny;
    const int ix = C % nx, iy = C / nx;
    const int E = iy * nx + (ix + 1 == nx ? 0 : ix + 1);
    const int W = iy * nx + (ix == 0 ? nx - 1 : ix - 1);
    const int N = (iy + 1 == ny ? 0 : iy + 1) * nx + ix;
    const int S = (iy == 0 ? ny - 1 : iy - 1) * nx + ix;
    const double* sC = fresh + (size_t)C * kMomStride;
    const double uC = sC[M_UBAR], vC = sC[M_VBAR];
    const double uE = E == C ? uC : mom[(size_t)E * kMomStride + M_UBAR];
    const double uW = W == C ? uC : mom[(size_t)W * kMomStride + M_UBAR];
    const double vN = N == C ? vC : mom[(size_t)N * kMomStride + M_VBAR];
    const double vS = S == C ? vC : mom[(size_t)S * kMomStride + M_VBAR];
    const double cx = dT / (2.0 * dX), cy = dT / (2.0 * dY);
    for (int f = 0; f < 4; ++f) {
        const double qE = Q[(size_t)f * nc + E], qW = Q[(size_t)f * nc + W];
        const double qN = Q[(size_t)f * nc + N], qS = Q[(size_t)f * nc + S];
        const double avg = 0.25 * (qE + qW + qN + qS);
        double qn;
        if (f == 0 || f == 3) {
            qn = avg - cx * (uE * qE - uW * qW) - cy * (vN * qN - vS * qS) +
                 (f == 3 ? dT * sC[M_SW] * inv_area : 0.0);
        } else {
            qn = avg - dT * (uC * (qE - qW) / (2.0 * dX) + vC * (qN - qS) / (2.0 * dY)) +
                 dT * sC[f == 1 ? M_SVX : M_SVY] * inv_area;
        }
        T[(size_t)i * 4 + f] = (float)((qn - Qb[(size_t)f * nc + C]) / dT);
    }
}

}  // namespace spdem

struct HybridState {
    sp_mlp* net = nullptr;
    std::vector<uint8_t> closure;        // cells flagged for the closure
    std::vector<int32_t> fallback_left;  // > 0: a flagged cell runs the DEM for that many more steps
    std::vector<int32_t> fallback_cells; // cells with fallback_left > 0
    std::vector<uint8_t> pool;           // closure cells the checks draw from; their floes keep stepping
    std::vector<int32_t> pool_h;         // the same cells in check order
    std::vector<double> red_t0;          // start time of each cell's reduced DEM (host copy)
    int check_every = 50, check_cells = 64, fallback_steps = 100;
    double tol = 0.2;
    double net_window = 0.0;              // seconds after a reduced DEM's start the network acts (<= 0: always)
    int64_t checks = 0, fallbacks = 0, cursor = 0, hsteps = 0;
    const double* last_mom = nullptr;     // statistics of the step just taken (the block ring, or momb)
    Bucket bk[kNumBuckets];               // DEM-mode cells, and the pool's closure-mode cells (shadow DEM:
                                          // their statistics go to scratch)
    std::vector<int32_t> clos_h;          // closure-mode cells
    int32_t* clos_d = nullptr;
    int32_t* row_d = nullptr;             // [ncells] row of a closure-mode cell in X and T, else -1
    float* X = nullptr;                   // [nclos][45]
    float* T = nullptr;                   // [nclos][4]
    int32_t* chk_d = nullptr;             // sampled cells of a check
    float* Xk = nullptr;
    float* Tk = nullptr;
    float* Tdem = nullptr;
    double* Qs = nullptr;                 // base-updated continuum state [4][ncells]
    double* rs = nullptr;                 // reduced DEM statistics of every cell at the step's time [ncells][5]
    int32_t* back_d = nullptr;            // cells whose fallback window ended [ncells]
    int ndem = 0;
    // the next block's DEM launch beside this block's closure work: its stream,
    // a block's DEM launch done (per ring half), closure work done with a half
    hipStream_t dem_stream = nullptr;
    hipEvent_t fork = nullptr, dem_done[2] = {nullptr, nullptr}, clos_done[2] = {nullptr, nullptr};
    bool clos_used[2] = {false, false};
};

namespace {

void hybrid_free_buffers(HybridState* h)
{
    for (auto& b : h->bk) {
        if (b.work_d) (void)hipFree(b.work_d);
        b.work_d = nullptr;
    }
    void* ps[] = {h->clos_d, h->row_d, h->X, h->T, h->chk_d, h->Xk, h->Tk, h->Tdem, h->Qs,
                  h->back_d, h->rs};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    h->clos_d = h->row_d = h->chk_d = h->back_d = nullptr;
    h->X = h->T = h->Xk = h->Tk = h->Tdem = nullptr;
    h->Qs = nullptr;
    h->rs = nullptr;
}

// Rebuild the DEM buckets and the closure list from the current modes.
sp_status hybrid_rebuild(sp_ctx* c)
{
    HybridState* h = c->hyb;
    std::vector<uint8_t> step(c->ncells), shadow(c->ncells);
    std::vector<int32_t> row(c->ncells, -1);
    h->clos_h.clear();
    for (int i = 0; i < c->ncells; ++i) {
        const bool clos = h->closure[i] && h->fallback_left[i] == 0;
        shadow[i] = clos && h->pool[i];
        // a cell without floes has no DEM work: its statistics stay zero
        step[i] = c->counts_h[i] > 0 && (!clos || shadow[i]);
        if (clos) {
            row[i] = (int32_t)h->clos_h.size();
            h->clos_h.push_back(i);
        }
    }
    h->ndem = c->ncells - (int)h->clos_h.size();
    HIP_TRY(c, hipStreamSynchronize(c->stream));   // queued work may still read the buffers replaced below
    SP_TRY(build_buckets_into(c, h->bk, c->counts_h.data(), step.data(), shadow.data()));
    for (auto& b : h->bk)
        if (!b.cells_h.empty()) SP_TRY(prepare_bucket(c, b));
    if (!h->clos_d) {   // sized for every cell once: modes change without reallocation
        const size_t nc = (size_t)c->ncells;
        SP_TRY(dalloc(c, &h->clos_d, nc));
        SP_TRY(dalloc(c, &h->X, nc * spmlp::kIn));
        SP_TRY(dalloc(c, &h->T, nc * spmlp::kOut));
    }
    if (!h->clos_h.empty())
        HIP_TRY(c, hipMemcpyAsync(h->clos_d, h->clos_h.data(), h->clos_h.size() * 4, hipMemcpyHostToDevice,
                                  c->stream));
    HIP_TRY(c, hipMemcpyAsync(h->row_d, row.data(), row.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));   // host temporaries
    return SP_OK;
}

// The network's de-normalised output for `rows` feature rows, on the
// simulation's stream.
sp_status net_forward_on(sp_ctx* c, sp_mlp* net, const float* x, int rows, float* y)
{
    if (rows <= 0) return SP_OK;
    const sp_status st = mlp_infer(net, x, rows, y, c->stream);
    if (st) return fail(c, st, "closure network: %s", net->err.c_str());
    return SP_OK;
}

// Restart the reduced DEM of the listed cells (device list) from their floes
// (skipping cells whose status entry is RS_INVALID); their statistics land in
// mom2.
sp_status restart_reduced(sp_ctx* c, const int32_t* cells_d, int ncl, const int32_t* status_d)
{
    if (ncl <= 0) return SP_OK;
    StepArgs a = make_args(c, 0.0);
    a.mom = c->mom2;
    hipLaunchKernelGGL(stats_kernel, dim3(ncl), dim3(256), 0, c->stream, a, cells_d, 0);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(reduced_init_kernel, dim3((ncl + 255) / 256), dim3(256), 0, c->stream, cells_d, ncl, status_d,
                       c->mom2, closure_args(c, c->t_now), c->red);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

// Re-synchronise the listed cells (device list) to targets_d; per-cell status
// into status_d; descriptors, drag coefficients and reduced DEMs follow.
sp_status resync_list(sp_ctx* c, const int32_t* cells_d, int ncl, const double* targets_d, int32_t* status_d)
{
    if (ncl <= 0) return SP_OK;
    hipLaunchKernelGGL(resync_kernel, dim3(ncl), dim3(64), 0, c->stream, cells_d, c->cell_start, c->r, c->h, c->u,
                       c->v, c->w, targets_d, nullptr, nullptr, 0.0, c->ncells, c->p.rho_ice,
                       c->p.cell_lx * c->p.cell_ly, c->r_bin, status_d, nullptr, nullptr);
    HIP_TRY(c, hipGetLastError());
    SP_TRY(invalidate_lists(c, cells_d, ncl));   // radii changed
    SP_TRY(ensure_cell_data(c));
    hipLaunchKernelGGL(descriptors_kernel, dim3(ncl), dim3(256), 0, c->stream, cells_d, c->cell_start, c->r, c->h,
                       1.0 / (c->p.cell_lx * c->p.cell_ly), c->p.rho_ice, c->p.cd * c->p.rho_ocean, c->desc, c->mf);
    HIP_TRY(c, hipGetLastError());
    SP_TRY(restart_reduced(c, cells_d, ncl, status_d));
    return SP_OK;
}

// Check the next check_cells closure-mode cells of the pool after a step (Q
// at level kstep): the pool's floes have kept stepping with the DEM, so they
// are the plain method's floes; their statistics give the plain method's
// residual tendency, and a cell whose closure misses it by more than tol of
// its state (projected over one check period) falls back to the DEM.  Every
// checked cell's reduced DEM then restarts from its floes.
sp_status hybrid_check(sp_ctx* c, double dt)
{
    HybridState* h = c->hyb;
    const int npool = (int)h->pool_h.size();
    if (npool == 0 || h->check_cells <= 0) return SP_OK;
    std::vector<int32_t> pick;   // round robin over the pool; cells in fallback run the DEM anyway
    for (int scanned = 0; scanned < npool && (int)pick.size() < h->check_cells; ++scanned) {
        const int32_t cell = h->pool_h[(size_t)h->cursor];
        h->cursor = (h->cursor + 1) % npool;
        if (h->fallback_left[cell] == 0) pick.push_back(cell);
    }
    const int nk = (int)pick.size();
    if (nk == 0) return SP_OK;
    // 1. the sampled cells' current floes
    HIP_TRY(c, hipMemcpyAsync(h->chk_d, pick.data(), (size_t)nk * 4, hipMemcpyHostToDevice, c->stream));
    // 2. their statistics and the plain method's residual tendency; the
    //    neighbours' coefficients are those of the step just taken
    StepArgs a = make_args(c, dt);
    a.mom = c->mom2;
    hipLaunchKernelGGL(stats_kernel, dim3(nk), dim3(256), 0, c->stream, a, h->chk_d, 0);
    HIP_TRY(c, hipGetLastError());
    const int64_t k = c->kstep - 1;
    const double inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    const ClosureArgs ca = closure_args(c, c->t_now);
    hipLaunchKernelGGL(base_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, c->Q[c->kstep & 1],
                       h->Qs, ca, dt);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(check_tendency_kernel, dim3((nk + 63) / 64), dim3(64), 0, c->stream, h->chk_d, nk, c->mom2,
                       h->last_mom ? h->last_mom : c->momb[k & 1], c->Q[c->kstep & 1], h->Qs, c->p.nx, c->p.ny, dt, c->p.cell_lx, c->p.cell_ly,
                       inv_area, h->Tdem);
    HIP_TRY(c, hipGetLastError());
    // 3. the closure's residual for the same cells
    hipLaunchKernelGGL(features_kernel, dim3((nk + 63) / 64), dim3(64), 0, c->stream, h->chk_d, nk, h->Qs, ca,
                       c->desc, h->Xk);
    HIP_TRY(c, hipGetLastError());
    SP_TRY(net_forward_on(c, h->net, h->Xk, nk, h->Tk));
    std::vector<float> tm((size_t)nk * 4), td((size_t)nk * 4), xk((size_t)nk * spmlp::kIn);
    HIP_TRY(c, hipMemcpyAsync(tm.data(), h->Tk, tm.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(td.data(), h->Tdem, td.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(xk.data(), h->Xk, xk.size() * 4, hipMemcpyDeviceToHost, c->stream));
    // 4. the reduced DEMs restart from the true floes
    SP_TRY(restart_reduced(c, h->chk_d, nk, nullptr));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // the cell's own state is feature 16..19 (centre of the 3 x 3 stencil)
    double floor[4] = {0, 0, 0, 0};
    for (int i = 0; i < nk; ++i)
        for (int f = 0; f < 4; ++f) floor[f] += fabs((double)xk[(size_t)i * spmlp::kIn + 16 + f]) / nk;
    bool changed = false;
    for (int i = 0; i < nk; ++i) {
        const int32_t cell = pick[i];
        const bool net = h->net_window <= 0.0 || c->t_now - h->red_t0[cell] < h->net_window;
        bool bad = false;
        for (int f = 0; f < 4 && !bad; ++f) {
            const double e = fabs((net ? (double)tm[i * 4 + f] : 0.0) - (double)td[i * 4 + f]);
            const double q = fabs((double)xk[(size_t)i * spmlp::kIn + 16 + f]) + 0.01 * floor[f];
            if (!(h->check_every * dt * e <= h->tol * q)) bad = true;
        }
        h->red_t0[cell] = c->t_now;
        h->checks++;
        if (bad) {
            h->fallbacks++;
            if (h->fallback_left[cell] == 0) h->fallback_cells.push_back(cell);
            h->fallback_left[cell] = h->fallback_steps;
            changed = true;
        }
    }
    if (changed) SP_TRY(hybrid_rebuild(c));
    return SP_OK;
}

}  // namespace

void hybrid_free(sp_ctx* c)
{
    if (!c || !c->hyb) return;
    HybridState* h = c->hyb;
    if (h->dem_stream) (void)hipStreamSynchronize(h->dem_stream);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : {h->fork, h->dem_done[0], h->dem_done[1], h->clos_done[0], h->clos_done[1]})
        if (e) (void)hipEventDestroy(e);
    if (h->dem_stream) (void)hipStreamDestroy(h->dem_stream);
    hybrid_free_buffers(c->hyb);
    delete c->hyb;
    c->hyb = nullptr;
}

extern "C" {

sp_status sp_resync_cells(sp_ctx* c, int32_t ncl, const int32_t* cells, const double* targets, int32_t* clamped)
{
    if (!c) return SP_EINVAL;
    if (ncl < 0 || (ncl > 0 && (!cells || !targets))) return fail(c, SP_EINVAL, "bad cell list or targets");
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_resync_cells before sp_set_floes");
    std::vector<uint8_t> seen(c->ncells, 0);
    for (int i = 0; i < ncl; ++i) {
        const int32_t cell = cells[i];
        if (cell < 0 || cell >= c->ncells) return fail(c, SP_EINVAL, "cell %d out of range", cell);
        if (seen[cell]) return fail(c, SP_EINVAL, "cell %d listed twice", cell);
        seen[cell] = 1;
        const double* t = targets + (size_t)i * 4;
        const bool fin = std::isfinite(t[0]) && std::isfinite(t[1]) && std::isfinite(t[2]) && std::isfinite(t[3]);
        if (c->counts_h[cell] == 0) {
            if (t[0] != 0.0 || t[1] != 0.0 || t[2] != 0.0 || t[3] != 0.0)
                return fail(c, SP_EINVAL, "nonzero target for the empty cell %d", cell);
        } else if (!fin || !(t[0] > 0.0)) {
            return fail(c, SP_EINVAL, "target of cell %d needs a positive density and finite values", cell);
        }
    }
    if (clamped) *clamped = 0;
    if (ncl == 0) return SP_OK;
    SP_TRY(flush_lf(c));
    int32_t* cd = nullptr;
    int32_t* sd = nullptr;
    double* td = nullptr;
    sp_status st = dalloc(c, &cd, ncl);
    if (!st) st = dalloc(c, &sd, ncl);
    if (!st) st = dalloc(c, &td, (size_t)ncl * 4);
    std::vector<int32_t> rs(ncl, 0);
    if (!st && (hipMemcpyAsync(cd, cells, (size_t)ncl * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
                hipMemcpyAsync(td, targets, (size_t)ncl * 4 * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess))
        st = fail(c, SP_EDEVICE, "target upload failed");
    if (!st) st = resync_list(c, cd, ncl, td, sd);
    if (!st && hipMemcpyAsync(rs.data(), sd, (size_t)ncl * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        st = fail(c, SP_EDEVICE, "status download failed");
    if (hipStreamSynchronize(c->stream) != hipSuccess && !st) st = fail(c, SP_EDEVICE, "synchronisation failed");
    (void)hipGetLastError();
    if (cd) (void)hipFree(cd);
    if (sd) (void)hipFree(sd);
    if (td) (void)hipFree(td);
    if (st) return st;
    int32_t nclamp = 0;
    for (int i = 0; i < ncl; ++i) nclamp += rs[i] == RS_CLAMPED;
    if (clamped) *clamped = nclamp;
    return SP_OK;
}

sp_status sp_hybrid_set(sp_ctx* c, sp_mlp* net, const uint8_t* closure_cells, int32_t check_every,
                        int32_t check_cells, double tol, int32_t fallback_steps, double net_window)
{
    if (!c) return SP_EINVAL;
    if (!closure_cells) {
        SP_TRY(flush_lf(c));
        hybrid_free(c);
        return SP_OK;
    }
    if (!net) return fail(c, SP_EINVAL, "the hybrid needs a network");
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_hybrid_set before sp_set_floes");
    if (check_every < 1 || check_cells < 0 || !(tol > 0) || fallback_steps < 1 || !std::isfinite(net_window))
        return fail(c, SP_EINVAL, "check_every and fallback_steps must be >= 1, check_cells >= 0, tol > 0");
    if (c->p.flags & SP_NO_CONTINUUM) return fail(c, SP_ESTATE, "the hybrid needs the continuum update");
    if (c->N0 > 1) return fail(c, SP_ESTATE, "the hybrid step runs with N0 = 1");
    if (c->p.flags & SP_TANGENTIAL_SPRING) return fail(c, SP_ESTATE, "the hybrid runs the viscous contact law");
    if (c->p.flags & SP_WALL_X) return fail(c, SP_ESTATE, "the hybrid runs on the periodic coarse grid");
    HIP_TRY(c, hipStreamSynchronize(net->stream));   // parameters and normalisation in place
    SP_TRY(flush_lf(c));
    hybrid_free(c);
    HybridState* h = new HybridState();
    c->hyb = h;
    h->net = net;
    h->closure.assign(closure_cells, closure_cells + c->ncells);
    for (int i = 0; i < c->ncells; ++i)   // a cell without floes has no DEM work: the plain update is exact
        if (c->counts_h[i] == 0) h->closure[i] = 0;
    h->fallback_left.assign(c->ncells, 0);
    // the check pool: up to 4 check_cells closure cells spread evenly over the
    // closure cells; they keep running the DEM (shadow), so a check compares
    // against the plain method's current floes and a fallback starts from them
    {
        std::vector<int32_t> clos;
        for (int i = 0; i < c->ncells; ++i)
            if (h->closure[i]) clos.push_back(i);
        const size_t np = std::min(clos.size(), (size_t)4 * (size_t)std::max(0, check_cells));
        h->pool.assign(c->ncells, 0);
        for (size_t i = 0; i < np; ++i) {
            const int32_t cell = clos[i * clos.size() / np];
            h->pool[cell] = 1;
            h->pool_h.push_back(cell);
        }
    }
    h->check_every = check_every;
    h->check_cells = check_cells;
    h->tol = tol;
    h->fallback_steps = fallback_steps;
    h->net_window = net_window;
    for (int q = 0; q < kNumBuckets; ++q) {
        h->bk[q].waves = c->bk[q].waves;
        h->bk[q].persist = c->bk[q].persist;
        h->bk[q].bwaves = c->bk[q].bwaves;
    }
    const size_t nk = (size_t)std::max(1, check_cells);
    SP_TRY(dalloc(c, &h->row_d, (size_t)c->ncells));
    SP_TRY(dalloc(c, &h->chk_d, nk));
    SP_TRY(dalloc(c, &h->Xk, nk * spmlp::kIn));
    SP_TRY(dalloc(c, &h->Tk, nk * spmlp::kOut));
    SP_TRY(dalloc(c, &h->Tdem, nk * spmlp::kOut));
    SP_TRY(dalloc(c, &h->Qs, (size_t)c->ncells * 4));
    SP_TRY(dalloc(c, &h->rs, (size_t)c->ncells * 5));
    SP_TRY(dalloc(c, &h->back_d, (size_t)c->ncells));
    SP_TRY(upload_phase(c));
    SP_TRY(ensure_cell_data(c));
    {
        std::vector<double> red((size_t)c->ncells * 4);
        HIP_TRY(c, hipMemcpyAsync(red.data(), c->red, red.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        h->red_t0.resize(c->ncells);
        for (int i = 0; i < c->ncells; ++i) h->red_t0[i] = red[(size_t)i * 4 + 3];
    }
    drop_graph(c);
    return hybrid_rebuild(c);
}

sp_status sp_step_hybrid(sp_ctx* c, double dt, int64_t nsteps)
{
    if (!c) return SP_EINVAL;
    if (!c->hyb) return fail(c, SP_ESTATE, "sp_step_hybrid before sp_hybrid_set");
    if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0)
        return fail(c, SP_EINVAL, "dt must be positive and nsteps non-negative");
    HybridState* h = c->hyb;
    SP_TRY(upload_phase(c));
    SP_TRY(flush_lf(c));
    if (nsteps == 0) return SP_OK;
    StepArgs base = make_args(c, dt);
    base.mom_alt = c->mom2;
    const double inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    const size_t slot = (size_t)c->ncells * kMomStride;
    // The DEM cells never read the continuum between checks (no coarse-to-fine
    // update at this cadence), so their steps up to the next check or the end
    // of a fallback window run as blocked launches (statistics of step t into
    // slot t of the block ring), followed by the closure and continuum work of
    // each step in order, on the library stream.
    // When nothing at a block's end changes the DEM cells (no check, no
    // fallback window ending), the next block's DEM launch is issued at once on
    // a second stream, into the other half of the ring, and runs beside this
    // block's closure work (it waits for this block's DEM launch and for the
    // closure work that last read its half).
    const bool can_block = c->block_k > 1;
    if (can_block) {
        SP_TRY(block_prepare(c));
        if (!h->dem_stream) {
            HIP_TRY(c, hipStreamCreateWithFlags(&h->dem_stream, hipStreamNonBlocking));
            HIP_TRY(c, hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
            for (int i = 0; i < 2; ++i) {
                HIP_TRY(c, hipEventCreateWithFlags(&h->dem_done[i], hipEventDisableTiming));
                HIP_TRY(c, hipEventCreateWithFlags(&h->clos_done[i], hipEventDisableTiming));
            }
        }
    }
    // steps of the block from loop step i0, with h->hsteps = hs and every
    // fallback window `done` steps shorter
    auto block_len = [&](int64_t i0, int64_t hs, int64_t done) -> int64_t {
        if (!can_block) return 1;
        int64_t L = std::min<int64_t>(c->block_k, nsteps - i0);
        L = std::min<int64_t>(L, h->check_every - hs % h->check_every);
        for (int32_t cell : h->fallback_cells) L = std::min<int64_t>(L, h->fallback_left[cell] - done);
        return L;
    };
    BlockNudge none;
    memset(&none, 0, sizeof none);
    const size_t half = (size_t)c->blk_ring_slots * slot;
    int hp = 0;                 // ring half of the current block
    int64_t early_K = 0;        // steps of the block already launched on the DEM stream (0: none)
    for (int64_t it = 0; it < nsteps;) {
        const int64_t K = block_len(it, h->hsteps, 0);
        double* ring = nullptr;
        if (K > 1) {
            ring = c->blk_ring + (size_t)hp * half;
            if (early_K > 0) {
                if (early_K != K) return fail(c, SP_EDEVICE, "hybrid block of %lld steps launched as %lld",
                                              (long long)K, (long long)early_K);
                HIP_TRY(c, hipStreamWaitEvent(c->stream, h->dem_done[hp], 0));
            } else {
                SP_TRY(join_block_lf(c));
                SP_TRY(launch_blocks(c, base, ring, (int)K, none, h->bk));
            }
            early_K = 0;
            c->blk_steps += K;
            bool quiet = (h->hsteps + K) % h->check_every != 0 && it + K < nsteps;
            for (int32_t cell : h->fallback_cells) quiet = quiet && h->fallback_left[cell] > K;
            const int64_t K2 = quiet ? block_len(it + K, h->hsteps + K, K) : 0;
            if (K2 > 1) {
                const int q = hp ^ 1;
                HIP_TRY(c, hipEventRecord(h->fork, c->stream));   // after this block's DEM launch
                HIP_TRY(c, hipStreamWaitEvent(h->dem_stream, h->fork, 0));
                if (h->clos_used[q]) HIP_TRY(c, hipStreamWaitEvent(h->dem_stream, h->clos_done[q], 0));
                SP_TRY(launch_blocks(c, base, c->blk_ring + (size_t)q * half, (int)K2, none, h->bk, h->dem_stream));
                HIP_TRY(c, hipEventRecord(h->dem_done[q], h->dem_stream));
                early_K = K2;
            }
        }
        for (int64_t t = 0; t < K; ++t, ++it) {
            const int64_t k = c->kstep;
            double* const mom = ring ? ring + (size_t)t * slot : c->momb[k & 1];
            const int nclos = (int)h->clos_h.size();
            if (nclos > 0) {
                // base-updated level-k state, the network's residual for its
                // features, the closure cells' coefficients from their reduced DEMs
                ClosureArgs ca = closure_args(c, c->t_now);
                // (the closure cells' <v> go into this step's statistics row as well)
                hipLaunchKernelGGL(reduced_stats_kernel, dim3((c->ncells + 255) / 256), dim3(256), 0, c->stream, ca,
                                   h->rs, h->row_d, mom);
                HIP_TRY(c, hipGetLastError());
                ca.rs = h->rs;   // every cell's reduced statistics once, read by the stencils below
                hipLaunchKernelGGL(base_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, c->Q[k & 1],
                                   h->Qs, ca, dt);
                HIP_TRY(c, hipGetLastError());
                hipLaunchKernelGGL(features_kernel, dim3((nclos + 127) / 128), dim3(128), 0, c->stream, h->clos_d,
                                   nclos, h->Qs, ca, c->desc, h->X);
                HIP_TRY(c, hipGetLastError());
                SP_TRY(net_forward_on(c, h->net, h->X, nclos, h->T));
            }
            // DEM step of the other cells (statistics of level k), and of the
            // check pool's closure cells (statistics into scratch: the closure
            // drives them); in a block, already done
            if (!ring)
                for (auto& b : h->bk) SP_TRY(launch_bucket(c, b, base, k, false));
            hipLaunchKernelGGL(hybrid_continuum_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, mom,
                               c->Q[k & 1], h->Qs, c->Q[(k + 1) & 1], h->row_d, h->T, c->red, c->t_now,
                               h->net_window, c->p.nx, c->p.ny, dt, c->p.cell_lx, c->p.cell_ly, inv_area,
                               c->cfl_bits_d, c->err_d);
            HIP_TRY(c, hipGetLastError());
            h->last_mom = mom;
            c->kstep++;
            c->steps++;
            c->t_now += dt;
            h->hsteps++;
            // fallback windows that end with this step (in a block, only its
            // last step): those cells' reduced DEMs restart from their floes
            std::vector<int32_t> back;
            size_t keep = 0;
            for (size_t i = 0; i < h->fallback_cells.size(); ++i) {
                const int32_t cell = h->fallback_cells[i];
                if (--h->fallback_left[cell] == 0) {
                    if (h->closure[cell]) back.push_back(cell);
                } else {
                    h->fallback_cells[keep++] = cell;
                }
            }
            h->fallback_cells.resize(keep);
            if (!back.empty()) {
                HIP_TRY(c, hipMemcpyAsync(h->back_d, back.data(), back.size() * 4, hipMemcpyHostToDevice, c->stream));
                SP_TRY(restart_reduced(c, h->back_d, (int)back.size(), nullptr));
                for (int32_t cell : back) h->red_t0[cell] = c->t_now;
                SP_TRY(hybrid_rebuild(c));   // synchronises: `back` may go
            }
            if (h->hsteps % h->check_every == 0) SP_TRY(hybrid_check(c, dt));
        }
        if (ring) {   // this block's closure work is done with its half of the ring
            HIP_TRY(c, hipEventRecord(h->clos_done[hp], c->stream));
            h->clos_used[hp] = true;
            hp ^= 1;
        }
    }
    return SP_OK;
}

sp_status sp_hybrid_stats(sp_ctx* c, int32_t* dem_cells, int32_t* closure_cells, int64_t* checks,
                          int64_t* fallbacks)
{
    if (!c) return SP_EINVAL;
    if (!c->hyb) return fail(c, SP_ESTATE, "sp_hybrid_stats before sp_hybrid_set");
    if (dem_cells) *dem_cells = c->hyb->ndem;
    if (closure_cells) *closure_cells = (int32_t)c->hyb->clos_h.size();
    if (checks) *checks = c->hyb->checks;
    if (fallbacks) *fallbacks = c->hyb->fallbacks;
    return SP_OK;
}

}  // extern "C"
