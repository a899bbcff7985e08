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
// state takes the part of the update the coarse state determines by itself
// (transport_cell, the Lax-Friedrichs step with <v> = P / rho, then
// relax_cell, mean-field drag) plus the network's residual tendency for the
// features of the transported state Q*: Q <- relax(Q*) + dt T(features(Q*)).
// The other
// cells run the DEM step and the Lax-Friedrichs update, which reads the
// coefficient <v> = P / rho of neighbouring closure cells.  Every check_every
// steps a rotating sample of closure cells is re-synchronised to its continuum
// state; its DEM statistics give the residual tendency the plain method would
// apply there, and a cell whose network output misses it by more than the
// tolerance runs the DEM for the next fallback_steps steps.
#pragma once

namespace spdem {

enum { RS_OK = 0, RS_CLAMPED = 1, RS_INVALID = 2 };

// One workgroup per listed cell.  Targets come from `targets` [ncl][4] or, if
// null, from the continuum state Q [4][nc].  The radius scale is limited so
// that no radius exceeds r_lim (the contact-search bin radius); such a cell
// reports RS_CLAMPED and keeps a smaller mass than its target.  A target that
// cannot be met (rho <= 0 or not finite for a cell with floes, anything
// nonzero for an empty cell, or, with max_ratio > 0, a mass more than
// max_ratio times above or below the floes' mass, a mean speed |P| / rho above
// max_speed or a mean spin above max_spin) leaves the cell unchanged and
// reports RS_INVALID.
__global__ __launch_bounds__(256) void resync_kernel(const int32_t* cells, const int32_t* cell_start, float* r,
                                                     const float* h, float* u, float* v, float* w,
                                                     const double* targets, const double* Q, int nc,
                                                     double rho_ice, double area, float r_lim, double max_ratio,
                                                     double max_speed, double max_spin, int32_t* status)
{
    __shared__ double part[5][256];
    __shared__ double tot[5];
    __shared__ float rpart[256];
    const int c = cells[blockIdx.x];
    const int s = cell_start[c], n = cell_start[c + 1] - s;
    const int tid = threadIdx.x;
    double tg[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) tg[f] = targets ? targets[(size_t)blockIdx.x * 4 + f] : Q[(size_t)f * nc + c];
    if (n == 0) {
        if (tid == 0)
            status[blockIdx.x] = (tg[0] != 0.0 || tg[1] != 0.0 || tg[2] != 0.0 || tg[3] != 0.0) ? RS_INVALID : RS_OK;
        return;
    }
    bool finite = true;
#pragma unroll
    for (int f = 0; f < 4; ++f) finite = finite && isfinite(tg[f]);
    if (!finite || !(tg[0] > 0.0)) {
        if (tid == 0) status[blockIdx.x] = RS_INVALID;
        return;
    }
    // mass, inertia and largest radius of the cell
    double m0 = 0.0, i0 = 0.0;
    float r0 = 0.0f;
    for (int l = tid; l < n; l += 256) {
        const double rl = r[s + l];
        const double m = rho_ice * (double)h[s + l] * kPi * rl * rl;
        m0 += m;
        i0 += m * rl * rl;
        r0 = fmaxf(r0, r[s + l]);
    }
    part[0][tid] = m0;
    part[1][tid] = i0;
    rpart[tid] = r0;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) {
            part[0][tid] += part[0][tid + k];
            part[1][tid] += part[1][tid + k];
            rpart[tid] = fmaxf(rpart[tid], rpart[tid + k]);
        }
        __syncthreads();
    }
    const double ratio = tg[0] * area / part[0][0];
    if (max_ratio > 0.0) {
        // inertia scales with the fourth power of the radius scale
        const double spin = fabs(tg[3]) * area / (part[1][0] * ratio * ratio);
        const double speed = sqrt(tg[1] * tg[1] + tg[2] * tg[2]) / tg[0];
        if (ratio > max_ratio || ratio * max_ratio < 1.0 || speed > max_speed || spin > max_spin) {
            if (tid == 0) status[blockIdx.x] = RS_INVALID;
            return;
        }
    }
    __syncthreads();
    double sc = sqrt(ratio);
    const double lim = (double)r_lim / (double)rpart[0];
    const bool clamped = sc > lim;
    if (clamped) sc = lim;
    __syncthreads();
    // rescale the radii, then the sums of the rescaled cell
    double acc[5] = {0, 0, 0, 0, 0};   // M, sum m u, sum m v, L, sum I
    for (int l = tid; l < n; l += 256) {
        const float rn = fminf((float)((double)r[s + l] * sc), r_lim);
        r[s + l] = rn;
        const double rl = rn;
        const double m = rho_ice * (double)h[s + l] * kPi * rl * rl;
        acc[0] += m;
        acc[1] += m * (double)u[s + l];
        acc[2] += m * (double)v[s + l];
        acc[3] += m * rl * rl * (double)w[s + l];
        acc[4] += m * rl * rl;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) part[k][tid] = acc[k];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k)
#pragma unroll
            for (int q = 0; q < 5; ++q) part[q][tid] += part[q][tid + k];
        __syncthreads();
    }
    if (tid < 5) tot[tid] = part[tid][0];
    __syncthreads();
    const double dvx = (tg[1] * area - tot[1]) / tot[0];
    const double dvy = (tg[2] * area - tot[2]) / tot[0];
    const double dw = (tg[3] * area - tot[3]) / tot[4];
    for (int l = tid; l < n; l += 256) {
        u[s + l] = (float)((double)u[s + l] + dvx);
        v[s + l] = (float)((double)v[s + l] + dvy);
        w[s + l] = (float)((double)w[s + l] + dw);
    }
    if (tid == 0) status[blockIdx.x] = clamped ? RS_CLAMPED : RS_OK;
}

// Features (layout of features_kernel) of the listed cells into consecutive rows.
__global__ void features_list_kernel(const int32_t* cells, int ncl, const double* Q, int nx, int ny,
                                     const float2* phase, int nmodes, Modes modes, float u0, float v0,
                                     const float* desc, float* x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    const int c = cells[i];
    const int nc = nx * ny;
    const int ix = c % nx, iy = c / nx;
    float* o = x + (size_t)i * spmlp::kIn;
    int k = 0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = (iy + dy + ny) % ny;
        for (int dx = -1; dx <= 1; ++dx) {
            const int nb = yy * nx + (ix + dx + nx) % nx;
#pragma unroll
            for (int f = 0; f < 4; ++f) o[k++] = (float)Q[(size_t)f * nc + nb];
        }
    }
    float uo = u0, vo = v0, zeta = 0.0f;
    for (int m = 0; m < nmodes; ++m) {
        const float2 sc = phase[(size_t)c * nmodes + m];
        uo += modes.au[m] * sc.x;
        vo += modes.av[m] * sc.x;
        zeta += modes.cz[m] * sc.y;
    }
    o[36] = uo;
    o[37] = vo;
    o[38] = zeta;
#pragma unroll
    for (int q = 0; q < 6; ++q) o[39 + q] = desc[(size_t)c * 6 + q];
}

// Continuum coefficient <v> = P / rho (coarse_velocity) of the listed closure cells.
__global__ void closure_coeff_kernel(const int32_t* cells, int ncl, const double* Q, int nc, double* mom)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    const int c = cells[i];
    mom[(size_t)c * kMomStride + M_UBAR] = coarse_velocity(Q, nc, c, 1);
    mom[(size_t)c * kMomStride + M_VBAR] = coarse_velocity(Q, nc, c, 2);
}

// Continuum step of the hybrid: closure cells relax_cell(Qs) + dT T (Qs: the
// transported state, T: the network's residual tendency for its features), the
// others the LF step of their statistics.
__global__ void hybrid_continuum_kernel(const double* mom, const double* Q, const double* Qs, double* Qn,
                                        const int32_t* row, const float* T, const double* mf, const float2* phase,
                                        int nmodes, Modes modes, float u0, float v0, int nx, int ny, double dT,
                                        double dX, double dY, double inv_area, unsigned long long* max_cfl_bits,
                                        uint32_t* err)
{
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = nx * ny;
    if (C >= nc) return;
    const int q = row[C];
    if (q >= 0) {
        double b[4];
        relax_cell(C, Qs, nc, mf, phase, nmodes, modes, u0, v0, dT, b);
#pragma unroll
        for (int f = 0; f < 4; ++f) Qn[(size_t)f * nc + C] = b[f] + dT * (double)T[(size_t)q * 4 + f];
    } else {
        lf_cell(C, mom, Q, Qn, nx, ny, dT, dX, dY, inv_area, max_cfl_bits, err);
    }
}

// Plain-method residual tendency (LF(Q) - relax_cell(Qs)) / dT of the listed
// cells: their own coefficients and sources from the statistics `fresh`, the
// neighbours' coefficients from `mom`; Qs is the transported state.
__global__ void check_tendency_kernel(const int32_t* cells, int ncl, const double* fresh, const double* mom,
                                      const double* Q, const double* Qs, const double* mf, const float2* phase,
                                      int nmodes, Modes modes, float u0, float v0, int nx, int ny, double dT,
                                      double dX, double dY, double inv_area, float* T)
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
    double base[4];
    relax_cell(C, Qs, nc, mf, phase, nmodes, modes, u0, v0, dT, base);
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
        T[(size_t)i * 4 + f] = (float)((qn - base[f]) / dT);
    }
}

}  // namespace spdem

struct HybridState {
    sp_mlp* net = nullptr;
    std::vector<uint8_t> closure;        // cells flagged for the closure
    std::vector<int32_t> fallback_left;  // > 0: a flagged cell runs the DEM for that many more steps
    std::vector<int32_t> fallback_cells; // cells with fallback_left > 0
    int check_every = 50, check_cells = 64, fallback_steps = 100;
    double tol = 0.2;
    int64_t checks = 0, fallbacks = 0, clamped = 0, cursor = 0, hsteps = 0;
    Bucket bk[kNumBuckets];               // DEM-mode cells only
    std::vector<int32_t> clos_h;          // closure-mode cells
    int32_t* clos_d = nullptr;
    int32_t* row_d = nullptr;             // [ncells] row of a closure-mode cell in X and T, else -1
    float* X = nullptr;                   // [nclos][45]
    float* T = nullptr;                   // [nclos][4]
    int32_t* chk_d = nullptr;             // sampled cells of a check
    int32_t* rs_d = nullptr;              // their re-synchronisation status
    float* Xk = nullptr;
    float* Tk = nullptr;
    float* Tdem = nullptr;
    double* fresh = nullptr;              // statistics of re-synchronised cells [ncells][kMomStride]
    double* Qs = nullptr;                 // transported continuum state [4][ncells]
    int ndem = 0;
};

namespace {

// Limits of the state a check re-synchronises a cell to: beyond them the
// closure has failed there and the cell falls back with its floes as they are.
// The speed and spin limits keep the floes inside the range where the explicit
// quadratic drag is stable (k |du| dt < 2 with k = C_d rho_o / (rho_ice h)).
constexpr double kCheckMassRatio = 4.0;   // mass change factor
constexpr double kCheckMaxSpeed = 2.0;    // m/s
constexpr double kCheckMaxSpin = 1e-2;    // 1/s

void hybrid_free_buffers(HybridState* h)
{
    for (auto& b : h->bk) {
        if (b.work_d) (void)hipFree(b.work_d);
        if (b.q_d) (void)hipFree(b.q_d);
        b.work_d = nullptr;
        b.q_d = nullptr;
    }
    void* ps[] = {h->clos_d, h->row_d, h->X, h->T, h->chk_d, h->rs_d, h->Xk, h->Tk, h->Tdem, h->fresh, h->Qs};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    h->clos_d = h->row_d = h->chk_d = h->rs_d = nullptr;
    h->X = h->T = h->Xk = h->Tk = h->Tdem = nullptr;
    h->fresh = h->Qs = nullptr;
}

// Rebuild the DEM buckets and the closure list from the current modes.
sp_status hybrid_rebuild(sp_ctx* c)
{
    HybridState* h = c->hyb;
    std::vector<uint8_t> dem(c->ncells);
    std::vector<int32_t> row(c->ncells, -1);
    h->clos_h.clear();
    for (int i = 0; i < c->ncells; ++i) {
        const bool clos = h->closure[i] && h->fallback_left[i] == 0;
        dem[i] = clos ? 0 : 1;
        if (clos) {
            row[i] = (int32_t)h->clos_h.size();
            h->clos_h.push_back(i);
        }
    }
    h->ndem = c->ncells - (int)h->clos_h.size();
    HIP_TRY(c, hipStreamSynchronize(c->stream));   // queued work may still read the buffers replaced below
    SP_TRY(build_buckets_into(c, h->bk, c->counts_h.data(), dem.data()));
    for (auto& b : h->bk)
        if (!b.cells_h.empty()) SP_TRY(prepare_bucket(c, b));
    const size_t nclos = std::max<size_t>(1, h->clos_h.size());
    SP_TRY(dalloc(c, &h->clos_d, nclos));
    SP_TRY(dalloc(c, &h->X, nclos * spmlp::kIn));
    SP_TRY(dalloc(c, &h->T, nclos * spmlp::kOut));
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
    hipStream_t keep = net->stream;
    net->stream = c->stream;
    sp_status st = ensure_rows(net, rows);
    if (!st) st = mlp_forward(net, x, nullptr, rows, false, y);
    net->stream = keep;
    if (st) return fail(c, st, "closure network: %s", net->err.c_str());
    return SP_OK;
}

// Re-synchronise the listed cells (device list); per-cell status into status_d;
// descriptors refreshed if they exist.
sp_status resync_list(sp_ctx* c, const int32_t* cells_d, int ncl, const double* targets_d, bool guarded,
                      int32_t* status_d)
{
    if (ncl <= 0) return SP_OK;
    hipLaunchKernelGGL(resync_kernel, dim3(ncl), dim3(256), 0, c->stream, cells_d, c->cell_start, c->r, c->h, c->u,
                       c->v, c->w, targets_d, c->Q[c->kstep & 1], c->ncells, c->p.rho_ice,
                       c->p.cell_lx * c->p.cell_ly, c->r_bin, guarded ? kCheckMassRatio : 0.0, kCheckMaxSpeed,
                       kCheckMaxSpin, status_d);
    HIP_TRY(c, hipGetLastError());
    if (c->desc && c->mf) {
        hipLaunchKernelGGL(descriptors_kernel, dim3(ncl), dim3(256), 0, c->stream, cells_d, c->cell_start, c->r, c->h,
                           1.0 / (c->p.cell_lx * c->p.cell_ly), c->p.cd * c->p.rho_ocean / c->p.rho_ice, c->desc,
                           c->mf);
        HIP_TRY(c, hipGetLastError());
    }
    return SP_OK;
}

// Check a rotating sample of closure cells after a step (Q at level kstep).
sp_status hybrid_check(sp_ctx* c, double dt)
{
    HybridState* h = c->hyb;
    const int nclos = (int)h->clos_h.size();
    if (nclos == 0 || h->check_cells <= 0) return SP_OK;
    const int nk = std::min(h->check_cells, nclos);
    std::vector<int32_t> pick(nk);
    for (int i = 0; i < nk; ++i) pick[i] = h->clos_h[(size_t)((h->cursor + i) % nclos)];
    h->cursor = (h->cursor + nk) % nclos;
    HIP_TRY(c, hipMemcpyAsync(h->chk_d, pick.data(), (size_t)nk * 4, hipMemcpyHostToDevice, c->stream));
    // 1. the sampled cells' floes to their continuum state, unless it asks for a
    //    mass change beyond kCheckMassRatio: the closure has then failed there
    SP_TRY(resync_list(c, h->chk_d, nk, nullptr, true, h->rs_d));
    // 2. their statistics and the plain method's tendency; the neighbours'
    //    coefficients are those of the step just taken
    StepArgs a = make_args(c, dt);
    a.mom = h->fresh;
    hipLaunchKernelGGL(stats_kernel, dim3(nk), dim3(256), 0, c->stream, a, h->chk_d);
    HIP_TRY(c, hipGetLastError());
    const int64_t k = c->kstep - 1;
    const double inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    hipLaunchKernelGGL(transport_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, c->Q[c->kstep & 1],
                       h->Qs, c->p.nx, c->p.ny, dt, c->p.cell_lx, c->p.cell_ly);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(check_tendency_kernel, dim3((nk + 63) / 64), dim3(64), 0, c->stream, h->chk_d, nk, h->fresh,
                       c->momb[k & 1], c->Q[c->kstep & 1], h->Qs, c->mf, c->phase, c->nmodes, a.modes, a.u0, a.v0,
                       c->p.nx, c->p.ny, dt, c->p.cell_lx, c->p.cell_ly, inv_area, h->Tdem);
    HIP_TRY(c, hipGetLastError());
    // 3. the network's tendency for the same cells
    hipLaunchKernelGGL(features_list_kernel, dim3((nk + 63) / 64), dim3(64), 0, c->stream, h->chk_d, nk, h->Qs,
                       c->p.nx, c->p.ny, c->phase, c->nmodes, a.modes, a.u0, a.v0, c->desc, h->Xk);
    HIP_TRY(c, hipGetLastError());
    SP_TRY(net_forward_on(c, h->net, h->Xk, nk, h->Tk));
    std::vector<float> tm((size_t)nk * 4), td((size_t)nk * 4), ys(4);
    std::vector<int32_t> rs(nk);
    HIP_TRY(c, hipMemcpyAsync(tm.data(), h->Tk, tm.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(td.data(), h->Tdem, td.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(rs.data(), h->rs_d, rs.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ys.data(), h->net->norm + 2 * spmlp::kIn + 2 * spmlp::kOut, 16,
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    bool changed = false;
    for (int i = 0; i < nk; ++i) {
        bool bad = rs[i] == RS_INVALID;
        if (rs[i] == RS_CLAMPED) h->clamped++;
        for (int f = 0; f < 4 && !bad; ++f) {
            // relative to the DEM tendency, with a floor of a tenth of its training spread
            const double e = fabs((double)tm[i * 4 + f] - (double)td[i * 4 + f]);
            if (!(e <= h->tol * (fabs((double)td[i * 4 + f]) + 0.1 * (double)ys[f]))) bad = true;
        }
        h->checks++;
        if (bad) {
            h->fallbacks++;
            if (h->fallback_left[pick[i]] == 0) h->fallback_cells.push_back(pick[i]);
            h->fallback_left[pick[i]] = h->fallback_steps;
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
    if (c->stream) (void)hipStreamSynchronize(c->stream);
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
    if (!st) st = resync_list(c, cd, ncl, td, false, sd);
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
                        int32_t check_cells, double tol, int32_t fallback_steps)
{
    if (!c) return SP_EINVAL;
    if (!closure_cells) {
        SP_TRY(flush_lf(c));
        hybrid_free(c);
        return SP_OK;
    }
    if (!net) return fail(c, SP_EINVAL, "the hybrid needs a network");
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_hybrid_set before sp_set_floes");
    if (check_every < 1 || check_cells < 0 || !(tol > 0) || fallback_steps < 1)
        return fail(c, SP_EINVAL, "check_every and fallback_steps must be >= 1, check_cells >= 0, tol > 0");
    if (c->p.flags & SP_NO_CONTINUUM) return fail(c, SP_ESTATE, "the hybrid needs the continuum update");
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
    h->check_every = check_every;
    h->check_cells = check_cells;
    h->tol = tol;
    h->fallback_steps = fallback_steps;
    for (int q = 0; q < kNumBuckets; ++q) {
        h->bk[q].waves = c->bk[q].waves;
        h->bk[q].queue = c->bk[q].queue;
    }
    const size_t nk = (size_t)std::max(1, check_cells);
    SP_TRY(dalloc(c, &h->row_d, (size_t)c->ncells));
    SP_TRY(dalloc(c, &h->chk_d, nk));
    SP_TRY(dalloc(c, &h->rs_d, nk));
    SP_TRY(dalloc(c, &h->Xk, nk * spmlp::kIn));
    SP_TRY(dalloc(c, &h->Tk, nk * spmlp::kOut));
    SP_TRY(dalloc(c, &h->Tdem, nk * spmlp::kOut));
    SP_TRY(dalloc(c, &h->fresh, (size_t)c->ncells * kMomStride));
    SP_TRY(dalloc(c, &h->Qs, (size_t)c->ncells * 4));
    SP_TRY(upload_phase(c));
    SP_TRY(ensure_cell_data(c));
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
    // plain steps may have run since the last hybrid one
    SP_TRY(zero_queues(c, h->bk));
    c->plain_queues_stale = true;
    const StepArgs base = make_args(c, dt);
    const double inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    for (int64_t it = 0; it < nsteps; ++it) {
        const int64_t k = c->kstep;
        const int nclos = (int)h->clos_h.size();
        if (nclos > 0) {
            // transported level-k state, closure tendencies for its features,
            // closure-cell coefficients of the level-k state
            hipLaunchKernelGGL(transport_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, c->Q[k & 1],
                               h->Qs, c->p.nx, c->p.ny, dt, c->p.cell_lx, c->p.cell_ly);
            HIP_TRY(c, hipGetLastError());
            hipLaunchKernelGGL(features_list_kernel, dim3((nclos + 127) / 128), dim3(128), 0, c->stream, h->clos_d,
                               nclos, h->Qs, c->p.nx, c->p.ny, c->phase, c->nmodes, base.modes, base.u0, base.v0,
                               c->desc, h->X);
            HIP_TRY(c, hipGetLastError());
            SP_TRY(net_forward_on(c, h->net, h->X, nclos, h->T));
            hipLaunchKernelGGL(closure_coeff_kernel, dim3((nclos + 255) / 256), dim3(256), 0, c->stream, h->clos_d,
                               nclos, c->Q[k & 1], c->ncells, c->momb[k & 1]);
            HIP_TRY(c, hipGetLastError());
        }
        // DEM step of the other cells (statistics of level k)
        for (auto& b : h->bk) SP_TRY(launch_bucket(c, b, base, k, false));
        hipLaunchKernelGGL(hybrid_continuum_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream,
                           c->momb[k & 1], c->Q[k & 1], h->Qs, c->Q[(k + 1) & 1], h->row_d, h->T, c->mf, c->phase,
                           c->nmodes, base.modes, base.u0, base.v0, c->p.nx, c->p.ny, dt, c->p.cell_lx, c->p.cell_ly,
                           inv_area, c->cfl_bits_d, c->err_d);
        HIP_TRY(c, hipGetLastError());
        c->kstep++;
        c->steps++;
        h->hsteps++;
        // fallback windows that end with this step
        bool changed = false;
        size_t keep = 0;
        for (size_t i = 0; i < h->fallback_cells.size(); ++i) {
            const int32_t cell = h->fallback_cells[i];
            if (--h->fallback_left[cell] == 0) {
                changed = changed || h->closure[cell];
            } else {
                h->fallback_cells[keep++] = cell;
            }
        }
        h->fallback_cells.resize(keep);
        if (changed) SP_TRY(hybrid_rebuild(c));
        if (h->hsteps % h->check_every == 0) SP_TRY(hybrid_check(c, dt));
    }
    return SP_OK;
}

sp_status sp_hybrid_stats(sp_ctx* c, int32_t* dem_cells, int32_t* closure_cells, int64_t* checks,
                          int64_t* fallbacks, int64_t* clamped)
{
    if (!c) return SP_EINVAL;
    if (!c->hyb) return fail(c, SP_ESTATE, "sp_hybrid_stats before sp_hybrid_set");
    if (dem_cells) *dem_cells = c->hyb->ndem;
    if (closure_cells) *closure_cells = (int32_t)c->hyb->clos_h.size();
    if (checks) *checks = c->hyb->checks;
    if (fallbacks) *fallbacks = c->hyb->fallbacks;
    if (clamped) *clamped = c->hyb->clamped;
    return SP_OK;
}

}  // extern "C"
