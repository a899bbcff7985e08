// Two-way coupling of the coarse model and the cell DEMs with a coarse step of
// N0 fine steps (Algorithm 1; coarse step Sec. 3.2; coarse-to-fine update
// Sec. 3.3).  Included at the end of spdem.hip, after hybrid_host.h.
//
// Fine step j writes the statistics of its pre-step state into slot
// (j - 1) mod N0 of a ring of N0 statistics buffers instead of running the
// fused continuum update.  When j is a multiple of N0 the window's mean drives
// N1 Lax-Friedrichs sub-steps of N0 dt / N1, and the statistics of the state
// reached are kept as the start values X0 of the next coarse step.  From the
// second coarse step on, when r = j mod N0 is a nonzero multiple of n_t, every
// cell with floes is re-synchronised to X0 + (r / N0) (Q - X0).
//
// Both continuum buffers hold the current coarse state between coarse steps,
// so readers that take the level of the current step find it at either
// parity.  Re-synchronised cells keep their candidate lists: the radius growth
// goes into the lists' displacement bound.
#pragma once

namespace spdem {

// mean[i] = (sum over the window's slots, oldest first) / N0, i over
// ncells x kMomStride statistics.
__global__ __launch_bounds__(256) void window_mean_kernel(const double* ring, int N0, size_t slot_len, double* mean)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= slot_len) return;
    double s = 0.0;
    for (int k = 0; k < N0; ++k) s += ring[(size_t)k * slot_len + i];
    mean[i] = s / (double)N0;
}

// Targets X0 + frac (Q - X0) of the listed cells; X0 from the statistics x0m
// (M, P_x, P_y, L over the cell area), Q [4][nc].
__global__ __launch_bounds__(256) void nudge_targets_kernel(const int32_t* cells, int ncl, const double* x0m,
                                                            const double* Q, int nc, double frac, double inv_area,
                                                            double* targets)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    const int c = cells[i];
    const double* s = x0m + (size_t)c * kMomStride;
    const double x0[4] = {s[M_MASS] * inv_area, s[M_PX] * inv_area, s[M_PY] * inv_area, s[M_L] * inv_area};
#pragma unroll
    for (int f = 0; f < 4; ++f) targets[(size_t)i * 4 + f] = x0[f] + frac * (Q[(size_t)f * nc + c] - x0[f]);
}

}  // namespace spdem

namespace {

void coupling_free(sp_ctx* c)
{
    void* ps[] = {c->cpl_ring, c->cpl_mean, c->cpl_x0, c->cpl_cells, c->cpl_tg, c->cpl_status, c->cpl_count};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    c->cpl_ring = c->cpl_mean = c->cpl_x0 = c->cpl_tg = nullptr;
    c->cpl_cells = c->cpl_status = nullptr;
    c->cpl_count = nullptr;
    c->cpl_ring_slots = 0;
    c->cpl_ncl = 0;
}

// Buffers of the coupled step for the current floes (the ring starts zeroed:
// cells without floes keep zero statistics in every slot).
sp_status coupling_prepare(sp_ctx* c)
{
    if (c->cpl_ring && c->cpl_ring_slots == c->N0) return SP_OK;
    coupling_free(c);
    const size_t slot = (size_t)c->ncells * kMomStride;
    SP_TRY(dalloc(c, &c->cpl_ring, slot * (size_t)c->N0));
    SP_TRY(dalloc(c, &c->cpl_mean, slot));
    SP_TRY(dalloc(c, &c->cpl_x0, slot));
    SP_TRY(dalloc(c, &c->cpl_count, 2));
    HIP_TRY(c, hipMemsetAsync(c->cpl_ring, 0, slot * (size_t)c->N0 * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->cpl_count, 0, 2 * sizeof(unsigned long long), c->stream));
    std::vector<int32_t> cells;
    for (int i = 0; i < c->ncells; ++i)
        if (c->counts_h[i] > 0) cells.push_back(i);
    c->cpl_ncl = (int)cells.size();
    const size_t m = std::max<size_t>(1, cells.size());
    SP_TRY(dalloc(c, &c->cpl_cells, m));
    SP_TRY(dalloc(c, &c->cpl_tg, m * 4));
    SP_TRY(dalloc(c, &c->cpl_status, m));
    if (!cells.empty())
        HIP_TRY(c, hipMemcpyAsync(c->cpl_cells, cells.data(), cells.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));   // `cells` is a host temporary
    c->cpl_ring_slots = c->N0;
    return SP_OK;
}

// The coarse step that ends a window: N1 sub-steps from the window's mean,
// the result in both continuum buffers, then X0 of the next coarse step.
sp_status coarse_step(sp_ctx* c, double dt)
{
    const size_t slot = (size_t)c->ncells * kMomStride;
    hipLaunchKernelGGL(window_mean_kernel, dim3((unsigned)((slot + 255) / 256)), dim3(256), 0, c->stream,
                       c->cpl_ring, c->N0, slot, c->cpl_mean);
    HIP_TRY(c, hipGetLastError());
    const double dTs = (double)c->N0 * dt / (double)c->N1;
    const double inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    for (int i = 0; i < c->N1; ++i) {
        hipLaunchKernelGGL(lf_kernel, dim3((c->ncells + 63) / 64), dim3(64), 0, c->stream, c->cpl_mean, c->Q[i & 1],
                           c->Q[(i + 1) & 1], c->p.nx, c->p.ny, dTs, c->p.cell_lx, c->p.cell_ly, inv_area,
                           c->cfl_bits_d, c->err_d);
        HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipMemcpyAsync(c->Q[(c->N1 + 1) & 1], c->Q[c->N1 & 1], (size_t)c->ncells * 4 * 8,
                              hipMemcpyDeviceToDevice, c->stream));
    StepArgs a = make_args(c, 0.0);
    a.mom = c->cpl_x0;
    hipLaunchKernelGGL(stats_kernel, dim3(c->ncells), dim3(256), 0, c->stream, a, nullptr);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

// Re-synchronise every cell with floes to X0 + frac (Q - X0).
sp_status nudge(sp_ctx* c, double frac)
{
    if (c->cpl_ncl == 0) return SP_OK;
    const double area = c->p.cell_lx * c->p.cell_ly;
    hipLaunchKernelGGL(nudge_targets_kernel, dim3((c->cpl_ncl + 255) / 256), dim3(256), 0, c->stream, c->cpl_cells,
                       c->cpl_ncl, c->cpl_x0, c->Q[0], c->ncells, frac, 1.0 / area, c->cpl_tg);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(resync_kernel, dim3(c->cpl_ncl), dim3(256), 0, c->stream, c->cpl_cells, c->cell_start, c->r,
                       c->h, c->u, c->v, c->w, c->cpl_tg, c->ncells, c->p.rho_ice, area, c->r_bin, c->cpl_status,
                       c->vdisp, c->cpl_count);
    HIP_TRY(c, hipGetLastError());
    if (c->desc) {   // closure descriptors follow the radii
        hipLaunchKernelGGL(descriptors_kernel, dim3(c->cpl_ncl), dim3(256), 0, c->stream, c->cpl_cells, c->cell_start,
                           c->r, c->h, 1.0 / area, c->p.rho_ice, c->p.cd * c->p.rho_ocean, c->desc, c->mf);
        HIP_TRY(c, hipGetLastError());
    }
    c->cpl_nudges++;
    return SP_OK;
}

}  // namespace

// Fine steps of the coupled cadence (declared before sp_step).
sp_status coupled_steps(sp_ctx* c, const StepArgs& base, int64_t nsteps)
{
    SP_TRY(coupling_prepare(c));
    const size_t slot = (size_t)c->ncells * kMomStride;
    for (int64_t it = 0; it < nsteps; ++it) {
        double* to = c->cpl_ring + (size_t)(c->cpl_j % c->N0) * slot;
        for (auto& b : c->bk) SP_TRY(launch_bucket(c, b, base, c->kstep, false, false, to));
        c->kstep++;
        c->steps++;
        c->cpl_j++;
        const int64_t r = c->cpl_j % c->N0;
        if (r == 0) {
            SP_TRY(coarse_step(c, base.dtd));
        } else if (c->cpl_j > c->N0 && r % c->n_t == 0) {
            SP_TRY(nudge(c, (double)r / (double)c->N0));
        }
    }
    return SP_OK;
}

extern "C" {

sp_status sp_set_coupling(sp_ctx* c, int32_t N0, int32_t N1, int32_t n_t, double radius_headroom)
{
    if (!c) return SP_EINVAL;
    if (N0 < 1 || N1 < 1 || n_t < 1 || N0 > SP_MAX_COUPLING || N1 > SP_MAX_COUPLING)
        return fail(c, SP_EINVAL, "N0, N1 and n_t must be >= 1 and N0, N1 <= %d", SP_MAX_COUPLING);
    if (!(radius_headroom >= 0.0) || !std::isfinite(radius_headroom))
        return fail(c, SP_EINVAL, "radius_headroom must be finite and >= 0");
    if (N0 > 1 && (c->p.flags & SP_NO_CONTINUUM)) return fail(c, SP_ESTATE, "coupling needs the continuum update");
    if (N0 > 1 && c->hyb) return fail(c, SP_ESTATE, "the hybrid step runs with N0 = 1");
    SP_TRY(flush_lf(c));
    drop_graph(c);
    const bool was = c->N0 > 1;
    if (c->have_floes && c->ncells > 0) {
        // the current coarse state into both buffers (the coupled invariant;
        // harmless for the plain path, which reads the level's parity)
        const int k = (int)(c->kstep & 1);
        HIP_TRY(c, hipMemcpyAsync(c->Q[k ^ 1], c->Q[k], (size_t)c->ncells * 4 * 8, hipMemcpyDeviceToDevice,
                                  c->stream));
        if (was && c->cpl_nudges > 0 && c->red) SP_TRY(refresh_reduced_all(c));   // radii changed
    }
    coupling_free(c);
    c->N0 = N0;
    c->N1 = N1;
    c->n_t = n_t;
    c->cpl_j = 0;
    c->cpl_nudges = 0;
    if (c->have_floes && c->n > 0) {
        // contact search sized for the radii the updates may reach: with
        // N0 > 1, radius_headroom above the current largest radius (below a
        // quarter of the cell), else the current largest radius
        std::vector<float> rh((size_t)c->n);
        HIP_TRY(c, hipMemcpyAsync(rh.data(), c->r, rh.size() * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const float rcur = *std::max_element(rh.begin(), rh.end());
        const double quarter = 0.25 * std::min(c->p.cell_lx, c->p.cell_ly) * (1.0 - 1e-6);
        const float rplan = N0 > 1 ? (float)std::min((double)rcur * (1.0 + radius_headroom), quarter) : rcur;
        if (rplan != c->r_bin) {
            SP_TRY(plan_bins(c, rplan, true));
            SP_TRY(prepare_buckets(c));
        }
    }
    return SP_OK;
}

sp_status sp_get_coupling(sp_ctx* c, int32_t* N0, int32_t* N1, int32_t* n_t, int64_t* nudges, int64_t* clamped,
                          int64_t* invalid)
{
    if (!c) return SP_EINVAL;
    if (N0) *N0 = c->N0;
    if (N1) *N1 = c->N1;
    if (n_t) *n_t = c->n_t;
    if (nudges) *nudges = c->cpl_nudges;
    unsigned long long cnt[2] = {0, 0};
    if (c->cpl_count) {
        HIP_TRY(c, hipMemcpyAsync(cnt, c->cpl_count, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (clamped) *clamped = (int64_t)cnt[0];
    if (invalid) *invalid = (int64_t)cnt[1];
    return check_device_err(c);
}

}  // extern "C"
