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
// goes into the lists' displacement bound.  The contact search is re-planned
// at coarse steps for the largest radius the next coarse step's updates can
// produce (known then: a cell's radii scale by sqrt(rho_target / rho_X0) and
// its targets lie between X0 and Q), so radii are limited only by a quarter of
// the cell, the limit of the periodic cell DEM.
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

// Largest radius the next coarse step's updates can produce: a cell's radii
// stay below rmax_cell sqrt(max(1, Q_rho / X0_rho)).  Each wavefront strides
// over the listed cells; one atomic maximum per workgroup (plus a rounding
// margin) into *out as float bits (positive floats order as their bit
// patterns).
__global__ __launch_bounds__(256) void window_radius_kernel(const int32_t* cells, int ncl, const int32_t* cell_start,
                                                            const float* r, const double* x0m, const double* Q,
                                                            int nc, double inv_area, unsigned int* out)
{
    __shared__ float wmax[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float best = 0.0f;
    for (int i = blockIdx.x * 4 + wv; i < ncl; i += gridDim.x * 4) {
        const int c = cells[i];
        const int s = cell_start[c], n = cell_start[c + 1] - s;
        float m = 0.0f;
        for (int l = lane; l < n; l += 64) m = fmaxf(m, r[s + l]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        const double x0 = x0m[(size_t)c * kMomStride + M_MASS] * inv_area;
        const double q = Q[c];
        const double f = (x0 > 0.0 && q > x0) ? sqrt(q / x0) : 1.0;
        best = fmaxf(best, (float)((double)m * f * (1.0 + 1e-5)));
    }
    if (lane == 0) wmax[wv] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        atomicMax(out, __float_as_uint(b));
    }
}

}  // namespace spdem

namespace {

// Re-planning of the contact search at coarse steps: grow to the required
// radius plus kPlanMargin; shrink once the requirement falls below
// r_bin / kShrinkRatio.  The skin stays at most the one planned for the floes
// as they were set: sub-bins sized for a few grown floes must not widen every
// floe's candidate list (its capacity is fixed).
constexpr double kPlanMargin = 0.05;
constexpr double kShrinkRatio = 1.2;

sp_status plan_for_radius(sp_ctx* c, float req)
{
    const double quarter = 0.25 * std::min(c->p.cell_lx, c->p.cell_ly) * (1.0 - 1e-6);
    if (req <= c->r_bin && (double)req * kShrinkRatio >= (double)c->r_bin) return SP_OK;
    const float rplan = (float)std::min((double)req * (1.0 + kPlanMargin), quarter);
    if (rplan == c->r_bin) return SP_OK;
    SP_TRY(plan_bins(c, rplan, true, c->skin_set));
    SP_TRY(prepare_buckets(c));
    c->cpl_replans++;
    return SP_OK;
}

void coupling_free(sp_ctx* c)
{
    void* ps[] = {c->cpl_ring, c->cpl_mean, c->cpl_x0, c->cpl_cells, c->cpl_count, c->cpl_rreq};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    c->cpl_ring = c->cpl_mean = c->cpl_x0 = nullptr;
    c->cpl_cells = nullptr;
    c->cpl_count = nullptr;
    c->cpl_rreq = nullptr;
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
    SP_TRY(dalloc(c, &c->cpl_rreq, 1));
    HIP_TRY(c, hipMemsetAsync(c->cpl_ring, 0, slot * (size_t)c->N0 * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->cpl_count, 0, 2 * sizeof(unsigned long long), c->stream));
    std::vector<int32_t> cells;
    for (int i = 0; i < c->ncells; ++i)
        if (c->counts_h[i] > 0) cells.push_back(i);
    c->cpl_ncl = (int)cells.size();
    const size_t m = std::max<size_t>(1, cells.size());
    SP_TRY(dalloc(c, &c->cpl_cells, m));
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
                           c->cfl_bits_d, c->err_d, wall_x(c));
        HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipMemcpyAsync(c->Q[(c->N1 + 1) & 1], c->Q[c->N1 & 1], (size_t)c->ncells * 4 * 8,
                              hipMemcpyDeviceToDevice, c->stream));
    StepArgs a = make_args(c, 0.0);
    a.mom = c->cpl_x0;
    hipLaunchKernelGGL(stats_kernel, dim3(c->ncells), dim3(256), 0, c->stream, a, nullptr, 0);
    HIP_TRY(c, hipGetLastError());
    if (c->cpl_ncl == 0 || c->N0 <= c->n_t) return SP_OK;   // no update in the next coarse step
    HIP_TRY(c, hipMemsetAsync(c->cpl_rreq, 0, sizeof(unsigned int), c->stream));
    const int rgrid = std::min((c->cpl_ncl + 3) / 4, 2 * c->num_cus);
    hipLaunchKernelGGL(window_radius_kernel, dim3(rgrid), dim3(256), 0, c->stream, c->cpl_cells, c->cpl_ncl,
                       c->cell_start, c->r, c->cpl_x0, c->Q[0], c->ncells, inv_area, c->cpl_rreq);
    HIP_TRY(c, hipGetLastError());
    unsigned int bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&bits, c->cpl_rreq, sizeof bits, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float req;
    memcpy(&req, &bits, sizeof req);
    return plan_for_radius(c, req);
}

// Re-synchronise every cell with floes to X0 + frac (Q - X0).
sp_status nudge(sp_ctx* c, double frac)
{
    if (c->cpl_ncl == 0) return SP_OK;
    const double area = c->p.cell_lx * c->p.cell_ly;
    hipLaunchKernelGGL(resync_kernel, dim3(c->cpl_ncl), dim3(64), 0, c->stream, c->cpl_cells, c->cell_start, c->r,
                       c->h, c->u, c->v, c->w, nullptr, c->cpl_x0, c->Q[0], frac, c->ncells, c->p.rho_ice, area,
                       c->r_bin, nullptr, c->vdisp, c->cpl_count);
    HIP_TRY(c, hipGetLastError());
    c->desc_stale = true;   // closure descriptors follow the radii (recomputed when next needed)
    c->cpl_nudges++;
    return SP_OK;
}

}  // namespace

// Fine steps of the coupled cadence (declared before sp_step).  Cells are
// independent between coarse-to-fine updates, and an update needs only the
// cell's own X0 and Q: with a step block above one, each stretch up to the
// next update or coarse step runs as one blocked launch per bucket (the floes
// resident in LDS, one per lane), the update done in the same launch.
sp_status coupled_steps(sp_ctx* c, const StepArgs& args, int64_t nsteps)
{
    SP_TRY(coupling_prepare(c));
    const size_t slot = (size_t)c->ncells * kMomStride;
    // the step arguments, made again after every coarse step: its re-plan of
    // the contact search changes the sub-bins, the skin and the list buffers
    StepArgs base = args;
    if (c->block_k > 1) {
        int64_t left = nsteps;
        while (left > 0) {
            const int64_t r = c->cpl_j % c->N0;
            const int64_t bound = std::min<int64_t>((r / c->n_t + 1) * c->n_t, c->N0);
            const int64_t K = std::min<int64_t>(bound - r, left);
            const int64_t jend = c->cpl_j + K;
            const int64_t rend = jend % c->N0;
            const bool update = rend != 0 && jend > c->N0 && rend % c->n_t == 0;
            BlockNudge nd;
            memset(&nd, 0, sizeof nd);
            if (update && c->cpl_ncl > 0) {
                nd.x0m = c->cpl_x0;
                nd.Q = c->Q[0];
                nd.frac = (double)rend / (double)c->N0;
                nd.area = c->p.cell_lx * c->p.cell_ly;
                nd.r_lim = c->r_bin;
                nd.r = c->r;
                nd.counters = c->cpl_count;
            }
            SP_TRY(launch_blocks(c, base, c->cpl_ring + (size_t)r * slot, (int)K, nd));
            c->kstep += K;
            c->steps += K;
            c->blk_steps += K;
            c->cpl_j = jend;
            left -= K;
            if (update && c->cpl_ncl > 0) {
                c->cpl_nudges++;
                c->desc_stale = true;
            }
            if (rend == 0) {
                SP_TRY(coarse_step(c, base.dtd));
                base = make_args(c, base.dtd);
            }
        }
        return SP_OK;
    }
    for (int64_t it = 0; it < nsteps; ++it) {
        double* to = c->cpl_ring + (size_t)(c->cpl_j % c->N0) * slot;
        for (auto& b : c->bk) SP_TRY(launch_bucket(c, b, base, c->kstep, false, false, to));
        c->kstep++;
        c->steps++;
        c->cpl_j++;
        const int64_t r = c->cpl_j % c->N0;
        if (r == 0) {
            SP_TRY(coarse_step(c, base.dtd));
            base = make_args(c, base.dtd);
        } else if (c->cpl_j > c->N0 && r % c->n_t == 0) {
            SP_TRY(nudge(c, (double)r / (double)c->N0));
        }
    }
    return SP_OK;
}

extern "C" {

sp_status sp_set_coupling(sp_ctx* c, int32_t N0, int32_t N1, int32_t n_t)
{
    if (!c) return SP_EINVAL;
    if (N0 < 1 || N1 < 1 || n_t < 1 || N0 > SP_MAX_COUPLING || N1 > SP_MAX_COUPLING)
        return fail(c, SP_EINVAL, "N0, N1 and n_t must be >= 1 and N0, N1 <= %d", SP_MAX_COUPLING);
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
    c->cpl_replans = 0;
    if (c->have_floes && c->n > 0) {
        // contact search sized for the current radii (they may have changed
        // since the floes were set); later coarse steps re-plan it
        std::vector<float> rh((size_t)c->n);
        HIP_TRY(c, hipMemcpyAsync(rh.data(), c->r, rh.size() * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const float rcur = *std::max_element(rh.begin(), rh.end());
        if (rcur != c->r_bin) {
            SP_TRY(plan_bins(c, rcur, true, c->skin_set));
            SP_TRY(prepare_buckets(c));
        }
    }
    return SP_OK;
}

sp_status sp_get_coupling(sp_ctx* c, int32_t* N0, int32_t* N1, int32_t* n_t, int64_t* nudges, int64_t* replans,
                          int64_t* clamped, int64_t* invalid)
{
    if (!c) return SP_EINVAL;
    if (N0) *N0 = c->N0;
    if (N1) *N1 = c->N1;
    if (n_t) *n_t = c->n_t;
    if (nudges) *nudges = c->cpl_nudges;
    if (replans) *replans = c->cpl_replans;
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
