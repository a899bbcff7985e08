// K fine steps of a cell per launch (temporal blocking of the plain path).
//
// With the coarse step equal to the fine step the continuum never feeds back
// into the cell DEMs (Algorithm 1 with N0 = 1 takes no coarse-to-fine update),
// so a cell's floes can stay in LDS for K consecutive steps: the floe state and
// candidate lists are read once, every step's statistics go to their own slot
// of a K-slot ring for the continuum updates that follow the launch, and the
// state is written back once.  Per step the work is the per-step kernel's:
// list rebuild when the displacement bound passes half the skin (binned or
// all-pairs search), the exact contact decision of every candidate, FP64 drag,
// contact forces in ascending partner order, the update, the FP64 statistics
// of the pre-step state.  Statistics are reduced by a transposing DPP exchange
// within rows of 16 lanes and the 4 W row totals per cell (a fixed order).  One
// floe per lane: every cell of the launch has at most 64 W floes.  A floe's
// inverse mass and inverse m r^2 are computed once per launch and kept in LDS.
// Contacts and candidate tests (list entries examined, for the VALU accounting
// of the step) are counted per lane over the block and reduced once.
// TSP: the tangential spring (SP_TANGENTIAL_SPRING); each floe's contact
// history (partners and displacements, the per-step kernel's table) is staged
// in LDS at the end of the group's memory for the block, read before the
// floe's contacts of a step and rewritten with them exactly as the per-step
// kernel does, and written back once.
#pragma once

namespace spdem {

// Coarse-to-fine update at the end of a block (two-way coupling, Sec. 3.3):
// every cell of the launch is re-synchronised to X0 + frac (Q - X0) exactly as
// resync_kernel does (radii scaled by one factor up to r_lim, then uniform
// velocity and spin shifts), its floes still in LDS.  Inactive: x0m == null.
struct BlockNudge {
    const double* x0m;                 // [ncells][kMomStride] statistics at the coarse-step start
    const double* Q;                   // [4][ncells] coarse state
    double frac;
    double area;
    float r_lim;
    float* r;                          // radii (the launch's floes are rescaled in place)
    unsigned long long* counters;      // clamped, invalid cell updates
};

// Sum of one value per lane over a group of W wavefronts: DPP row sums, then
// the 4 W row totals in a fixed order (every lane gets the same value).  Every
// thread of the workgroup calls it.
template <int W>
__device__ __forceinline__ double group_sum_rows(double x, double* rows_g, int gt)
{
    x = row_sum(x);
    if ((gt & 15) == 15) rows_g[gt >> 4] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll 8
    for (int q = 0; q < 4 * W; ++q) t += rows_g[q];
    __syncthreads();
    return t;
}

template <int W>
__device__ __forceinline__ float group_max(float x, float* wmax_g, int gt)
{
    x = wave_max_f32(x);
    if ((gt & 63) == 0) wmax_g[gt >> 6] = x;
    __syncthreads();
    float t = 0.0f;
#pragma unroll
    for (int q = 0; q < W; ++q) t = fmaxf(t, wmax_g[q]);
    __syncthreads();
    return t;
}

// Five waves per SIMD: the step loop keeps more state live than one step does,
// and five resident waves with a few spilled registers beat three without.
// W = 16 (cells of up to 1024 floes) fills a compute unit's LDS with one cell:
// four waves per SIMD, the register file without spills.
template <int SCHED, int W, bool TSP = false>
__global__ __launch_bounds__(W >= 4 ? 64 * W : 256) __attribute__((amdgpu_waves_per_eu(W >= 16 ? 4 : 5)))
void dem_block_kernel(StepArgs a, int K, BlockNudge nd)
{
    constexpr int G = 64 * W;                  // threads per group (one floe per lane)
    constexpr int BT = G >= 256 ? G : 256;
    constexpr int GPB = BT / G;
    const int gpb = blockDim.x / G;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ ModeC mode_c[GPB][SP_MAX_MODES];        // per-cell mode constants (mode_consts)
    __shared__ int wsum[GPB][W];
    __shared__ float wdisp[BT / 64];
    __shared__ unsigned long long csum[BT / 64];
    __shared__ unsigned long long tsum[BT / 64];
    __shared__ double rows[GPB][kDyn][4 * W];  // row totals of every statistic
    __shared__ float vds[GPB];

    const int tid = threadIdx.x;
    const int g = tid / G, gt = tid % G;
    unsigned char* gsm = smem + (size_t)g * a.group_bytes;
    const int cap = a.cap;

    uint4* P = reinterpret_cast<uint4*>(gsm);                 // xi, yi, r bits, theta bits
    float4* V = reinterpret_cast<float4*>(P + cap);           // u, v, w, h
    double2* IM = reinterpret_cast<double2*>(V + cap);        // 1 / m, 1 / (m r^2)
    uint4* S = reinterpret_cast<uint4*>(IM + cap);            // sorted copy (binned search)
    uint16_t* lst = reinterpret_cast<uint16_t*>(S + (SCHED == 2 ? cap : 0));
    int* cnt = reinterpret_cast<int*>(lst + (size_t)cap * kListCap);
    int* binof = reinterpret_cast<int*>(lst);                 // sort scratch inside the lists
    int* rank = binof + cap;
    int* bcnt = cnt + cap;
    int* bstart = bcnt + (SCHED == 2 ? a.nbx * a.nby : 0);
    // contact history (TSP): displacements [cap][SP_SPRING_CAP], then partners [cap]
    double* const HX = TSP ? reinterpret_cast<double*>(gsm + a.group_bytes - (size_t)cap * kSpringBytes) : nullptr;
    uint4* const HJ = TSP ? reinterpret_cast<uint4*>(HX + (size_t)cap * SP_SPRING_CAP) : nullptr;

    const int item = blockIdx.x * gpb + g;
    const bool valid = item < a.ncl;
    int4 wk = valid ? a.work[item] : make_int4(0, 0, 0, 0);
    // a wavefront lies within one group: its work entry is uniform (scalar registers)
    wk.x = __builtin_amdgcn_readfirstlane(wk.x);
    wk.y = __builtin_amdgcn_readfirstlane(wk.y);
    wk.z = __builtin_amdgcn_readfirstlane(wk.z);
    wk.w = __builtin_amdgcn_readfirstlane(wk.w);
    const int c = wk.x, s = wk.y, n = wk.z;
    const bool has = valid && gt < n;          // this lane's floe
    const size_t slot_len = (size_t)a.ncells * kMomStride;
    uint16_t* const vlst = a.vlist + (size_t)s * kListCap;

    if (valid && gt < a.nmodes) mode_consts(a.modes, gt, a.phase[(size_t)c * a.nmodes + gt], mode_c[g]);
    float vd = valid ? a.vdisp[c] : 0.0f;
    if (has) {
        P[gt] = make_uint4(a.xi[s + gt], a.yi[s + gt], __float_as_uint(a.r[s + gt]), __float_as_uint(a.th[s + gt]));
        V[gt] = make_float4(a.u[s + gt], a.v[s + gt], a.w[s + gt], a.h[s + gt]);
        {
            const double rld = (double)a.r[s + gt];
            const double md = a.rho_ice_d * (double)a.h[s + gt] * kPi * rld * rld;
            IM[gt] = make_double2(1.0 / md, 1.0 / (md * (rld * rld)));
        }
        if (TSP) {
            HJ[gt] = a.tsp_j[s + gt];
#pragma unroll
            for (int q = 0; q < SP_SPRING_CAP; ++q) HX[gt * SP_SPRING_CAP + q] = a.tsp_x[(size_t)(s + gt) * SP_SPRING_CAP + q];
        }
        if (vd <= 0.5f * a.skin) {   // the kept lists are valid for the first step
            const int k = a.vcount[s + gt];
            cnt[gt] = k;
            uint16_t* my = lst + (size_t)gt * kListCap;
            for (int q = 0; q < k; q += 8)
                *reinterpret_cast<uint4*>(my + q) = *reinterpret_cast<const uint4*>(vlst + (size_t)q * n + (size_t)gt * 8);
        }
    }
    bool rebuilt = false;
    uint32_t my_contacts = 0, my_tests = 0;    // this lane's counts over the block
    // whether some cell of the workgroup rebuilds its lists this step, from the
    // displacement bounds in vds (the barrier also publishes the staged state)
    if (valid && gt == 0) vds[g] = vd;
    __syncthreads();
    auto any_rebuild = [&]() {
        bool any = false;
        for (int q = 0; q < gpb; ++q)
            any = any || (blockIdx.x * gpb + q < a.ncl && !(vds[q] <= 0.5f * a.skin));
        return any;
    };
    bool any_build = any_rebuild();

    for (int step = 0; step < K; ++step) {
        const bool build = valid && !(vd <= 0.5f * a.skin);
        const int nb_build = build ? n : 0;
        if (build && has) cnt[gt] = 0;
        if (SCHED == 2 && any_build) {
            const int nb = a.nbx * a.nby;
            for (int b = gt; b < nb; b += G) bcnt[b] = 0;
            __syncthreads();
            if (gt < nb_build) {
                const int bx = (int)__umulhi(P[gt].x, (uint32_t)a.nbx);
                const int by = (int)__umulhi(P[gt].y, (uint32_t)a.nby);
                const int b = by * a.nbx + bx;
                binof[gt] = b;
                rank[gt] = atomicAdd(&bcnt[b], 1);
            }
            __syncthreads();
            group_exclusive_scan<G>(bcnt, bstart, nb, gt, wsum[g]);
            if (gt < nb_build) {
                uint4 p = P[gt];
                p.w = (uint32_t)gt | ((uint32_t)binof[gt] << 16);
                S[bstart[binof[gt]] + rank[gt]] = p;
            }
            __syncthreads();
        }
        // ---- candidate lists (rebuilding cells only)
        if (SCHED == 1) {
            if (gt < nb_build) {
                const uint4 pl = P[gt];
                const float rl = __uint_as_float(pl.z) + a.skin;
                uint16_t* my = lst + (size_t)gt * kListCap;
                int k = 0;
                for (int j = 0; j < n; ++j) {
                    const uint4 pj = P[j];
                    float diff, R2;
                    screen((int)(pj.x - pl.x), (int)(pj.y - pl.y), rl, __uint_as_float(pj.z), a.qx, a.qy, diff, R2);
                    if (diff < kGuard * R2) {
                        if (k < kListCap) my[k] = (uint16_t)j;
                        ++k;
                    }
                }
                cnt[gt] = k;
            }
        } else if (gt < nb_build) {
            const int t = gt;
            const uint4 own = S[t];
            const int o = (int)(own.w & 0xffffu);
            const int b = (int)(own.w >> 16);
            const int bx = b % a.nbx, by = b / a.nbx;
            const float rl = __uint_as_float(own.z) + a.skin;
            if (a.nbx >= 3 && bx + 1 < a.nbx) {
                sweep(S, t + 1, bstart[b + 2], own.x, own.y, rl, o, lst, cnt, a);
            } else {
                sweep(S, t + 1, bstart[b + 1], own.x, own.y, rl, o, lst, cnt, a);
                if (a.nbx >= 3) {
                    const int be = by * a.nbx;
                    sweep(S, bstart[be], bstart[be + 1], own.x, own.y, rl, o, lst, cnt, a);
                }
            }
            if (a.nby >= 3) {
                const int row = (by + 1 == a.nby ? 0 : by + 1) * a.nbx;
                if (a.nbx < 3) {
                    sweep(S, bstart[row], bstart[row + a.nbx], own.x, own.y, rl, o, lst, cnt, a);
                } else if (bx == 0) {
                    sweep(S, bstart[row], bstart[row + 2], own.x, own.y, rl, o, lst, cnt, a);
                    sweep(S, bstart[row + a.nbx - 1], bstart[row + a.nbx], own.x, own.y, rl, o, lst, cnt, a);
                } else if (bx == a.nbx - 1) {
                    sweep(S, bstart[row + a.nbx - 2], bstart[row + a.nbx], own.x, own.y, rl, o, lst, cnt, a);
                    sweep(S, bstart[row], bstart[row + 1], own.x, own.y, rl, o, lst, cnt, a);
                } else {
                    sweep(S, bstart[row + bx - 1], bstart[row + bx + 2], own.x, own.y, rl, o, lst, cnt, a);
                }
            }
        }
        if (any_build) __syncthreads();   // lists complete (sweeps append to partners' lists)

        double acc[kDyn];
#pragma unroll
        for (int k = 0; k < kDyn; ++k) acc[k] = 0.0;
        float maxdisp = 0.0f;
        uint4 pn = make_uint4(0, 0, 0, 0);
        float4 vn4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        // ---- per floe: drag, decisions of the listed candidates (contacts as a
        // bit mask over the ascending list)
        const uint4 pl = has ? P[gt] : make_uint4(0, 0, 0, 0);
        const float4 vv = has ? V[gt] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const double rld = (double)__uint_as_float(pl.z), uld = (double)vv.x, vld = (double)vv.y,
                     wld = (double)vv.z;
        double fdx = 0.0, fdy = 0.0, tdr = 0.0;
        uint16_t* const my = lst + (size_t)gt * kListCap;
        uint32_t cmask = 0;
        if (has) {
            const int l = gt;
            if (!(a.flags & SP_OCEAN_OFF)) {
                const float fx = (float)(int)(pl.x - 0x80000000u) * 2.3283064365386963e-10f;
                const float fy = (float)(int)(pl.y - 0x80000000u) * 2.3283064365386963e-10f;
                double uo = a.u0, vo = a.v0, zeta = 0.0;
                ocean_modes(fx, fy, mode_c[g], a.nmodes, a.modes.direct != 0, uo, vo, zeta);
                const double du = uo - uld, dv = vo - vld;
                const double sp = sqrt_nonneg(du * du + dv * dv);
                const double alpha = a.cdrho * kPi * rld * rld;
                fdx = alpha * du * sp;
                fdy = alpha * dv * sp;
                const double dW = 0.5 * zeta - wld;
                const double r2 = rld * rld;
                const double beta = a.cdrho * kPi * r2 * r2 * rld;
                tdr = beta * dW * fabs(dW);
            }
            int k = cnt[l];
            if (build) {
                if (k > kListCap) {
                    atomicOr(a.err, kErrCapacity);
                    k = kListCap;
                    cnt[l] = k;
                }
                if (SCHED == 2) {
                    for (int i = 1; i < k; ++i) {
                        const uint16_t key = my[i];
                        int j = i - 1;
                        while (j >= 0 && my[j] > key) {
                            my[j + 1] = my[j];
                            --j;
                        }
                        my[j + 1] = key;
                    }
                }
            }
            my_tests += (uint32_t)k;
            // four candidates at a time: their partners' positions loaded
            // together (an index past the list reads the floe itself and is
            // skipped), then decided
            for (int q0 = 0; q0 < k; q0 += 4) {
                const uint2 ix = *reinterpret_cast<const uint2*>(my + q0);
                int jv[4];
                jv[0] = (int)(ix.x & 0xffffu);
                jv[1] = (int)(ix.x >> 16);
                jv[2] = (int)(ix.y & 0xffffu);
                jv[3] = (int)(ix.y >> 16);
                uint4 pj[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    jv[t] = q0 + t < k ? jv[t] : l;
                    pj[t] = P[jv[t]];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (jv[t] != l &&
                        decide((int)(pj[t].x - pl.x), (int)(pj[t].y - pl.y), __uint_as_float(pl.z),
                               __uint_as_float(pj[t].z), a))
                        cmask |= 1u << (q0 + t);
            }
            // ---- contact forces and torques in ascending partner order (FP64)
            double Fx = fdx, Fy = fdy, T = tdr;
            // the floe's contact history (TSP), rewritten below with this step's contacts
            uint4 hj = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
            double hx[SP_SPRING_CAP];
            uint16_t* const tj = TSP ? reinterpret_cast<uint16_t*>(HJ + l) : nullptr;
            double* const tx = TSP ? HX + (size_t)l * SP_SPRING_CAP : nullptr;
            bool had = false;   // the floe was in contact after the previous step
            if (TSP) {
                hj = HJ[l];
                had = (hj.x & hj.y & hj.z & hj.w) != 0xffffffffu;
#pragma unroll
                for (int q = 0; q < SP_SPRING_CAP; ++q) hx[q] = had ? tx[q] : 0.0;
            }
            int nh = 0;
            while (cmask) {
                const int q = __builtin_ctz(cmask);
                cmask &= cmask - 1u;
                const int j = my[q];
                const uint4 pj = P[j];
                double cx, cy, ct, xi = 0.0, xi_old = 0.0;
                if (TSP) {
#pragma unroll
                    for (int e = 0; e < SP_SPRING_CAP; ++e) {
                        const uint32_t wv = e < 2 ? hj.x : e < 4 ? hj.y : e < 6 ? hj.z : hj.w;
                        if ((int)((wv >> (16 * (e & 1))) & 0xffffu) == j) xi_old = hx[e];
                    }
                }
                if (!contact_terms<TSP>((int)(pj.x - pl.x), (int)(pj.y - pl.y), rld, uld, vld, wld,
                                        __uint_as_float(pj.z), V[j], l < j, a, cx, cy, ct, xi_old, &xi)) {
                    atomicOr(a.err, kErrOverlap);
                    continue;
                }
                if (TSP) {
                    if (nh < SP_SPRING_CAP) {
                        tj[nh] = (uint16_t)j;
                        tx[nh] = xi;
                    } else {
                        atomicOr(a.err, kErrCapacity);
                    }
                    ++nh;
                }
                add_terms(Fx, Fy, T, cx, cy, ct);
                my_contacts += (l < j) ? 1u : 0u;
            }
            if (TSP && (had || nh > 0))   // a floe out of contact before and now keeps its empty table
                for (int e = nh; e < SP_SPRING_CAP; ++e) {
                    tj[e] = 0xffffu;
                    tx[e] = 0.0;
                }
            const double2 im = IM[l];
            const double inv_m = im.x, inv_i = im.y;
            const double md = a.rho_ice_d * (double)vv.w * kPi * rld * rld;
            const double dt = a.dtd;
            const double und = uld + dt * (Fx * inv_m);
            const double vnd = vld + dt * (Fy * inv_m);
            const double wnd = wld + dt * (T * inv_i);
            const bool fe = (a.flags & SP_FORWARD_EULER) != 0;
            const double ux = fe ? uld : und, vx = fe ? vld : vnd, wx = fe ? wld : wnd;
            const int sx = __double2int_rn(dt * ux * a.inv_qxd);
            const int sy = __double2int_rn(dt * vx * a.inv_qyd);
            {
                const float ddx = (float)sx * a.qx, ddy = (float)sy * a.qy;
                maxdisp = ddx * ddx + ddy * ddy;   // squared: one root per cell below
            }
            const float un = (float)und, vn = (float)vnd, wn = (float)wnd;
            pn = make_uint4(pl.x + (uint32_t)sx, pl.y + (uint32_t)sy, pl.z,
                            __float_as_uint((float)((double)__uint_as_float(pl.w) + dt * wx)));
            vn4 = make_float4(un, vn, wn, vv.w);
            if (!(isfinite(un) && isfinite(vn) && isfinite(wn))) atomicOr(a.err, kErrNaN);
            acc[0] = md * uld;
            acc[1] = md * vld;
            acc[2] = md * rld * rld * wld;
            acc[3] = uld;
            acc[4] = vld;
            acc[5] = fdx;
            acc[6] = fdy;
            acc[7] = tdr;
        }
        // ---- group reductions (the floe data is still read by nobody after this barrier)
        const float wd = wave_max_nonneg(maxdisp);
        {
            const double x = row_sum8(acc, gt & 15);
            if ((gt & 1) == 0) rows[g][(gt & 15) >> 1][gt >> 4] = x;
        }
        if ((tid & 63) == 0) wdisp[tid >> 6] = wd;
        __syncthreads();
        if (has) {                               // the new state, for the next step
            P[gt] = pn;
            V[gt] = vn4;
        }
        if (valid && gt < kDyn) {
            double x = 0.0;
#pragma unroll 8
            for (int q = 0; q < 4 * W; ++q) x += rows[g][gt][q];
            const int slot = dyn_slot(gt);
            double* const mo = (wk.w ? a.mom_alt : a.mom + (size_t)step * slot_len) + (size_t)c * kMomStride;
            mo[slot] = x;
            if (slot == M_UX || slot == M_UY) mo[slot == M_UX ? M_UBAR : M_VBAR] = n > 0 ? x / (double)n : 0.0;
        }
        if (valid && gt == 0) {
            float d = 0.0f;
            for (int q = 0; q < W; ++q) d = fmaxf(d, wdisp[g * W + q]);
            vds[g] = (build ? 0.0f : vd) + sqrtf(d) * 1.0001f + 1e-3f;
        }
        rebuilt = rebuilt || build;
        __syncthreads();
        vd = valid ? vds[g] : 0.0f;
        any_build = any_rebuild();
    }

    unsigned long long ctot = 0, ttot = 0;
    {
        const unsigned long long cs = wave_sum_u64(my_contacts);
        const unsigned long long ts = wave_sum_u64(my_tests);
        if ((tid & 63) == 0) {
            csum[tid >> 6] = cs;
            tsum[tid >> 6] = ts;
        }
        __syncthreads();
        if (valid && gt == 0)
            for (int q = 0; q < W; ++q) {
                ctot += csum[g * W + q];
                ttot += tsum[g * W + q];
            }
    }

    // ---- coarse-to-fine update of the cell (coupled cadence)
    if (nd.x0m) {
        double tg[4] = {0.0, 0.0, 0.0, 0.0};
        if (valid) {
            const double* st = nd.x0m + (size_t)c * kMomStride;
            const double inv_area = 1.0 / nd.area;
            const double x0[4] = {st[M_MASS] * inv_area, st[M_PX] * inv_area, st[M_PY] * inv_area,
                                  st[M_L] * inv_area};
#pragma unroll
            for (int f = 0; f < 4; ++f) tg[f] = x0[f] + nd.frac * (nd.Q[(size_t)f * a.ncells + c] - x0[f]);
        }
        const bool ok = valid && n > 0 && isfinite(tg[0]) && isfinite(tg[1]) && isfinite(tg[2]) &&
                        isfinite(tg[3]) && tg[0] > 0.0;
        if (valid && !ok && gt == 0 && nd.counters) atomicAdd(&nd.counters[1], 1ull);
        const uint4 p0 = has ? P[gt] : make_uint4(0, 0, 0, 0);
        const float4 v0 = has ? V[gt] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float ro = __uint_as_float(p0.z);
        const double rod = ro;
        const double mass = group_sum_rows<W>(has ? a.rho_ice_d * (double)v0.w * kPi * rod * rod : 0.0,
                                              rows[g][0], gt);
        const float rmax = group_max<W>(has ? ro : 0.0f, wdisp + g * W, gt);
        double sc = ok ? sqrt(tg[0] * nd.area / mass) : 1.0;
        const bool clamped = ok && sc > (double)nd.r_lim / (double)rmax;
        if (clamped) sc = (double)nd.r_lim / (double)rmax;
        const float rn = (ok && has) ? fminf((float)(rod * sc), nd.r_lim) : ro;
        const double rnd = rn;
        const double m = has ? a.rho_ice_d * (double)v0.w * kPi * rnd * rnd : 0.0;
        const double M = group_sum_rows<W>(m, rows[g][1], gt);
        const double Px = group_sum_rows<W>(m * (double)v0.x, rows[g][2], gt);
        const double Py = group_sum_rows<W>(m * (double)v0.y, rows[g][3], gt);
        const double L = group_sum_rows<W>(m * rnd * rnd * (double)v0.z, rows[g][4], gt);
        const double I = group_sum_rows<W>(m * rnd * rnd, rows[g][5], gt);
        const float gmax = group_max<W>(has ? rn - ro : 0.0f, wdisp + g * W, gt);
        if (ok && has) {
            const double dvx = (tg[1] * nd.area - Px) / M;
            const double dvy = (tg[2] * nd.area - Py) / M;
            const double dw = (tg[3] * nd.area - L) / I;
            P[gt].z = __float_as_uint(rn);
            V[gt] = make_float4((float)((double)v0.x + dvx), (float)((double)v0.y + dvy),
                                (float)((double)v0.z + dw), v0.w);
            nd.r[s + gt] = rn;
        }
        if (ok && gt == 0) {
            if (gmax > 0.0f) vd = (vd + gmax * (1.0f + 0x1p-22f)) * (1.0f + 0x1p-22f);
            if (clamped && nd.counters) atomicAdd(&nd.counters[0], 1ull);
        }
        __syncthreads();
    }

    // ---- state, lists, bound and contact count back to HBM (the floe index
    // formed afresh from the scalar cell start: nothing per lane is kept
    // across the step loop for it)
    int s_end = s;
    asm volatile("" : "+s"(s_end));
    const int fi = s_end + gt;
    if (has) {
        const uint4 p = P[gt];
        const float4 v = V[gt];
        a.xi[fi] = p.x;
        a.yi[fi] = p.y;
        a.th[fi] = __uint_as_float(p.w);
        a.u[fi] = v.x;
        a.v[fi] = v.y;
        a.w[fi] = v.z;
        if (TSP) {
            a.tsp_j[fi] = HJ[gt];
#pragma unroll
            for (int q = 0; q < SP_SPRING_CAP; ++q) a.tsp_x[(size_t)fi * SP_SPRING_CAP + q] = HX[gt * SP_SPRING_CAP + q];
        }
        if (rebuilt) {
            const int k = cnt[gt];
            const uint16_t* my = lst + (size_t)gt * kListCap;
            for (int q = 0; q < k; ++q) vlst[(size_t)(q & ~7) * n + (size_t)gt * 8 + (q & 7)] = my[q];
            a.vcount[fi] = (uint8_t)k;
        }
    }
    if (valid && gt == 0) {
        a.vdisp[c] = vd;
        a.contacts[c] += ctot;   // read here, not at the start: nothing long-lived
        a.cands[c] += ttot;
    }
}

}  // namespace spdem
