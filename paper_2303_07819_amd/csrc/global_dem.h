// The global DEM of the paper's error study (Sec. 4): one DEM over the whole
// periodic domain, floes free to cross coarse cells, every pair a potential
// contact.  It is the reference ("truth") the superparameterised model is
// compared with; its coarse-grid statistics are read for that comparison.
// Included at the end of spdem.hip.
//
// Per fine step: every floe's sub-bin (side >= 2 r_max, so contacts only join
// neighbouring sub-bins) from its fixed-point position; a stable radix sort of
// (sub-bin, slot) pairs; the state gathered into sub-bin order; sub-bin starts
// by binary search; then one thread per floe sweeps the 3 x 3 neighbouring
// sub-bins, decides contacts exactly as the cell kernel does (FP32 screen, FP64
// in the guard band), sums drag and contact forces in FP64 and writes the
// updated floe in the same order.  The state stays in sub-bin order between
// steps, so the next sort moves few floes.
#pragma once

struct sp_gdem {
    sp_gdem_params p;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    double u0 = 0, v0 = 0;
    int nmodes = 0;
    double kx[SP_MAX_MODES], ky[SP_MAX_MODES], au[SP_MAX_MODES], av[SP_MAX_MODES], ph[SP_MAX_MODES];
    bool phase_dirty = true;

    int64_t n = 0;
    bool have_floes = false;
    int nbx = 1, nby = 1;
    float rmax = 0.0f;
    // floe state, two buffers; cur holds the state in sub-bin order
    uint32_t* xi[2] = {nullptr, nullptr};
    uint32_t* yi[2] = {nullptr, nullptr};
    float* u[2] = {nullptr, nullptr};
    float* v[2] = {nullptr, nullptr};
    float* w[2] = {nullptr, nullptr};
    float* th[2] = {nullptr, nullptr};
    float* r[2] = {nullptr, nullptr};
    float* h[2] = {nullptr, nullptr};
    int32_t* id[2] = {nullptr, nullptr};
    int cur = 0;
    // sort
    uint32_t* keys[2] = {nullptr, nullptr};
    int32_t* vals[2] = {nullptr, nullptr};
    void* sort_tmp = nullptr;
    size_t sort_bytes = 0;
    int32_t* bstart = nullptr;         // sub-bin starts [nbins + 1]
    int32_t* cstart = nullptr;         // coarse-cell starts (read-out)
    size_t cstart_cap = 0;
    double* cmom = nullptr;            // coarse statistics (read-out)
    size_t cmom_cap = 0;
    double2* phase = nullptr;          // (sin, cos) of every mode's phase at each sub-bin centre
    uint32_t* err_d = nullptr;
    unsigned long long* contacts_d = nullptr;
    int64_t steps = 0;
};

namespace spdem {

struct GArgs {
    // pre-step state in sub-bin order
    const uint32_t* xi;
    const uint32_t* yi;
    const float* u;
    const float* v;
    const float* w;
    const float* th;
    const float* r;
    const float* h;
    const int32_t* id;
    // updated state, same order
    uint32_t* xo;
    uint32_t* yo;
    float* uo;
    float* vo;
    float* wo;
    float* tho;
    float* ro;
    float* ho;
    int32_t* ido;
    const int32_t* bstart;
    const double2* phase;
    int n, nbx, nby, nmodes;
    uint32_t flags;
    float qx, qy;
    double u0, v0;
    double lxd;                        // domain length in x (position of the far wall with SP_WALL_X)
    double qxd, qyd, inv_qxd, inv_qyd;
    double dtd, Ed, Gd, mud, cdrho, rho_ice_d;
    Modes modes;                       // kxL, kyL per sub-bin side
    uint32_t* err;
    unsigned long long* contacts;
};

__device__ __forceinline__ uint32_t gbin_axis(uint32_t x, int nb)
{
    return (uint32_t)(((uint64_t)x * (uint64_t)nb) >> 32);
}

// Offset of a fixed-point coordinate from its sub-bin centre, in sub-bin sides.
__device__ __forceinline__ float gbin_offset(uint32_t x, int nb)
{
    const uint32_t lo = (uint32_t)((uint64_t)x * (uint64_t)nb);
    return (float)(int)(lo - 0x80000000u) * 2.3283064365386963e-10f;
}

__global__ __launch_bounds__(256) void gkey_kernel(const uint32_t* xi, const uint32_t* yi, int n, int nbx, int nby,
                                                   uint32_t* keys, int32_t* vals)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    keys[k] = gbin_axis(yi[k], nby) * (uint32_t)nbx + gbin_axis(xi[k], nbx);
    vals[k] = k;
}

__global__ __launch_bounds__(256) void ggather_kernel(const int32_t* perm, int n, const uint32_t* xi,
                                                      const uint32_t* yi, const float* u, const float* v,
                                                      const float* w, const float* th, const float* r,
                                                      const float* h, const int32_t* id, uint32_t* xo,
                                                      uint32_t* yo, float* uo, float* vo, float* wo, float* tho,
                                                      float* ro, float* ho, int32_t* ido)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int p = perm[k];
    xo[k] = xi[p];
    yo[k] = yi[p];
    uo[k] = u[p];
    vo[k] = v[p];
    wo[k] = w[p];
    tho[k] = th[p];
    ro[k] = r[p];
    ho[k] = h[p];
    ido[k] = id[p];
}

// start[b] = first position of key b in the sorted keys (b = 0 .. nb).
__global__ __launch_bounds__(256) void gstart_kernel(const uint32_t* keys, int n, int nb, int32_t* start)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < (uint32_t)b) lo = mid + 1;
        else hi = mid;
    }
    start[b] = lo;
}

// Ocean current and curl at a floe from the phase table of its sub-bin: the
// offset's sin and cos in FP32, the angle addition and the sum over modes in
// FP64 (as the cell kernels).
__device__ __forceinline__ void gocean(const GArgs& a, uint32_t x, uint32_t y, double& uo, double& vo, double& zeta)
{
    uo = a.u0;
    vo = a.v0;
    zeta = 0.0;
    if (a.nmodes == 0) return;
    const int b = (int)(gbin_axis(y, a.nby) * (uint32_t)a.nbx + gbin_axis(x, a.nbx));
    const float fx = gbin_offset(x, a.nbx), fy = gbin_offset(y, a.nby);
    const double2* ph = a.phase + (size_t)b * a.nmodes;
    for (int m = 0; m < a.nmodes; ++m) {
        const float d = a.modes.kxL[m] * fx + a.modes.kyL[m] * fy;
        float sdf, cdf;
        if (a.modes.direct)
            sincos_direct(d, sdf, cdf);
        else
            sincos_small(d, sdf, cdf);
        const double sd = sdf, cd = cdf;
        const double2 q = ph[m];
        const double sn = fma(q.x, cd, q.y * sd);
        const double cn = fma(q.y, cd, -(q.x * sd));
        uo = fma(a.modes.au[m], sn, uo);
        vo = fma(a.modes.av[m], sn, vo);
        zeta = fma(a.modes.cz[m], cn, zeta);
    }
}

// Drag force and drag torque of a floe (FP64), as in the cell kernel.
__device__ __forceinline__ void gdrag(const GArgs& a, uint32_t x, uint32_t y, double rld, double uld, double vld,
                                      double wld, double& fdx, double& fdy, double& tdr)
{
    fdx = fdy = tdr = 0.0;
    if (a.flags & SP_OCEAN_OFF) return;
    double uo, vo, zeta;
    gocean(a, x, y, uo, vo, zeta);
    const double du = uo - uld, dv = vo - vld;
    const double sp = sqrt(du * du + dv * dv);
    const double alpha = a.cdrho * kPi * rld * rld;
    fdx = alpha * du * sp;
    fdy = alpha * dv * sp;
    const double dW = 0.5 * zeta - wld;
    const double r2 = rld * rld;
    const double beta = a.cdrho * kPi * r2 * r2 * rld;
    tdr = beta * dW * fabs(dW);
}

__global__ __launch_bounds__(256) void gstep_kernel(GArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long ncontact = 0;
    if (k < a.n) {
        const uint32_t xl = a.xi[k], yl = a.yi[k];
        const float rl = a.r[k];
        const int idl = a.id[k];
        const double rld = rl, uld = a.u[k], vld = a.v[k], wld = a.w[k];
        double Fx, Fy, T;
        gdrag(a, xl, yl, rld, uld, vld, wld, Fx, Fy, T);
        const double md = a.rho_ice_d * (double)a.h[k] * kPi * rld * rld;
        const int bx = (int)gbin_axis(xl, a.nbx), by = (int)gbin_axis(yl, a.nby);
        const int oy0 = a.nby >= 3 ? -1 : 0, oy1 = a.nby >= 3 ? 1 : 0;
        const int ox0 = a.nbx >= 3 ? -1 : 0, ox1 = a.nbx >= 3 ? 1 : 0;
        const bool wall = (a.flags & SP_WALL_X) != 0;
        for (int oy = oy0; oy <= oy1; ++oy) {
            const int byy = (by + oy + a.nby) % a.nby;
            for (int ox = ox0; ox <= ox1; ++ox) {
                if (wall && (bx + ox < 0 || bx + ox >= a.nbx)) continue;   // no periodic image across a wall
                const int b = byy * a.nbx + (bx + ox + a.nbx) % a.nbx;
                const int j1 = a.bstart[b + 1];
                for (int j = a.bstart[b]; j < j1; ++j) {
                    if (j == k) continue;
                    // between walls the x difference is the plain one (pairs
                    // more than half the domain apart are far from contact)
                    const long long ddx = (long long)a.xi[j] - (long long)xl;
                    if (wall && (ddx >= 0x80000000ll || ddx < -0x80000000ll)) continue;
                    const int dxi = wall ? (int)ddx : (int)(a.xi[j] - xl), dyi = (int)(a.yi[j] - yl);
                    const float rj = a.r[j];
                    float diff, R2;
                    screen(dxi, dyi, rl, rj, a.qx, a.qy, diff, R2);
                    if (diff > kGuard * R2) continue;
                    if (fabsf(diff) <= kGuard * R2 && !exact_contact(dxi, dyi, rl, rj, a.qxd, a.qyd)) continue;
                    const double dx = (double)dxi * a.qxd, dy = (double)dyi * a.qyd;
                    const double d2 = dx * dx + dy * dy;
                    if (!(d2 > 0.0)) {
                        atomicOr(a.err, kErrOverlap);
                        continue;
                    }
                    const int idj = a.id[j];
                    const double rjd = (double)rj;
                    const double d = sqrt(d2);
                    const double inv_d = 1.0 / d;
                    const double nx = dx * inv_d, ny = dy * inv_d;
                    const double tx = -ny, ty = nx;
                    const double R = rld + rjd;
                    const double delta = d - R;
                    const double dr = fabs(rld - rjd);
                    double cc;
                    if (d <= dr) {
                        cc = 2.0 * fmin(rld, rjd);
                    } else {
                        const double p = (((-delta) * (d + R)) * (d - dr)) * (d + dr);
                        cc = sqrt(fmax(p, 0.0)) * inv_d;
                    }
                    const double Fn = cc * a.Ed * delta;
                    const double wjd = (double)a.w[j];
                    // spin sum with the lower floe id first: exactly antisymmetric pair forces
                    const double spin = (idl < idj) ? (wld * rld + wjd * rjd) : (wjd * rjd + wld * rld);
                    const double vt = (((double)a.u[j] - uld) * tx + ((double)a.v[j] - vld) * ty) - spin;
                    const double capf = a.mud * fabs(Fn);
                    const double Ft = fmin(fmax(cc * a.Gd * vt, -capf), capf);
                    Fx += Fn * nx + Ft * tx;
                    Fy += Fn * ny + Ft * ty;
                    T += rld * Ft;
                    ncontact += (idl < idj) ? 1ull : 0ull;
                }
            }
        }
        if (wall) {
            // the walls at x = 0 and x = lx, after the floe contacts: the
            // contact law with a fixed body, in contact iff the centre's
            // distance d to the wall is below r
            const double dw[2] = {(double)xl * a.qxd, (double)(0x100000000ull - (unsigned long long)xl) * a.qxd};
            const double sgn[2] = {-1.0, 1.0};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double d = dw[q];
                if (!(d < rld)) continue;
                const double cc = 2.0 * sqrt(fmax(rld * rld - d * d, 0.0));
                const double Fn = cc * a.Ed * (d - rld);
                const double vt = -(vld * sgn[q]) - wld * rld;     // t = (0, sgn): -v.t - w r
                const double capf = a.mud * fabs(Fn);
                const double Ft = fmin(fmax(cc * a.Gd * vt, -capf), capf);
                Fx += Fn * sgn[q];
                Fy += Ft * sgn[q];
                T += rld * Ft;
                ncontact += 1ull;
            }
        }
        // semi-implicit Euler (positions with the new velocities) unless forward Euler
        const double inv_m = 1.0 / md;
        const double dt = a.dtd;
        const double und = uld + dt * (Fx * inv_m);
        const double vnd = vld + dt * (Fy * inv_m);
        const double wnd = wld + dt * (T * inv_m / (rld * rld));
        const bool fe = (a.flags & SP_FORWARD_EULER) != 0;
        const double ux = fe ? uld : und, vx = fe ? vld : vnd, wx = fe ? wld : wnd;
        const int sx = __double2int_rn(dt * ux * a.inv_qxd);
        const int sy = __double2int_rn(dt * vx * a.inv_qyd);
        const float un = (float)und, vn = (float)vnd, wn = (float)wnd;
        if (wall) {
            const long long xn = (long long)xl + sx;
            if (xn < 0 || xn >= 0x100000000ll) atomicOr(a.err, kErrWall);
        }
        a.xo[k] = xl + (uint32_t)sx;
        a.yo[k] = yl + (uint32_t)sy;
        a.uo[k] = un;
        a.vo[k] = vn;
        a.wo[k] = wn;
        a.tho[k] = (float)((double)a.th[k] + dt * wx);
        a.ro[k] = rl;
        a.ho[k] = a.h[k];
        a.ido[k] = idl;
        if (!(isfinite(un) && isfinite(vn) && isfinite(wn))) atomicOr(a.err, kErrNaN);
    }
    const unsigned long long cs = wave_sum_u64(ncontact);
    if ((threadIdx.x & 63) == 0 && cs) atomicAdd(a.contacts, cs);
}

// Coarse cell of every floe (read-out).
__global__ __launch_bounds__(256) void ckey_kernel(const uint32_t* xi, const uint32_t* yi, int n, int nxc, int nyc,
                                                   uint32_t* keys, int32_t* vals)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    keys[k] = gbin_axis(yi[k], nyc) * (uint32_t)nxc + gbin_axis(xi[k], nxc);
    vals[k] = k;
}

// The 11 statistics of every coarse cell, one wavefront per cell over its
// floes in sorted order (fixed summation order).
__global__ __launch_bounds__(64) void cmom_kernel(GArgs a, const int32_t* perm, const int32_t* cstart, int ncoarse,
                                                  double* out)
{
    const int c = blockIdx.x;
    if (c >= ncoarse) return;
    const int lane = threadIdx.x;
    double acc[SP_NMOM];
#pragma unroll
    for (int q = 0; q < SP_NMOM; ++q) acc[q] = 0.0;
    for (int i = cstart[c] + lane; i < cstart[c + 1]; i += 64) {
        const int k = perm[i];
        const uint32_t x = a.xi[k], y = a.yi[k];
        const double rl = a.r[k], ul = a.u[k], vl = a.v[k], wl = a.w[k];
        const double m = a.rho_ice_d * (double)a.h[k] * kPi * rl * rl;
        double fdx, fdy, tdr;
        gdrag(a, x, y, rl, ul, vl, wl, fdx, fdy, tdr);
        acc[M_N] += 1.0;
        acc[M_MASS] += m;
        acc[M_PX] += m * ul;
        acc[M_PY] += m * vl;
        acc[M_L] += m * rl * rl * wl;
        acc[M_UX] += ul;
        acc[M_UY] += vl;
        acc[M_SVX] += fdx;
        acc[M_SVY] += fdy;
        acc[M_SW] += tdr;
        acc[M_AICE] += kPi * rl * rl;
    }
#pragma unroll
    for (int q = 0; q < SP_NMOM; ++q) {
        double x = acc[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) out[(size_t)c * SP_NMOM + q] = x;
    }
}

// Scatter the state back into input order (read-out).
__global__ __launch_bounds__(256) void gscatter_kernel(const int32_t* id, int n, const uint32_t* xi, const uint32_t* yi,
                                                       const float* u, const float* v, const float* w, const float* th,
                                                       const float* r, uint32_t* xo, uint32_t* yo, float* uo,
                                                       float* vo, float* wo, float* tho, float* ro)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int p = id[k];
    xo[p] = xi[k];
    yo[p] = yi[k];
    uo[p] = u[k];
    vo[p] = v[k];
    wo[p] = w[k];
    tho[p] = th[k];
    ro[p] = r[k];
}

}  // namespace spdem

namespace {

sp_status gfail(sp_gdem* g, sp_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (g) g->err = buf;
    return st;
}

#define GD_TRY(g, expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return gfail((g), SP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));             \
        }                                                                                      \
    } while (0)

template <class T>
sp_status galloc(sp_gdem* g, T** p, size_t count)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc((void**)p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return gfail(g, SP_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
    }
    return SP_OK;
}

void gdem_free(sp_gdem* g)
{
    for (int b = 0; b < 2; ++b) {
        void* ps[] = {g->xi[b], g->yi[b], g->u[b], g->v[b], g->w[b], g->th[b], g->r[b], g->h[b], g->id[b],
                      g->keys[b], g->vals[b]};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        g->xi[b] = g->yi[b] = nullptr;
        g->u[b] = g->v[b] = g->w[b] = g->th[b] = g->r[b] = g->h[b] = nullptr;
        g->id[b] = nullptr;
        g->keys[b] = nullptr;
        g->vals[b] = nullptr;
    }
    void* ps[] = {g->sort_tmp, g->bstart, g->cstart, g->cmom, g->phase, g->err_d, g->contacts_d};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    g->sort_tmp = nullptr;
    g->bstart = g->cstart = nullptr;
    g->cmom = nullptr;
    g->phase = nullptr;
    g->err_d = nullptr;
    g->contacts_d = nullptr;
    g->sort_bytes = g->cstart_cap = g->cmom_cap = 0;
}

int key_bits(uint32_t nkeys)
{
    int b = 1;
    while (b < 32 && (1u << b) < nkeys) ++b;
    return b;
}

// Sort (key, slot) pairs of the n floes; the sorted slots in vals[1].
sp_status gsort(sp_gdem* g, int nkeys)
{
    size_t bytes = 0;
    GD_TRY(g, hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, g->keys[0], g->keys[1], g->vals[0], g->vals[1],
                                                  (int)g->n, 0, key_bits((uint32_t)nkeys), g->stream));
    if (bytes > g->sort_bytes) {
        if (g->sort_tmp) (void)hipFree(g->sort_tmp);
        g->sort_tmp = nullptr;
        if (hipMalloc(&g->sort_tmp, bytes) != hipSuccess) {
            (void)hipGetLastError();
            g->sort_bytes = 0;
            return gfail(g, SP_ENOMEM, "sort workspace of %zu bytes", bytes);
        }
        g->sort_bytes = bytes;
    }
    GD_TRY(g, hipcub::DeviceRadixSort::SortPairs(g->sort_tmp, bytes, g->keys[0], g->keys[1], g->vals[0], g->vals[1],
                                                  (int)g->n, 0, key_bits((uint32_t)nkeys), g->stream));
    return SP_OK;
}

GArgs gargs(const sp_gdem* g, double dt, int from, int to)
{
    GArgs a;
    memset(&a, 0, sizeof a);
    a.xi = g->xi[from];
    a.yi = g->yi[from];
    a.u = g->u[from];
    a.v = g->v[from];
    a.w = g->w[from];
    a.th = g->th[from];
    a.r = g->r[from];
    a.h = g->h[from];
    a.id = g->id[from];
    a.xo = g->xi[to];
    a.yo = g->yi[to];
    a.uo = g->u[to];
    a.vo = g->v[to];
    a.wo = g->w[to];
    a.tho = g->th[to];
    a.ro = g->r[to];
    a.ho = g->h[to];
    a.ido = g->id[to];
    a.bstart = g->bstart;
    a.phase = g->phase;
    a.n = (int)g->n;
    a.nbx = g->nbx;
    a.nby = g->nby;
    a.nmodes = g->nmodes;
    a.flags = g->p.flags;
    a.qxd = g->p.lx / 4294967296.0;
    a.qyd = g->p.ly / 4294967296.0;
    a.qx = (float)a.qxd;
    a.qy = (float)a.qyd;
    a.inv_qxd = 1.0 / a.qxd;
    a.inv_qyd = 1.0 / a.qyd;
    a.dtd = dt;
    a.Ed = g->p.E;
    a.Gd = g->p.G;
    a.mud = g->p.mu;
    a.cdrho = g->p.cd * g->p.rho_ocean;
    a.rho_ice_d = g->p.rho_ice;
    a.u0 = g->u0;
    a.v0 = g->v0;
    a.lxd = g->p.lx;
    const double bx = g->p.lx / g->nbx, by = g->p.ly / g->nby;
    float reach = 0.0f;
    for (int m = 0; m < g->nmodes; ++m) {
        a.modes.kxL[m] = (float)(g->kx[m] * bx);
        a.modes.kyL[m] = (float)(g->ky[m] * by);
        a.modes.au[m] = g->au[m];
        a.modes.av[m] = g->av[m];
        a.modes.cz[m] = g->av[m] * g->kx[m] - g->au[m] * g->ky[m];
        reach = std::max(reach, 0.5f * (fabsf(a.modes.kxL[m]) + fabsf(a.modes.kyL[m])));
    }
    a.modes.direct = reach <= 1.6f ? 1 : 0;
    a.err = g->err_d;
    a.contacts = g->contacts_d;
    return a;
}

sp_status gupload_phase(sp_gdem* g)
{
    if (!g->phase_dirty || !g->have_floes) return SP_OK;
    const int nm = std::max(1, g->nmodes);
    const size_t nb = (size_t)g->nbx * g->nby;
    std::vector<double2> tab(nb * nm, make_double2(0.0, 1.0));
    for (size_t b = 0; b < nb; ++b) {
        const double Xc = ((double)(b % g->nbx) + 0.5) * g->p.lx / g->nbx;
        const double Yc = ((double)(b / g->nbx) + 0.5) * g->p.ly / g->nby;
        for (int m = 0; m < g->nmodes; ++m) {
            const double t = g->kx[m] * Xc + g->ky[m] * Yc + g->ph[m];
            tab[b * nm + m] = make_double2(sin(t), cos(t));
        }
    }
    SP_TRY(galloc(g, &g->phase, tab.size()));
    GD_TRY(g, hipMemcpyAsync(g->phase, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    g->phase_dirty = false;
    return SP_OK;
}

sp_status gcheck(sp_gdem* g)
{
    uint32_t e = 0;
    GD_TRY(g, hipMemcpyAsync(&e, g->err_d, 4, hipMemcpyDeviceToHost, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    if (e & kErrOverlap) return gfail(g, SP_EOVERLAP, "two floe centres coincide");
    if (e & kErrNaN) return gfail(g, SP_ENAN, "non-finite floe state");
    if (e & kErrWall) return gfail(g, SP_EWALL, "a floe crossed a wall");
    return SP_OK;
}

}  // namespace

extern "C" {

sp_status sp_gdem_create(const sp_gdem_params* p, void* stream, sp_gdem** out)
{
    if (!p || !out) return SP_EINVAL;
    *out = nullptr;
    if (!(p->lx > 0) || !(p->ly > 0) || !(p->rho_ice > 0) || !(p->rho_ocean > 0) || !(p->cd >= 0) ||
        !(p->E >= 0) || !(p->G >= 0) || !(p->mu >= 0))
        return SP_EINVAL;
    sp_gdem* g = new sp_gdem();
    g->p = *p;
    if (stream) {
        g->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&g->stream) != hipSuccess) {
            delete g;
            return SP_EDEVICE;
        }
        g->own_stream = true;
    }
    sp_status st = galloc(g, &g->err_d, 1);
    if (!st) st = galloc(g, &g->contacts_d, 1);
    if (!st && (hipMemsetAsync(g->err_d, 0, 4, g->stream) != hipSuccess ||
                hipMemsetAsync(g->contacts_d, 0, 8, g->stream) != hipSuccess))
        st = SP_EDEVICE;
    if (st) {
        gdem_free(g);
        if (g->own_stream) (void)hipStreamDestroy(g->stream);
        delete g;
        return st;
    }
    *out = g;
    return SP_OK;
}

void sp_gdem_destroy(sp_gdem* g)
{
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    gdem_free(g);
    if (g->own_stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

const char* sp_gdem_last_error(const sp_gdem* g) { return g ? g->err.c_str() : "null context"; }

sp_status sp_gdem_set_ocean(sp_gdem* g, double u0, double v0, int32_t nmodes, const double* kx, const double* ky,
                            const double* au, const double* av, const double* phase)
{
    if (!g) return SP_EINVAL;
    if (nmodes < 0 || nmodes > SP_MAX_MODES) return gfail(g, SP_EINVAL, "nmodes %d out of range", nmodes);
    if (nmodes > 0 && (!kx || !ky || !au || !av || !phase)) return gfail(g, SP_EINVAL, "null mode array");
    g->u0 = u0;
    g->v0 = v0;
    g->nmodes = nmodes;
    for (int m = 0; m < nmodes; ++m) {
        g->kx[m] = kx[m];
        g->ky[m] = ky[m];
        g->au[m] = au[m];
        g->av[m] = av[m];
        g->ph[m] = phase[m];
    }
    g->phase_dirty = true;
    return SP_OK;
}

sp_status sp_gdem_set_floes(sp_gdem* g, int64_t n, const uint32_t* xi, const uint32_t* yi, const float* u,
                            const float* v, const float* omega, const float* theta, const float* r, const float* h)
{
    if (!g) return SP_EINVAL;
    if (n < 1 || n > INT32_MAX / 2) return gfail(g, SP_EINVAL, "floe count %lld out of range", (long long)n);
    if (!xi || !yi || !u || !v || !r || !h) return gfail(g, SP_EINVAL, "null floe array");
    GD_TRY(g, hipStreamSynchronize(g->stream));
    g->have_floes = false;
    float rmax = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        if (!(r[i] > 0.0f) || !std::isfinite(r[i])) return gfail(g, SP_EINVAL, "radius %lld not positive", (long long)i);
        if (!(h[i] > 0.0f) || !std::isfinite(h[i])) return gfail(g, SP_EINVAL, "thickness %lld not positive", (long long)i);
        rmax = std::max(rmax, r[i]);
    }
    const double lmin = std::min(g->p.lx, g->p.ly);
    if (!((double)rmax < 0.25 * lmin))
        return gfail(g, SP_EINVAL, "r_max %g must stay below a quarter of the domain (%g)", rmax, 0.25 * lmin);
    // sub-bins of side >= 2 r_max: contacts only join neighbouring sub-bins;
    // fewer than 3 along an axis: one sub-bin spans it
    int bx = (int)std::min(4096.0, floor(g->p.lx / (2.0 * (double)rmax)));
    int by = (int)std::min(4096.0, floor(g->p.ly / (2.0 * (double)rmax)));
    if (bx < 3) bx = 1;
    if (by < 3) by = 1;
    g->nbx = bx;
    g->nby = by;
    g->rmax = rmax;
    g->n = n;
    const size_t N = (size_t)n;
    for (int b = 0; b < 2; ++b) {
        SP_TRY(galloc(g, &g->xi[b], N));
        SP_TRY(galloc(g, &g->yi[b], N));
        SP_TRY(galloc(g, &g->u[b], N));
        SP_TRY(galloc(g, &g->v[b], N));
        SP_TRY(galloc(g, &g->w[b], N));
        SP_TRY(galloc(g, &g->th[b], N));
        SP_TRY(galloc(g, &g->r[b], N));
        SP_TRY(galloc(g, &g->h[b], N));
        SP_TRY(galloc(g, &g->id[b], N));
        SP_TRY(galloc(g, &g->keys[b], N));
        SP_TRY(galloc(g, &g->vals[b], N));
    }
    SP_TRY(galloc(g, &g->bstart, (size_t)bx * by + 1));
    g->cur = 0;
    std::vector<int32_t> ids(N);
    for (size_t i = 0; i < N; ++i) ids[i] = (int32_t)i;
    const void* src[8] = {xi, yi, u, v, omega, theta, r, h};
    void* dst[8] = {g->xi[0], g->yi[0], g->u[0], g->v[0], g->w[0], g->th[0], g->r[0], g->h[0]};
    for (int k = 0; k < 8; ++k) {
        if (src[k]) {
            GD_TRY(g, hipMemcpyAsync(dst[k], src[k], N * 4, hipMemcpyHostToDevice, g->stream));
        } else {
            GD_TRY(g, hipMemsetAsync(dst[k], 0, N * 4, g->stream));
        }
    }
    GD_TRY(g, hipMemcpyAsync(g->id[0], ids.data(), N * 4, hipMemcpyHostToDevice, g->stream));
    GD_TRY(g, hipMemsetAsync(g->err_d, 0, 4, g->stream));
    GD_TRY(g, hipMemsetAsync(g->contacts_d, 0, 8, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));   // ids is a host temporary
    g->steps = 0;
    g->phase_dirty = true;
    g->have_floes = true;
    return SP_OK;
}

sp_status sp_gdem_step(sp_gdem* g, double dt, int64_t nsteps)
{
    if (!g) return SP_EINVAL;
    if (!g->have_floes) return gfail(g, SP_ESTATE, "sp_gdem_step before sp_gdem_set_floes");
    if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0) return gfail(g, SP_EINVAL, "dt must be positive");
    SP_TRY(gupload_phase(g));
    const int n = (int)g->n;
    const int nb = g->nbx * g->nby;
    const dim3 grid((n + 255) / 256), blk(256);
    for (int64_t it = 0; it < nsteps; ++it) {
        const int c = g->cur, o = c ^ 1;
        hipLaunchKernelGGL(gkey_kernel, grid, blk, 0, g->stream, g->xi[c], g->yi[c], n, g->nbx, g->nby, g->keys[0],
                           g->vals[0]);
        GD_TRY(g, hipGetLastError());
        SP_TRY(gsort(g, nb));
        hipLaunchKernelGGL(ggather_kernel, grid, blk, 0, g->stream, g->vals[1], n, g->xi[c], g->yi[c], g->u[c],
                           g->v[c], g->w[c], g->th[c], g->r[c], g->h[c], g->id[c], g->xi[o], g->yi[o], g->u[o],
                           g->v[o], g->w[o], g->th[o], g->r[o], g->h[o], g->id[o]);
        GD_TRY(g, hipGetLastError());
        hipLaunchKernelGGL(gstart_kernel, dim3((nb + 1 + 255) / 256), blk, 0, g->stream, g->keys[1], n, nb,
                           g->bstart);
        GD_TRY(g, hipGetLastError());
        hipLaunchKernelGGL(gstep_kernel, grid, blk, 0, g->stream, gargs(g, dt, o, c));
        GD_TRY(g, hipGetLastError());
        g->steps++;
    }
    return SP_OK;
}

sp_status sp_gdem_read_floes(sp_gdem* g, uint32_t* xi, uint32_t* yi, float* u, float* v, float* omega,
                             float* theta, float* r)
{
    if (!g) return SP_EINVAL;
    if (!g->have_floes) return gfail(g, SP_ESTATE, "no floes");
    const int n = (int)g->n, c = g->cur, o = c ^ 1;
    hipLaunchKernelGGL(gscatter_kernel, dim3((n + 255) / 256), dim3(256), 0, g->stream, g->id[c], n, g->xi[c],
                       g->yi[c], g->u[c], g->v[c], g->w[c], g->th[c], g->r[c], g->xi[o], g->yi[o], g->u[o], g->v[o],
                       g->w[o], g->th[o], g->r[o]);
    GD_TRY(g, hipGetLastError());
    void* dst[7] = {xi, yi, u, v, omega, theta, r};
    const void* src[7] = {g->xi[o], g->yi[o], g->u[o], g->v[o], g->w[o], g->th[o], g->r[o]};
    for (int k = 0; k < 7; ++k)
        if (dst[k]) GD_TRY(g, hipMemcpyAsync(dst[k], src[k], (size_t)n * 4, hipMemcpyDeviceToHost, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    return gcheck(g);
}

sp_status sp_gdem_coarse_moments(sp_gdem* g, int32_t nxc, int32_t nyc, double* out)
{
    if (!g) return SP_EINVAL;
    if (!g->have_floes) return gfail(g, SP_ESTATE, "no floes");
    if (nxc < 1 || nyc < 1 || (int64_t)nxc * nyc > (1 << 26) || !out)
        return gfail(g, SP_EINVAL, "coarse grid %d x %d out of range or null output", nxc, nyc);
    SP_TRY(gupload_phase(g));
    const int n = (int)g->n, c = g->cur;
    const int ncoarse = nxc * nyc;
    if ((size_t)ncoarse + 1 > g->cstart_cap) {
        SP_TRY(galloc(g, &g->cstart, (size_t)ncoarse + 1));
        g->cstart_cap = (size_t)ncoarse + 1;
    }
    if ((size_t)ncoarse * SP_NMOM > g->cmom_cap) {
        SP_TRY(galloc(g, &g->cmom, (size_t)ncoarse * SP_NMOM));
        g->cmom_cap = (size_t)ncoarse * SP_NMOM;
    }
    hipLaunchKernelGGL(ckey_kernel, dim3((n + 255) / 256), dim3(256), 0, g->stream, g->xi[c], g->yi[c], n, nxc, nyc,
                       g->keys[0], g->vals[0]);
    GD_TRY(g, hipGetLastError());
    SP_TRY(gsort(g, ncoarse));
    hipLaunchKernelGGL(gstart_kernel, dim3((ncoarse + 1 + 255) / 256), dim3(256), 0, g->stream, g->keys[1], n, ncoarse,
                       g->cstart);
    GD_TRY(g, hipGetLastError());
    hipLaunchKernelGGL(cmom_kernel, dim3(ncoarse), dim3(64), 0, g->stream, gargs(g, 0.0, c, c ^ 1), g->vals[1],
                       g->cstart, ncoarse, g->cmom);
    GD_TRY(g, hipGetLastError());
    GD_TRY(g, hipMemcpyAsync(out, g->cmom, (size_t)ncoarse * SP_NMOM * 8, hipMemcpyDeviceToHost, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    return gcheck(g);
}

sp_status sp_gdem_get_stats(sp_gdem* g, int64_t* contacts, int64_t* steps, int32_t* bins_x, int32_t* bins_y)
{
    if (!g) return SP_EINVAL;
    unsigned long long cnt = 0;
    GD_TRY(g, hipMemcpyAsync(&cnt, g->contacts_d, 8, hipMemcpyDeviceToHost, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    if (contacts) *contacts = (int64_t)cnt;
    if (steps) *steps = g->steps;
    if (bins_x) *bins_x = g->nbx;
    if (bins_y) *bins_y = g->nby;
    return gcheck(g);
}

}  // extern "C"
