// The global DEM of the paper's error study (Sec. 4): one DEM over the whole
// periodic domain, floes free to cross coarse cells, every pair a potential
// contact.  It is the reference ("truth") the superparameterised model is
// compared with; its coarse-grid statistics are read for that comparison.
// Included at the end of spdem.hip.
//
// Per fine step, two launches.  The re-binning (gpull_kernel) is a stable
// counting sort of the floes by sub-bin (side >= 2 r_max, so contacts only
// join neighbouring sub-bins): the counts per sub-bin and per sub-bin row come
// from the previous step's atomics, every row's workgroup takes its row start
// from the row counts and its sub-bin starts by a scan, and every sub-bin
// gathers its floes in their current order from the 3 x 3 sub-bins around it
// (the state is grouped by the previous sub-bins and a floe moves far less
// than a sub-bin per step; a sub-bin that finds fewer floes than its count
// scans all floes instead).  The result is the order a stable sort by sub-bin
// gives.  Then one thread per floe (gstep_kernel) sweeps the 3 x 3
// neighbouring sub-bins, decides contacts exactly as the cell kernel does
// (FP32 screen, FP64 in the guard band), sums drag and contact forces in FP64,
// writes the updated floe in the same order, and counts the sub-bin of its
// new position for the next re-binning.
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
    // re-binning: the sub-bin of every floe's position (order of buffer cur),
    // floes per sub-bin and per sub-bin row of those, sub-bin starts
    int32_t* key = nullptr;            // [n]
    int32_t* bcount[2] = {nullptr, nullptr};   // [nb], alternating per step
    int32_t* rcount[2] = {nullptr, nullptr};   // [nby], alternating per step
    int32_t* starts[2] = {nullptr, nullptr};   // [nb + 1]
    int sb = 0;                        // starts[sb] groups buffer cur
    int rb = 0;                        // bcount[rb] and rcount[rb] count sub-bins and rows of key
    unsigned long long* fallbacks_d = nullptr;  // sub-bins (and coarse cells) gathered by a full scan
    // coarse read-out: coarse cell of every floe, counts, starts, floes in cell order
    int32_t* ckey = nullptr;           // [n]
    int32_t* perm = nullptr;           // [n]
    int32_t* ccount = nullptr;         // [ncoarse]
    int32_t* crow = nullptr;           // [nyc]
    size_t ccount_cap = 0, crow_cap = 0;
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
    // the sub-bin of every updated position, counted per sub-bin and per row
    int32_t* key_out;
    int32_t* count;
    int32_t* rows;
};

constexpr uint32_t kErrRebin = 32u;    // a re-binning gathered another number of floes than it counted

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

// The axis indices lo - 1 .. hi + 1 modulo n as at most two ascending,
// disjoint segments [a0, a1] and [b0, b1] (b0 > b1: none), the first below
// the second; all of 0 .. n - 1 when they cover the axis.
struct Segs {
    int a0, a1, b0, b1;
};

__device__ __forceinline__ Segs wrap_segments(int lo, int hi, int n)
{
    if (hi - lo + 3 >= n) return Segs{0, n - 1, 1, 0};
    const int s = lo - 1, e = hi + 1;
    if (s < 0) return Segs{0, e, s + n, n - 1};
    if (e >= n) return Segs{0, e - n, s, n - 1};
    return Segs{s, e, 1, 0};
}

// Every position p of the grouped order whose sub-bin lies in rows ry and
// columns rx (segments of wrap_segments), in ascending p: sub-bins are visited
// in ascending index (rows, then columns, ascending), and the grouping puts a
// lower sub-bin's floes first.
template <class F>
__device__ __forceinline__ void for_sources(const int32_t* ostart, int nbx, Segs ry, Segs rx, F f)
{
    const int ys[4] = {ry.a0, ry.a1, ry.b0, ry.b1};
    const int xs[4] = {rx.a0, rx.a1, rx.b0, rx.b1};
    for (int sy = 0; sy < 2; ++sy)
        for (int yy = ys[2 * sy]; yy <= ys[2 * sy + 1]; ++yy)
            for (int sx = 0; sx < 2; ++sx) {
                if (xs[2 * sx] > xs[2 * sx + 1]) continue;
                const int p1 = ostart[yy * nbx + xs[2 * sx + 1] + 1];
                for (int p = ostart[yy * nbx + xs[2 * sx]]; p < p1; ++p) f(p);
            }
}

// Exclusive prefix over a 256-thread workgroup (LDS s[256]); total of all in tot.
__device__ __forceinline__ int block_exclusive_scan(int v, int* s, int& tot)
{
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int x = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    const int incl = s[t];
    tot = s[255];
    __syncthreads();
    return incl - v;
}

// Sum over the rows before `row` of per-row counts (every thread gets it).
__device__ __forceinline__ int rows_before(const int32_t* rows, int row, int* s)
{
    int part = 0;
    for (int i = threadIdx.x; i < row; i += 256) part += rows[i];
    int tot;
    (void)block_exclusive_scan(part, s, tot);
    return tot;
}

// Sum over the wavefront (every lane gets it) and exclusive prefix over its lanes.
__device__ __forceinline__ int wave_sum_i32(int x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ int wave_exclusive_i32(int x)
{
    const int lane = threadIdx.x & 63;
    int incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    return incl - x;
}

struct GPull {
    // buffer cur, grouped by ostart -> buffer out, grouped by nstart
    const uint32_t* xi;
    const uint32_t* yi;
    const float *u, *v, *w, *th, *r, *h;
    const int32_t* id;
    uint32_t* xo;
    uint32_t* yo;
    float *uo, *vo, *wo, *tho, *ro, *ho;
    int32_t* ido;
    const int32_t* key;        // [n] sub-bin of every floe of buffer cur
    const int32_t* ostart;     // [nb + 1]
    int32_t* nstart;           // [nb + 1]
    const int32_t* count;      // [nb] floes per sub-bin of key
    int32_t* count_next;       // [nb] zeroed here for the next step's counts
    const int32_t* rows;       // [nby] floes per sub-bin row of key
    int32_t* rows_next;        // [nby] zeroed here
    int n, nbx, nby;
    uint32_t* err;
    unsigned long long* fallbacks;
};

// Re-binning: one wavefront per run of 64 sub-bins of a row, one lane per
// sub-bin.  A run starts after the floes of the rows before it and of its
// row's earlier sub-bins.
__global__ __launch_bounds__(256) void gpull_kernel(GPull g)
{
    const int lane = threadIdx.x & 63;
    const int wid = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int runs = (g.nbx + 63) >> 6;
    if (wid >= g.nby * runs) return;          // whole wavefronts
    const int by = wid / runs, c0 = (wid % runs) * 64;
    int part = 0;
    for (int i = lane; i < by; i += 64) part += g.rows[i];
    for (int i = lane; i < c0; i += 64) part += g.count[by * g.nbx + i];
    const int base = wave_sum_i32(part);
    const int bx = c0 + lane;
    const bool in = bx < g.nbx;
    const int b = by * g.nbx + bx;
    const int cnt = in ? g.count[b] : 0;
    const int q0 = base + wave_exclusive_i32(cnt);
    if (c0 == 0 && lane == 0) g.rows_next[by] = 0;
    if (wid == g.nby * runs - 1 && lane == 63) g.nstart[g.nbx * g.nby] = g.n;
    if (!in) return;
    g.count_next[b] = 0;
    g.nstart[b] = q0;
    int i = 0;
    auto take = [&](int p) {
        if (g.key[p] != b) return;
        if (i < cnt) {
            const int q = q0 + i;
            g.xo[q] = g.xi[p];
            g.yo[q] = g.yi[p];
            g.uo[q] = g.u[p];
            g.vo[q] = g.v[p];
            g.wo[q] = g.w[p];
            g.tho[q] = g.th[p];
            g.ro[q] = g.r[p];
            g.ho[q] = g.h[p];
            g.ido[q] = g.id[p];
        }
        ++i;
    };
    // the (at most 3 x 2) position ranges of the neighbouring sub-bins in
    // ascending order, their bounds read together, then 4 keys at a time
    {
        const Segs ry = wrap_segments(by, by, g.nby), rx = wrap_segments(bx, bx, g.nbx);
        int row[3], nrow = 0;
        for (int y = ry.a0; y <= ry.a1 && nrow < 3; ++y) row[nrow++] = y;
        for (int y = ry.b0; y <= ry.b1 && nrow < 3; ++y) row[nrow++] = y;
        const bool two = rx.b0 <= rx.b1;
        int lo[6], hi[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int rr = k >> 1, sg = k & 1;
            const bool use = rr < nrow && (sg == 0 || two);
            const int b0 = use ? row[rr] * g.nbx + (sg ? rx.b0 : rx.a0) : 0;
            const int b1 = use ? row[rr] * g.nbx + (sg ? rx.b1 : rx.a1) + 1 : 0;
            lo[k] = use ? g.ostart[b0] : 0;
            hi[k] = use ? g.ostart[b1] : 0;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k)
            for (int p = lo[k]; p < hi[k]; p += 4) {
                int kk[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) kk[e] = p + e < hi[k] ? g.key[p + e] : -1;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (kk[e] == b) take(p + e);
            }
    }
    if (i != cnt) {   // a floe came from further away: every floe, in order
        atomicAdd(g.fallbacks, 1ull);
        i = 0;
        for (int p = 0; p < g.n; ++p) take(p);
        if (i != cnt) atomicOr(g.err, kErrRebin);
    }
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
    int row = -1;   // sub-bin row of the updated position
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
        const uint32_t xn = xl + (uint32_t)sx, yn = yl + (uint32_t)sy;
        a.xo[k] = xn;
        a.yo[k] = yn;
        {
            row = (int)gbin_axis(yn, a.nby);
            const int b = row * a.nbx + (int)gbin_axis(xn, a.nbx);
            a.key_out[k] = b;
            atomicAdd(&a.count[b], 1);
        }
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
    // floes per row: one atomic per wavefront when its floes share a row (the
    // order is by sub-bin, so they mostly do)
    const int row0 = __shfl(row, 0);
    const unsigned long long valid = __ballot(row >= 0), same = __ballot(row >= 0 && row == row0);
    if (same == valid) {
        if ((threadIdx.x & 63) == 0 && valid) atomicAdd(&a.rows[row0], (int)__popcll(valid));
    } else if (row >= 0) {
        atomicAdd(&a.rows[row], 1);
    }
}

// Coarse cell of every floe of buffer cur (read-out), counted per cell and per row.
__global__ __launch_bounds__(256) void ckey_kernel(const uint32_t* xi, const uint32_t* yi, int n, int nxc, int nyc,
                                                   int32_t* ckey, int32_t* ccount, int32_t* crow)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int cy = (int)gbin_axis(yi[k], nyc);
    const int c = cy * nxc + (int)gbin_axis(xi[k], nxc);
    ckey[k] = c;
    atomicAdd(&ccount[c], 1);
    atomicAdd(&crow[cy], 1);
}

// The floes of every coarse cell in the current order (perm, from cstart): a
// stable counting sort as the re-binning, one workgroup per coarse row, the
// row's cells scanned for their starts, then one wavefront per cell gathering
// in order (ballot and prefix count) from the sub-bins its cell overlaps, one
// more on every side (the grouping is that of the last re-binning, the
// positions a step later); a cell that finds fewer floes than its count scans
// all floes instead.
__global__ __launch_bounds__(256) void cpull_kernel(const int32_t* ckey, const int32_t* ccount, const int32_t* crow,
                                                    const int32_t* ostart, int n, int nbx, int nby, int nxc,
                                                    int nyc, int32_t* cstart, int32_t* perm, uint32_t* err,
                                                    unsigned long long* fallbacks)
{
    __shared__ int s[256];
    const int cy = blockIdx.x;
    const int row0 = rows_before(crow, cy, s);
    if (threadIdx.x == 0 && cy == nyc - 1) cstart[nxc * nyc] = n;
    int carry = 0;
    for (int c0 = 0; c0 < nxc; c0 += 256) {
        const int cx = c0 + (int)threadIdx.x;
        const int cnt = cx < nxc ? ccount[cy * nxc + cx] : 0;
        int tot;
        const int q0 = row0 + carry + block_exclusive_scan(cnt, s, tot);
        carry += tot;
        if (cx < nxc) cstart[cy * nxc + cx] = q0;
    }
    __syncthreads();
    // sub-bin rows and columns a coarse cell overlaps
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ylo = (int)(((long long)cy * nby) / nyc), yhi = (int)(((long long)(cy + 1) * nby - 1) / nyc);
    for (int cx = wave; cx < nxc; cx += 4) {
        const int c = cy * nxc + cx;
        const int q0 = cstart[c], cnt = ccount[c];
        const int xlo = (int)(((long long)cx * nbx) / nxc), xhi = (int)(((long long)(cx + 1) * nbx - 1) / nxc);
        int i = 0;   // floes of c gathered so far (the same in every lane)
        auto chunk = [&](int p0, int p1) {   // positions [p0, p1), 64 at a time, in order
            for (int b = p0; b < p1; b += 64) {
                const int p = b + lane;
                const bool hit = p < p1 && ckey[p] == c;
                const unsigned long long m = __ballot(hit);
                const int before = __popcll(m & ((1ull << lane) - 1ull));
                if (hit && i + before < cnt) perm[q0 + i + before] = p;
                i += __popcll(m);
            }
        };
        const Segs ry = wrap_segments(ylo, yhi, nby), rx = wrap_segments(xlo, xhi, nbx);
        const int ys[4] = {ry.a0, ry.a1, ry.b0, ry.b1};
        const int xs[4] = {rx.a0, rx.a1, rx.b0, rx.b1};
        for (int sy = 0; sy < 2; ++sy)
            for (int yy = ys[2 * sy]; yy <= ys[2 * sy + 1]; ++yy)
                for (int sx = 0; sx < 2; ++sx)
                    if (xs[2 * sx] <= xs[2 * sx + 1])
                        chunk(ostart[yy * nbx + xs[2 * sx]], ostart[yy * nbx + xs[2 * sx + 1] + 1]);
        if (i != cnt) {
            if (lane == 0) atomicAdd(fallbacks, 1ull);
            i = 0;
            chunk(0, n);
            if (i != cnt && lane == 0) atomicOr(err, kErrRebin);
        }
    }
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
                      g->rcount[b], g->starts[b], g->bcount[b]};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        g->xi[b] = g->yi[b] = nullptr;
        g->u[b] = g->v[b] = g->w[b] = g->th[b] = g->r[b] = g->h[b] = nullptr;
        g->id[b] = nullptr;
        g->rcount[b] = g->starts[b] = g->bcount[b] = nullptr;
    }
    void* ps[] = {g->key, g->ckey, g->perm, g->ccount, g->crow, g->cstart, g->cmom, g->phase, g->err_d,
                  g->contacts_d, g->fallbacks_d};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    g->key = g->ckey = g->perm = g->ccount = g->crow = g->cstart = nullptr;
    g->cmom = nullptr;
    g->phase = nullptr;
    g->err_d = nullptr;
    g->contacts_d = nullptr;
    g->fallbacks_d = nullptr;
    g->ccount_cap = g->crow_cap = g->cstart_cap = g->cmom_cap = 0;
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
    a.bstart = g->starts[g->sb ^ 1];   // the starts the re-binning before the step makes
    a.key_out = g->key;
    a.count = g->bcount[g->rb ^ 1];
    a.rows = g->rcount[g->rb ^ 1];
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
    if (e & kErrRebin) return gfail(g, SP_EDEVICE, "re-binning gathered another number of floes than it counted");
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
    const size_t nb = (size_t)bx * by;
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
        SP_TRY(galloc(g, &g->rcount[b], (size_t)by));
        SP_TRY(galloc(g, &g->starts[b], nb + 1));
        SP_TRY(galloc(g, &g->bcount[b], nb));
    }
    SP_TRY(galloc(g, &g->key, N));
    SP_TRY(galloc(g, &g->ckey, N));
    SP_TRY(galloc(g, &g->perm, N));
    if (!g->fallbacks_d) SP_TRY(galloc(g, &g->fallbacks_d, 1));
    // the first grouping: a stable counting sort by sub-bin on the host, the
    // counts and starts the first re-binning reads
    std::vector<int32_t> key(N), count(nb, 0), rows((size_t)by, 0), start(nb + 1, 0), order(N);
    for (size_t i = 0; i < N; ++i) {
        const uint32_t ky = (uint32_t)(((uint64_t)yi[i] * (uint64_t)by) >> 32);
        const uint32_t kx = (uint32_t)(((uint64_t)xi[i] * (uint64_t)bx) >> 32);
        key[i] = (int32_t)(ky * (uint32_t)bx + kx);
        ++count[key[i]];
        ++rows[ky];
    }
    for (size_t b = 0; b < nb; ++b) start[b + 1] = start[b] + count[b];
    {
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (size_t i = 0; i < N; ++i) order[fill[key[i]]++] = (int32_t)i;
    }
    std::vector<int32_t> skey(N);
    for (size_t q = 0; q < N; ++q) skey[q] = key[order[q]];
    std::vector<uint32_t> bits(N);
    const void* src[8] = {xi, yi, u, v, omega, theta, r, h};
    void* dst[8] = {g->xi[0], g->yi[0], g->u[0], g->v[0], g->w[0], g->th[0], g->r[0], g->h[0]};
    for (int k = 0; k < 8; ++k) {
        const uint32_t* sk = static_cast<const uint32_t*>(src[k]);
        for (size_t q = 0; q < N; ++q) bits[q] = sk ? sk[order[q]] : 0u;
        GD_TRY(g, hipMemcpy(dst[k], bits.data(), N * 4, hipMemcpyHostToDevice));
    }
    GD_TRY(g, hipMemcpy(g->id[0], order.data(), N * 4, hipMemcpyHostToDevice));
    GD_TRY(g, hipMemcpy(g->key, skey.data(), N * 4, hipMemcpyHostToDevice));
    GD_TRY(g, hipMemcpy(g->bcount[0], count.data(), nb * 4, hipMemcpyHostToDevice));
    GD_TRY(g, hipMemsetAsync(g->bcount[1], 0, nb * 4, g->stream));
    GD_TRY(g, hipMemcpy(g->rcount[0], rows.data(), (size_t)by * 4, hipMemcpyHostToDevice));
    GD_TRY(g, hipMemcpy(g->starts[0], start.data(), (nb + 1) * 4, hipMemcpyHostToDevice));
    GD_TRY(g, hipMemsetAsync(g->rcount[1], 0, (size_t)by * 4, g->stream));
    GD_TRY(g, hipMemsetAsync(g->err_d, 0, 4, g->stream));
    GD_TRY(g, hipMemsetAsync(g->contacts_d, 0, 8, g->stream));
    GD_TRY(g, hipMemsetAsync(g->fallbacks_d, 0, 8, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    g->cur = 0;
    g->sb = 0;
    g->rb = 0;
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
    const dim3 grid((n + 255) / 256), blk(256);
    for (int64_t it = 0; it < nsteps; ++it) {
        const int c = g->cur, o = c ^ 1;
        GPull pl;
        pl.xi = g->xi[c];
        pl.yi = g->yi[c];
        pl.u = g->u[c];
        pl.v = g->v[c];
        pl.w = g->w[c];
        pl.th = g->th[c];
        pl.r = g->r[c];
        pl.h = g->h[c];
        pl.id = g->id[c];
        pl.xo = g->xi[o];
        pl.yo = g->yi[o];
        pl.uo = g->u[o];
        pl.vo = g->v[o];
        pl.wo = g->w[o];
        pl.tho = g->th[o];
        pl.ro = g->r[o];
        pl.ho = g->h[o];
        pl.ido = g->id[o];
        pl.key = g->key;
        pl.ostart = g->starts[g->sb];
        pl.nstart = g->starts[g->sb ^ 1];
        pl.count = g->bcount[g->rb];
        pl.count_next = g->bcount[g->rb ^ 1];
        pl.rows = g->rcount[g->rb];
        pl.rows_next = g->rcount[g->rb ^ 1];
        pl.n = n;
        pl.nbx = g->nbx;
        pl.nby = g->nby;
        pl.err = g->err_d;
        pl.fallbacks = g->fallbacks_d;
        const int64_t waves = (int64_t)g->nby * ((g->nbx + 63) / 64);
        hipLaunchKernelGGL(gpull_kernel, dim3((unsigned)((waves + 3) / 4)), blk, 0, g->stream, pl);
        GD_TRY(g, hipGetLastError());
        hipLaunchKernelGGL(gstep_kernel, grid, blk, 0, g->stream, gargs(g, dt, o, c));
        GD_TRY(g, hipGetLastError());
        g->sb ^= 1;
        g->rb ^= 1;
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
    if ((size_t)ncoarse > g->ccount_cap) {
        SP_TRY(galloc(g, &g->ccount, (size_t)ncoarse));
        g->ccount_cap = (size_t)ncoarse;
    }
    if ((size_t)nyc > g->crow_cap) {
        SP_TRY(galloc(g, &g->crow, (size_t)nyc));
        g->crow_cap = (size_t)nyc;
    }
    GD_TRY(g, hipMemsetAsync(g->ccount, 0, (size_t)ncoarse * 4, g->stream));
    GD_TRY(g, hipMemsetAsync(g->crow, 0, (size_t)nyc * 4, g->stream));
    hipLaunchKernelGGL(ckey_kernel, dim3((n + 255) / 256), dim3(256), 0, g->stream, g->xi[c], g->yi[c], n, nxc, nyc,
                       g->ckey, g->ccount, g->crow);
    GD_TRY(g, hipGetLastError());
    hipLaunchKernelGGL(cpull_kernel, dim3(nyc), dim3(256), 0, g->stream, g->ckey, g->ccount, g->crow,
                       g->starts[g->sb], n, g->nbx, g->nby, nxc, nyc, g->cstart, g->perm, g->err_d,
                       g->fallbacks_d);
    GD_TRY(g, hipGetLastError());
    hipLaunchKernelGGL(cmom_kernel, dim3(ncoarse), dim3(64), 0, g->stream, gargs(g, 0.0, c, c ^ 1), g->perm,
                       g->cstart, ncoarse, g->cmom);
    GD_TRY(g, hipGetLastError());
    GD_TRY(g, hipMemcpyAsync(out, g->cmom, (size_t)ncoarse * SP_NMOM * 8, hipMemcpyDeviceToHost, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    return gcheck(g);
}

sp_status sp_gdem_read_order(sp_gdem* g, int32_t* ids, int32_t* starts, int64_t* fallbacks)
{
    if (!g) return SP_EINVAL;
    if (!g->have_floes) return gfail(g, SP_ESTATE, "no floes");
    const size_t N = (size_t)g->n, nb = (size_t)g->nbx * g->nby;
    if (ids) GD_TRY(g, hipMemcpyAsync(ids, g->id[g->cur], N * 4, hipMemcpyDeviceToHost, g->stream));
    if (starts) GD_TRY(g, hipMemcpyAsync(starts, g->starts[g->sb], (nb + 1) * 4, hipMemcpyDeviceToHost, g->stream));
    unsigned long long fb = 0;
    GD_TRY(g, hipMemcpyAsync(&fb, g->fallbacks_d, 8, hipMemcpyDeviceToHost, g->stream));
    GD_TRY(g, hipStreamSynchronize(g->stream));
    if (fallbacks) *fallbacks = (int64_t)fb;
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
