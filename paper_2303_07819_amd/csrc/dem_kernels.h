// Device code of spdem: the fused DEM cell step, the cell statistics, the
// Lax-Friedrichs continuum update and the contact-pair export.
//
// Method: Deng, Stechmann & Chen, "Particle-continuum multiscale modeling of
// sea ice floes".  One doubly periodic DEM per coarse cell (Sec. 3.1); the DEM
// system and contact law of Sec. 2.1; cell statistics feeding the moment
// equations of Sec. 2.3; Lax-Friedrichs with the Oseen momentum advection
// (Sec. 3.2).
//
// Work decomposition: a "group" of W wavefronts owns one cell for one step.
// A workgroup holds max(1, 4 / W) groups (256 threads, or 512 for W = 8), so
// small cells run a wavefront each and large cells a tile of up to 8
// wavefronts.  Cells reach groups either in grid order from a cost-sorted cell
// list, or through a per-launch work counter (persistent workgroups).
//
// Per cell and step the group:
//   1. stages positions, radii, velocities and spins in LDS;
//   2. when the cell's candidate lists are stale (its floes may have moved by
//      half the skin since they were built), rebuilds them: binned schedule
//      counting sort into sub-bins of side >= 2 r_max + skin, FP32 screen of
//      candidate pairs with R + skin (all pairs, or a half shell over the
//      bin-sorted copy), each pair appended to both floes' lists, sorted and
//      kept in HBM; otherwise reads the kept lists.  Every listed candidate is
//      decided each step: within a 2^-19 relative guard band of touching by the
//      FP64 expression (dx dx + dy dy) < R R without contraction, outside it by
//      the FP32 screen, so the contact set is the one that expression defines;
//   3. per floe: ocean current and curl (angle addition around the cell centre,
//      minimax sincos), FP64 drag and drag torque, contacts in ascending
//      partner index (FP64), semi-implicit update, FP32 / fixed-point store;
//   4. reduces the FP64 statistics of the pre-step state (LDS + DPP, fixed
//      order, deterministic);
//   5. (optionally) advances the continuum of its cell by one LF step from the
//      previous time level's statistics (the continuum update of step k is
//      fused into the DEM launch of step k + 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spdem.h"

namespace spdem {

constexpr int kMomStride = 16;          // doubles per cell in the statistics buffers (128 B)
constexpr int kListCap = SP_CONTACT_CAP;
static_assert(kListCap % 8 == 0 && kListCap <= 32, "candidate lists: groups of eight, one 32-bit contact mask");
constexpr int kMaxBinsSide = 32;
constexpr double kPi = 3.14159265358979323846;
constexpr float kGuard = 1.0f / 524288.0f;  // 2^-19
constexpr int kDyn = 8;                 // statistics reduced by every step
constexpr int kSpringBytes = SP_SPRING_CAP * 8 + 16;   // LDS per floe of a blocked spring launch's contact history

// device fault bits
constexpr uint32_t kErrOverlap = 1u;
constexpr uint32_t kErrNaN = 2u;
constexpr uint32_t kErrCFL = 4u;
constexpr uint32_t kErrCapacity = 8u;
constexpr uint32_t kErrWall = 16u;

enum { M_N = 0, M_MASS, M_PX, M_PY, M_L, M_UX, M_UY, M_SVX, M_SVY, M_SW, M_AICE, M_UBAR, M_VBAR };

struct Modes {
    float kxL[SP_MAX_MODES];  // kx * Lx: phase per cell fraction
    float kyL[SP_MAX_MODES];
    double au[SP_MAX_MODES];
    double av[SP_MAX_MODES];
    double cz[SP_MAX_MODES];  // curl coefficient av kx - au ky
    int direct;               // every phase offset |kxL fx + kyL fy| (|fx|, |fy| <= 1/2) is <= 1.6
};

struct StepArgs {
    // floe state, SoA sorted by cell
    uint32_t* xi;
    uint32_t* yi;
    float* u;
    float* v;
    float* w;
    float* th;
    const float* r;
    const float* h;
    const int32_t* cell_start;
    const double2* phase;      // [ncells][nmodes]: (sin, cos) of the phase at the cell centre
    double* mom;               // statistics written by this step [ncells][kMomStride]
    double* mom_alt;           // where the statistics of work entries with w = 1 go instead
    uint32_t* err;
    unsigned long long* contacts;   // [ncells] contacts counted per cell since the floes were set
    unsigned long long* cands;
    uint4* tsp_j;              // tangential spring: per floe SP_SPRING_CAP partners (u16, 0xffff none)
    double* tsp_x;             // and their tangential displacements [n][SP_SPRING_CAP]      // [ncells] candidate tests counted per cell by blocked steps
    // candidate lists kept between steps (Verlet lists with a skin): per cell,
    // from floe-index start * kListCap, [kListCap / 8][n][8] (groups of eight
    // entries per floe), partner indices in ascending order; per floe its
    // candidate count; per cell a bound on the
    // largest floe displacement since the lists were built (a cell rebuilds when
    // it passes skin / 2, or is not finite)
    uint16_t* vlist;
    uint8_t* vcount;
    float* vdisp;
    float skin;                // m, added to R when the lists are built
    // work list
    const int4* work;          // (cell, first floe, floe count, statistics to mom_alt) of this launch, costliest first
    int32_t ncl;
    int32_t group_bytes;       // LDS bytes per group
    int32_t cap;               // LDS floe capacity per group
    // fused continuum update of the previous time level
    int32_t lf;
    const double* mom_prev;
    const double* Qp;          // [4][ncells]
    double* Qn;
    unsigned long long* max_cfl_bits;
    int32_t nx, ny;
    double dX, dY, inv_area;
    // geometry and constants
    int32_t ncells;
    int32_t nmodes;
    int32_t nbx, nby;          // sub-bins per side (1: all pairs along that axis)
    uint32_t flags;
    float qx, qy;              // Lx 2^-32, Ly 2^-32
    double qxd, qyd;
    double inv_qxd, inv_qyd;
    double dtd;
    double Ed, Gd, mud;
    double cdrho;              // Cd rho_o
    double rho_ice_d;
    double u0, v0;
    Modes modes;
};

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ float wave_max_f32(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    return x;
}

// Maximum over the wavefront of x >= 0 by DPP: row scans (row_shr 1, 2, 4, 8,
// zeros shifted in), then rows 1 and 3 take the last lane of rows 0 and 2
// (row_bcast:15) and rows 2 and 3 that of row 1 (row_bcast:31); lane 63 holds
// the maximum and every lane returns it.  No LDS traffic.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float x)
{
    // a row shift with every row enabled writes every lane (zero where the
    // source lies outside the row): no old value to keep
    if (CTRL < 0x140 && ROWS == 0xf) return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xf, CTRL < 0x140));
}

__device__ __forceinline__ float wave_max_nonneg(float x)
{
    x = fmaxf(x, dpp_f32<0x111, 0xf>(x));
    x = fmaxf(x, dpp_f32<0x112, 0xf>(x));
    x = fmaxf(x, dpp_f32<0x114, 0xf>(x));
    x = fmaxf(x, dpp_f32<0x118, 0xf>(x));
    x = fmaxf(x, dpp_f32<0x142, 0xa>(x));
    x = fmaxf(x, dpp_f32<0x143, 0xc>(x));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Square root of a finite x >= 0 (the drag speed): the hardware reciprocal
// square root y0, then Goldschmidt's coupled iteration for g ~ sqrt(x) and
// h ~ 1 / (2 sqrt(x)) (g = x y0, h = y0 / 2, r = 1/2 - g h, g += g r,
// h += h r) and one Newton correction g += (x - g^2) h; within an ulp of the
// rounded root.  0 at x = 0 (where the reciprocal root is infinite).
__device__ __forceinline__ double sqrt_nonneg(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}

// Square root d of a finite x > 0 and its reciprocal: the iteration of
// sqrt_nonneg, then one Newton step for h ~ 1 / (2 d) against the refined d
// (h += 2 h (1/2 - d h), quadratic in the error of h), and 1 / d = 2 h; within
// a few ulp of 1 / d.
__device__ __forceinline__ void root_and_reciprocal(double x, double& d, double& inv_d)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double e = fma(-g, g, x);
    g = fma(e, h, g);
    h = fma(2.0 * h, fma(-g, h, 0.5), h);
    d = g;
    inv_d = 2.0 * h;
}

// FP64 contact predicate: (dx*dx + dy*dy) < R*R without contraction.
__device__ __noinline__ bool exact_contact(int dxi, int dyi, float rl, float rj, double qxd,
                                           double qyd)
{
#pragma clang fp contract(off)
    double dx = (double)dxi * qxd;
    double dy = (double)dyi * qyd;
    double R = (double)rl + (double)rj;
    double d2 = dx * dx + dy * dy;
    return d2 < R * R;
}

// FP32 screen value d^2 - R^2 and R^2.
__device__ __forceinline__ void screen(int dxi, int dyi, float rl, float rj, float qx, float qy,
                                       float& diff, float& R2)
{
    float dx = (float)dxi * qx;
    float dy = (float)dyi * qy;
    float R = rl + rj;
    R2 = R * R;
    diff = (dx * dx + dy * dy) - R2;
}

// Final contact decision for a listed candidate.
__device__ __forceinline__ bool decide(int dxi, int dyi, float rl, float rj, const StepArgs& a)
{
    float diff, R2;
    screen(dxi, dyi, rl, rj, a.qx, a.qy, diff, R2);
    if (fabsf(diff) <= kGuard * R2) return exact_contact(dxi, dyi, rl, rj, a.qxd, a.qyd);
    return diff < 0.0f;
}

// sin and cos of a moderate FP32 argument: Cody-Waite reduction by pi/2 and
// Taylor polynomials on [-pi/4, pi/4] (truncation below 2e-9).
__device__ __forceinline__ void sincos_small(float x, float& s, float& c)
{
    const float k = rintf(x * 0.63661977236758134f);
    float r = fmaf(-k, 1.57079637050628662109375f, x);
    r = fmaf(k, 4.37113900018624283e-8f, r);
    const float r2 = r * r;
    float sp = fmaf(r2, 2.7557319224e-6f, -1.9841269841e-4f);
    sp = fmaf(r2, sp, 8.3333333333e-3f);
    sp = fmaf(r2, sp, -1.6666666667e-1f);
    const float sr = fmaf(r * r2, sp, r);
    float cp = fmaf(r2, -2.7557319224e-7f, 2.4801587302e-5f);
    cp = fmaf(r2, cp, -1.3888888889e-3f);
    cp = fmaf(r2, cp, 4.1666666667e-2f);
    cp = fmaf(r2, cp, -0.5f);
    const float cr = fmaf(r2, cp, 1.0f);
    const int q = (int)k;
    const float s1 = (q & 1) ? cr : sr;
    const float c1 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s1 : s1;
    c = ((q + 1) & 2) ? -c1 : c1;
}

// sin and cos of |x| <= 1.62 from minimax polynomials (Remez exchange for the
// absolute error on [-1.62, 1.62]): odd of degree 9 for sin (error 4.0e-8),
// even of degree 10 for cos (3.5e-10).  Evaluated in FP32, FP32 rounding
// included, they stay within 1.2e-7 and 1.6e-7 of sin and cos.
__device__ __forceinline__ void sincos_direct(float x, float& s, float& c)
{
    const float x2 = x * x;
    float sp = fmaf(x2, 2.62724643e-06f, -0.000198211215f);
    sp = fmaf(x2, sp, 0.0083332425f);
    sp = fmaf(x2, sp, -0.166666657f);
    s = fmaf(x * x2, sp, x);
    float cp = fmaf(x2, -2.59854716e-07f, 2.47567714e-05f);
    cp = fmaf(x2, cp, -0.0013888306f);
    cp = fmaf(x2, cp, 0.0416666344f);
    cp = fmaf(x2, cp, -0.5f);
    c = fmaf(x2, cp, 1.0f);
}

// Per-cell constants of ocean mode m: with a the mode's velocity amplitudes
// (au, av), cz its curl coefficient and theta_c its phase at the cell centre
// (S = sin theta_c, C = cos theta_c): the products au S, au C, av S, av C,
// cz C, -cz S in FP64, and the mode's phase per cell fraction kx Lx, ky Ly.
struct ModeC {
    double aS, aC, bS, bC, zC, zS;
    float kxL, kyL;
};

__device__ __forceinline__ void mode_consts(const Modes& md, int m, double2 sc, ModeC* mc)
{
    const double au = md.au[m], av = md.av[m], cz = md.cz[m];
    ModeC q;
    q.aS = au * sc.x;
    q.aC = au * sc.y;
    q.bS = av * sc.x;
    q.bC = av * sc.y;
    q.zC = cz * sc.y;
    q.zS = -(cz * sc.x);
    q.kxL = md.kxL[m];
    q.kyL = md.kyL[m];
    mc[m] = q;
}

// Ocean current (sum of a sin theta) and curl (sum of cz cos theta) at cell
// fraction (fx, fy), by angle addition around the cell centre: theta = theta_c
// + d with d = kx Lx fx + ky Ly fy, sin theta = S cos d + C sin d and
// cos theta = C cos d - S sin d, the amplitudes folded into the constants of
// mode_consts.  sin d and cos d are FP32 polynomials of the FP32 offset
// (within 2e-7 of the exact values); the products with the cell constants and
// the sum over modes are FP64: the drag depends on the current minus the floe
// velocity, a small difference of nearly equal values, and FP32 constants and
// sums (relative error about 3e-7 of the current) moved cell drag sums by up
// to 3e-7 of their scale, ten times what the FP32 storage of the state does.
// DIRECT: every |d| <= 1.6.
template <bool DIRECT>
__device__ __forceinline__ void ocean_modes_t(float fx, float fy, const ModeC* mc, int nmodes, double& uo,
                                              double& vo, double& zeta)
{
#pragma unroll 2
    for (int m = 0; m < nmodes; ++m) {
        const ModeC q = mc[m];
        const float d = q.kxL * fx + q.kyL * fy;
        float sdf, cdf;
        if (DIRECT)
            sincos_direct(d, sdf, cdf);
        else
            sincos_small(d, sdf, cdf);
        const double sd = sdf, cd = cdf;
        uo = fma(q.aC, sd, fma(q.aS, cd, uo));
        vo = fma(q.bC, sd, fma(q.bS, cd, vo));
        zeta = fma(q.zS, sd, fma(q.zC, cd, zeta));
    }
}

__device__ __forceinline__ void ocean_modes(float fx, float fy, const ModeC* mc, int nmodes, bool direct,
                                            double& uo, double& vo, double& zeta)
{
    if (direct)
        ocean_modes_t<true>(fx, fy, mc, nmodes, uo, vo, zeta);
    else
        ocean_modes_t<false>(fx, fy, mc, nmodes, uo, vo, zeta);
}

// Contact of floe l (radius rld, velocity (uld, vld), spin wld) with floe j at
// fixed-point offset (dxi, dyi), radius rj, velocity and spin vj (Sec. 2.1),
// FP64: with d the centre distance, n the unit normal and t = (-n_y, n_x), the
// overlap delta = d - (r_l + r_j) < 0 and the contact chord c (the full chord
// of the overlapping disks, the smaller diameter once one disk lies within the
// other), the normal force E c delta n and the tangential force
// G c v_t t capped at mu |F_n|, v_t the relative tangential velocity with the
// spins' surface speeds; the torque is r_l F_t.  The spin sum takes its
// operands in a fixed order (lower floe index first) so that the two floes of
// a pair see the same value.  The contributions are returned, not summed, so
// that any lane can evaluate a pair; false for coincident centres (no force).
// SPRING: the tangential force is the incremental spring (SP_TANGENTIAL_SPRING):
// the pair's displacement xi_old (0 for a new contact) grows by v_t dt, the
// force is c G xi, and past mu |F_n| the contact slips (the force at the
// Coulomb limit, xi the displacement that gives it); xi receives the new value.
template <bool SPRING = false>
__device__ __forceinline__ bool contact_terms(int dxi, int dyi, double rld, double uld, double vld, double wld,
                                              float rj, float4 vj, bool lower, const StepArgs& a, double& cx,
                                              double& cy, double& ct, double xi_old = 0.0, double* xi = nullptr)
{
    const double dx = (double)dxi * a.qxd, dy = (double)dyi * a.qyd;
    const double d2 = dx * dx + dy * dy;
    if (!(d2 > 0.0)) return false;
    const double rjd = (double)rj;
    double d, inv_d;
    root_and_reciprocal(d2, d, inv_d);
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
        cc = sqrt_nonneg(fmax(p, 0.0)) * inv_d;
    }
    const double Fn = cc * a.Ed * delta;
    const double wjd = (double)vj.z;
    const double spin = lower ? (wld * rld + wjd * rjd) : (wjd * rjd + wld * rld);
    const double vt = (((double)vj.x - uld) * tx + ((double)vj.y - vld) * ty) - spin;
    const double capf = a.mud * fabs(Fn);
    double Ft;
    if (SPRING) {
        const double k = cc * a.Gd;            // tangential stiffness of the contact
        double x = xi_old + vt * a.dtd;
        Ft = k * x;
        if (Ft > capf || Ft < -capf) {         // slip: the spring stretches no further
            Ft = Ft > capf ? capf : -capf;
            x = k > 0.0 ? Ft / k : 0.0;
        }
        *xi = x;
    } else {
        Ft = fmin(fmax(cc * a.Gd * vt, -capf), capf);
    }
    cx = fma(Fn, nx, Ft * tx);
    cy = fma(Fn, ny, Ft * ty);
    ct = rld * Ft;
    return true;
}

// Add one contact's contributions to a floe's sums.  The operands pass
// through an empty asm so that no product feeding them is fused into the
// sums: the result is the same whichever lane computed the contributions.
__device__ __forceinline__ void add_terms(double& Fx, double& Fy, double& T, double cx, double cy, double ct)
{
    asm volatile("" : "+v"(cx), "+v"(cy), "+v"(ct));
    Fx += cx;
    Fy += cy;
    T += ct;
}

// Sum over a row of 16 lanes with DPP row shifts (deterministic order); the
// row total lands in the row's last lane.
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row_sum(double x)
{
    x += dpp_shr<0x111>(x);   // row_shr:1
    x += dpp_shr<0x112>(x);   // row_shr:2
    x += dpp_shr<0x114>(x);   // row_shr:4
    x += dpp_shr<0x118>(x);   // row_shr:8
    return x;
}

// A lane permutation within rows (row_ror, row_half_mirror, quad_perm); every
// lane of the wavefront must be active, since no old value is kept.
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Row totals (16 lanes) of eight values per lane by a transposing exchange:
// at each stage a lane keeps half of its values and adds its partner's copy of
// that half (partners: lane i ^ 8 by row_ror:8, i ^ 7 by row_half_mirror,
// i ^ 2 and i ^ 1 by quad permutes), so lane i of a row ends with the row
// total of value i >> 1 (both lanes of a pair hold it).  About half the
// instructions of eight row sums.  Every lane of the wavefront must be active.
__device__ __forceinline__ double row_sum8(const double (&v)[8], int lane)
{
    const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    double a4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        a4[j] = (b3 ? v[j + 4] : v[j]) + dpp_perm<0x128>(b3 ? v[j] : v[j + 4]);
    double a2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
        a2[j] = (b2 ? a4[j + 2] : a4[j]) + dpp_perm<0x141>(b2 ? a4[j] : a4[j + 2]);
    const double a1 = (b1 ? a2[1] : a2[0]) + dpp_perm<0x4e>(b1 ? a2[0] : a2[1]);
    return a1 + dpp_perm<0xb1>(a1);
}

// Exclusive scan of cnt[0..nb) into start[0..nb] by the G threads of a group
// (thread gt of group g); nb <= 16 G.  Every thread of the workgroup calls it.
template <int G>
__device__ void group_exclusive_scan(const int* cnt, int* start, int nb, int gt, int* wsum)
{
    constexpr int W = G / 64;
    const int lane = gt & 63, wave = gt >> 6;
    const int ch = (nb + G - 1) / G;
    const int b0 = gt * ch;
    int tot = 0;
    for (int k = 0; k < ch; ++k) tot += (b0 + k < nb) ? cnt[b0 + k] : 0;
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int run = incl - tot;
#pragma unroll
    for (int k = 0; k < W; ++k) run += (k < wave) ? wsum[k] : 0;
    for (int k = 0; k < ch; ++k) {
        if (b0 + k < nb) start[b0 + k] = run;
        run += (b0 + k < nb) ? cnt[b0 + k] : 0;
    }
    if (gt == G - 1) start[nb] = run;
    __syncthreads();
}

// Statistics reduced by every step.  n, M and A_ice depend only on the radii
// and thicknesses; the statistics kernel writes them when the floes are set.
__device__ __forceinline__ int dyn_slot(int k)
{
    return k < 3 ? M_PX + k : M_UX + (k - 3);   // Px Py L | Ux Uy Svx Svy Sw
}

// Append partner index `who` to the contact list of floe `to`.
__device__ __forceinline__ void list_append(uint16_t* lst, int* cnt, int to, int who)
{
    const int slot = atomicAdd(&cnt[to], 1);
    if (slot < kListCap) lst[(size_t)to * kListCap + slot] = (uint16_t)who;
}

// Screen the candidates q in [q0, q1) of the sorted copy against floe o; the
// next candidate is loaded while the current one is screened.
__device__ __forceinline__ void sweep(const uint4* S, int q0, int q1, uint32_t xl, uint32_t yl,
                                     float rl, int o, uint16_t* lst, int* cnt, const StepArgs& a)
{
    if (q0 >= q1) return;
    uint4 pj = S[q0];
    for (int q = q0; q < q1; ++q) {
        const uint4 nxt = S[min(q + 1, q1 - 1)];
        float diff, R2;
        screen((int)(pj.x - xl), (int)(pj.y - yl), rl, __uint_as_float(pj.z), a.qx, a.qy, diff, R2);
        if (diff < kGuard * R2) {
            const int o2 = (int)(pj.w & 0xffffu);
            list_append(lst, cnt, o, o2);
            list_append(lst, cnt, o2, o);
        }
        pj = nxt;
    }
}

// ---------------------------------------------------------- continuum step
// One Lax-Friedrichs step of eq. pde for cell C (Sec. 3.2): mass and spin
// angular momentum in conservative form with flux <v> q, momentum with the
// Oseen approximation <v>.grad<rho v>, drag sources S / A; periodic grid.
// The step reads kLfOps operands (lf_operand), so that a caller can load them
// early and spread over lanes, then combines them (lf_from_ops).
constexpr int kLfOps = 25;

struct LfNeighbours {
    int E, W, N, S;
};

// With walls in x (SP_WALL_X, Sec. 4.4) the neighbour beyond the first or
// last column is a ghost cell of zero state and zero coefficients (-1).
__device__ __forceinline__ LfNeighbours lf_neighbours(int C, int nx, int ny, bool wall)
{
    const int ix = C % nx, iy = C / nx;
    LfNeighbours b;
    b.E = (wall && ix + 1 == nx) ? -1 : iy * nx + (ix + 1 == nx ? 0 : ix + 1);
    b.W = (wall && ix == 0) ? -1 : iy * nx + (ix == 0 ? nx - 1 : ix - 1);
    b.N = (iy + 1 == ny ? 0 : iy + 1) * nx + ix;
    b.S = (iy == 0 ? ny - 1 : iy - 1) * nx + ix;
    return b;
}

// Operand t of the step of cell C: 0..15 Q[f][E, W, N, S] (f = t / 4);
// 16..21 <u>_E, <u>_W, <v>_N, <v>_S, <u>_C, <v>_C; 22..24 the sources S_w,
// S_vx, S_vy of C.
__device__ __forceinline__ double lf_operand(int C, int t, const double* mom, const double* Q, int nx,
                                            int ny, bool wall)
{
    const LfNeighbours b = lf_neighbours(C, nx, ny, wall);
    const int nc = nx * ny;
    if (t < 16) {
        const int k = t & 3;
        const int cell = k == 0 ? b.E : k == 1 ? b.W : k == 2 ? b.N : b.S;
        return cell < 0 ? 0.0 : Q[(size_t)(t >> 2) * nc + cell];
    }
    int cell, slot;
    switch (t) {
    case 16: cell = b.E; slot = M_UBAR; break;
    case 17: cell = b.W; slot = M_UBAR; break;
    case 18: cell = b.N; slot = M_VBAR; break;
    case 19: cell = b.S; slot = M_VBAR; break;
    case 20: cell = C; slot = M_UBAR; break;
    case 21: cell = C; slot = M_VBAR; break;
    case 22: cell = C; slot = M_SW; break;
    case 23: cell = C; slot = M_SVX; break;
    default: cell = C; slot = M_SVY; break;
    }
    return cell < 0 ? 0.0 : mom[(size_t)cell * kMomStride + slot];
}

__device__ __forceinline__ void lf_from_ops(int C, const double* o, double* Qn, int nc, double dT, double dX,
                                            double dY, double inv_area, unsigned long long* max_cfl_bits,
                                            uint32_t* err)
{
    const double uE = o[16], uW = o[17], vN = o[18], vS = o[19], uC = o[20], vC = o[21];
    const double cx = dT / (2.0 * dX), cy = dT / (2.0 * dY);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const double qE = o[4 * f], qW = o[4 * f + 1];
        const double qN = o[4 * f + 2], qS = o[4 * f + 3];
        const double avg = 0.25 * (qE + qW + qN + qS);
        double q;
        if (f == 0) {
            q = avg - cx * (uE * qE - uW * qW) - cy * (vN * qN - vS * qS);
        } else if (f == 3) {
            q = avg - cx * (uE * qE - uW * qW) - cy * (vN * qN - vS * qS) + dT * o[22] * inv_area;
        } else {
            q = avg - dT * (uC * (qE - qW) / (2.0 * dX) + vC * (qN - qS) / (2.0 * dY)) +
                dT * o[f == 1 ? 23 : 24] * inv_area;
        }
        Qn[(size_t)f * nc + C] = q;
    }
    const double cfl = fabs(uC) * dT / dX + fabs(vC) * dT / dY;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(cfl);
    if (bits > *max_cfl_bits) atomicMax(max_cfl_bits, bits);
    if (cfl > 1.0) atomicOr(err, kErrCFL);
}

__device__ __forceinline__ void lf_cell(int C, const double* mom, const double* Q, double* Qn,
                                        int nx, int ny, double dT, double dX, double dY,
                                        double inv_area, unsigned long long* max_cfl_bits,
                                        uint32_t* err, bool wall)
{
    double o[kLfOps];
#pragma unroll
    for (int t = 0; t < kLfOps; ++t) o[t] = lf_operand(C, t, mom, Q, nx, ny, wall);
    lf_from_ops(C, o, Qn, nx * ny, dT, dX, dY, inv_area, max_cfl_bits, err);
}

// ------------------------------------------------------------- DEM step
// SCHED: 1 all pairs, 2 binned half shell.  W: wavefronts per cell.
// PERSIST: a grid of resident workgroups strides over the work list.
// ONE: no cell has more floes than the group has lanes (one floe per lane:
// the floe loop carries nothing, which frees registers for occupancy).
// TSP: the tangential spring (SP_TANGENTIAL_SPRING), each floe's contact
// history read before its contacts and rewritten with them.
template <int SCHED, int W, bool PERSIST, bool ONE, bool TSP = false>
__global__ __launch_bounds__(W >= 4 ? 64 * W : 256) void dem_step_kernel(StepArgs a)
{
    constexpr int G = 64 * W;                  // threads per group
    constexpr int BT = G >= 256 ? G : 256;     // largest workgroup
    constexpr int GPB = BT / G;                // largest number of groups (cells) per workgroup
    const int gpb = blockDim.x / G;            // groups in this launch (LDS may allow fewer)

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ ModeC mode_c[GPB][SP_MAX_MODES];        // per-cell mode constants (mode_consts)
    __shared__ int wsum[GPB][W];
    __shared__ float wdisp[BT / 64];
    __shared__ unsigned long long csum[BT / 64];
    __shared__ double lfops[GPB][kLfOps];

    const int tid = threadIdx.x;
    const int g = tid / G, gt = tid % G;
    unsigned char* gsm = smem + (size_t)g * a.group_bytes;
    const int cap = a.cap;

    uint4* P = reinterpret_cast<uint4*>(gsm);                 // xi, yi, r bits, theta bits
    float4* V = reinterpret_cast<float4*>(P + cap);           // u, v, w, -
    uint4* S = reinterpret_cast<uint4*>(V + cap);             // sorted copy: xi, yi, r bits, index | bin << 16
    uint16_t* lst = reinterpret_cast<uint16_t*>(S + (SCHED == 2 ? cap : 0));  // [cap][kListCap]
    int* cnt = reinterpret_cast<int*>(lst + (size_t)cap * kListCap);
    // sort scratch of the binned schedule, inside the list region: a group that
    // rebuilds its lists fills them only after the sort
    static_assert(2 * sizeof(int) <= kListCap * sizeof(uint16_t), "sort scratch fits the list region");
    int* binof = reinterpret_cast<int*>(lst);
    int* rank = binof + cap;
    int* bcnt = cnt + cap;
    int* bstart = bcnt + (SCHED == 2 ? a.nbx * a.nby : 0);
    double* red = reinterpret_cast<double*>(gsm);             // [kDyn][G], after the floes are done

    const int stride = PERSIST ? (int)gridDim.x * gpb : 0;
    for (int base = blockIdx.x * gpb; base < a.ncl; base += stride) {
        const int item = base + g;
        const bool valid = item < a.ncl;
        const int4 wk = valid ? a.work[item] : make_int4(0, 0, 0, 0);
        const int c = wk.x, s = wk.y, n = wk.z;
        const unsigned long long ccell = (valid && gt == 0) ? a.contacts[c] : 0ull;   // loaded early
        // the continuum update of the previous level for this cell reads only
        // buffers this launch does not write: its operands are loaded now, one
        // per lane, and combined after the floes are done
        const double lfo = (valid && a.lf && gt < kLfOps) ? lf_operand(c, gt, a.mom_prev, a.Qp, a.nx, a.ny, (a.flags & SP_WALL_X) != 0) : 0.0;
        // rebuild the cell's candidate lists when its floes may have moved by
        // skin / 2 since they were built (every pair then changed its distance
        // by less than the skin); the same for the whole group
        const float vd = valid ? a.vdisp[c] : 0.0f;
        const bool build = valid && !(vd <= 0.5f * a.skin);
        const int nb_build = build ? n : 0;        // loop bound of the build work
        uint16_t* const vlst = a.vlist + (size_t)s * kListCap;

        if (valid && gt < a.nmodes) mode_consts(a.modes, gt, a.phase[(size_t)c * a.nmodes + gt], mode_c[g]);
        for (int i = gt; i < n; i += G) {
            P[i] = make_uint4(a.xi[s + i], a.yi[s + i], __float_as_uint(a.r[s + i]), __float_as_uint(a.th[s + i]));
            V[i] = make_float4(a.u[s + i], a.v[s + i], a.w[s + i], a.h[s + i]);
            if (build) {
                cnt[i] = 0;
            } else {
                // kept candidates: the first eight in one 16-byte load issued with
                // the floe state, the rest (rare) after the count
                const int k = a.vcount[s + i];
                cnt[i] = k;
                uint16_t* my = lst + (size_t)i * kListCap;
                *reinterpret_cast<uint4*>(my) = *reinterpret_cast<const uint4*>(vlst + (size_t)i * 8);
                for (int q = 8; q < k; q += 8)
                    *reinterpret_cast<uint4*>(my + q) =
                        *reinterpret_cast<const uint4*>(vlst + (size_t)q * n + (size_t)i * 8);
            }
        }
        // the search runs only in workgroups where some cell rebuilds its lists
        // (the barriers below are workgroup-wide)
        const bool any_build = __syncthreads_or(build);
        if (SCHED == 2 && any_build) {
            const int nb = a.nbx * a.nby;
            for (int b = gt; b < nb; b += G) bcnt[b] = 0;
            __syncthreads();
            for (int i = gt; i < nb_build; i += G) {
                const int bx = (int)__umulhi(P[i].x, (uint32_t)a.nbx);
                const int by = (int)__umulhi(P[i].y, (uint32_t)a.nby);
                const int b = by * a.nbx + bx;
                binof[i] = b;
                rank[i] = atomicAdd(&bcnt[b], 1);
            }
            __syncthreads();
            group_exclusive_scan<G>(bcnt, bstart, nb, gt, wsum[g]);
            for (int i = gt; i < nb_build; i += G) {
                uint4 p = P[i];
                p.w = (uint32_t)i | ((uint32_t)binof[i] << 16);
                S[bstart[binof[i]] + rank[i]] = p;
            }
            __syncthreads();
        }

        // ---- phase 1: contact candidates -> per-floe lists
        if (SCHED == 1) {
            // every floe against every floe (itself included, skipped later);
            // the list comes out in ascending partner order
            for (int l = gt; l < nb_build; l += G) {
                const uint4 pl = P[l];
                const float rl = __uint_as_float(pl.z) + a.skin;
                uint16_t* my = lst + (size_t)l * kListCap;
                int k = 0;
                for (int j = 0; j < n; ++j) {
                    const uint4 pj = P[j];
                    float diff, R2;
                    screen((int)(pj.x - pl.x), (int)(pj.y - pl.y), rl, __uint_as_float(pj.z), a.qx,
                           a.qy, diff, R2);
                    if (diff < kGuard * R2) {
                        if (k < kListCap) my[k] = (uint16_t)j;
                        ++k;
                    }
                }
                cnt[l] = k;
            }
        } else {
            // half shell over the bin-sorted copy: lanes take consecutive sorted
            // floes (neighbouring lanes share their neighbourhood); each pair is
            // screened once, from the bin whose offset to the other is in
            // {own bin (later sorted index), E, NW, N, NE}, and appended to both lists
            for (int t = gt; t < nb_build; t += G) {
                const uint4 own = S[t];
                const int o = (int)(own.w & 0xffffu);
                const int b = (int)(own.w >> 16);
                const int bx = b % a.nbx, by = b / a.nbx;
                const float rl = __uint_as_float(own.z) + a.skin;
                if (a.nbx >= 3 && bx + 1 < a.nbx) {
                    // own-bin tail and the east bin are contiguous
                    sweep(S, t + 1, bstart[b + 2], own.x, own.y, rl, o, lst, cnt, a);
                } else {
                    sweep(S, t + 1, bstart[b + 1], own.x, own.y, rl, o, lst, cnt, a);
                    if (a.nbx >= 3) {
                        const int be = by * a.nbx;   // east neighbour across the seam
                        sweep(S, bstart[be], bstart[be + 1], own.x, own.y, rl, o, lst, cnt, a);
                    }
                }
                if (a.nby >= 3) {
                    const int row = (by + 1 == a.nby ? 0 : by + 1) * a.nbx;
                    if (a.nbx < 3) {
                        sweep(S, bstart[row], bstart[row + a.nbx], own.x, own.y, rl, o, lst, cnt, a);
                    } else if (bx == 0) {
                        sweep(S, bstart[row], bstart[row + 2], own.x, own.y, rl, o, lst, cnt, a);
                        sweep(S, bstart[row + a.nbx - 1], bstart[row + a.nbx], own.x, own.y, rl, o, lst,
                              cnt, a);
                    } else if (bx == a.nbx - 1) {
                        sweep(S, bstart[row + a.nbx - 2], bstart[row + a.nbx], own.x, own.y, rl, o, lst,
                              cnt, a);
                        sweep(S, bstart[row], bstart[row + 1], own.x, own.y, rl, o, lst, cnt, a);
                    } else {
                        sweep(S, bstart[row + bx - 1], bstart[row + bx + 2], own.x, own.y, rl, o, lst,
                              cnt, a);
                    }
                }
            }
        }
        __syncthreads();

        double acc[kDyn];
#pragma unroll
        for (int k = 0; k < kDyn; ++k) acc[k] = 0.0;
        unsigned long long ncontact = 0;
        float maxdisp = 0.0f;

        for (int l = gt; l < n; l += G) {
            if (ONE && l >= G) break;   // not reached: the launch guarantees n <= G
            const uint4 pl = P[l];
            const float4 vv = V[l];
            const uint32_t xl = pl.x, yl = pl.y;
            const float rl = __uint_as_float(pl.z);
            const float ul = vv.x, vl = vv.y, wl = vv.z;

            // ---- ocean current and curl at the floe centre (angle addition around
            // the cell centre keeps the FP32 arguments below (|kx| Lx + |ky| Ly) / 2),
            // then drag and drag torque in FP64
            const double rld = (double)rl, uld = (double)ul, vld = (double)vl, wld = (double)wl;
            double fdx = 0.0, fdy = 0.0, tdr = 0.0;
            if (!(a.flags & SP_OCEAN_OFF)) {
                const float fx = (float)(int)(xl - 0x80000000u) * 2.3283064365386963e-10f;
                const float fy = (float)(int)(yl - 0x80000000u) * 2.3283064365386963e-10f;
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
            const double md = a.rho_ice_d * (double)vv.w * kPi * rld * rld;

            uint16_t* my = lst + (size_t)l * kListCap;
            int k;
            if (build) {
                k = cnt[l];
                if (k > kListCap) {
                    atomicOr(a.err, kErrCapacity);
                    k = kListCap;
                }
                if (SCHED == 2) {
                    // ascending partner order: insertion sort of the short list
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
                // keep the list for the steps until the next rebuild
                for (int q = 0; q < k; ++q) vlst[(size_t)(q & ~7) * n + (size_t)l * 8 + (q & 7)] = my[q];
                a.vcount[s + l] = (uint8_t)k;
            } else {
                k = cnt[l];   // staged with the floe state
            }

            // ---- contact decisions: every candidate, eight indices per LDS read;
            // the contacts become a bit mask over the (ascending) list
            uint32_t cmask = 0;
            for (int q0 = 0; q0 < k; q0 += 8) {
                const uint4 ix = *reinterpret_cast<const uint4*>(my + q0);
                const int qe = min(8, k - q0);
                for (int t = 0; t < qe; ++t) {
                    const uint32_t wv = t < 2 ? ix.x : t < 4 ? ix.y : t < 6 ? ix.z : ix.w;
                    const int j = (int)((wv >> (16 * (t & 1))) & 0xffffu);
                    if (j == l) continue;
                    const uint4 pj = P[j];
                    if (decide((int)(pj.x - xl), (int)(pj.y - yl), rl, __uint_as_float(pj.z), a))
                        cmask |= 1u << (q0 + t);
                }
            }

            // ---- contact forces and torques in ascending partner order (FP64);
            // a wave runs as many rounds as its lanes have contacts at most
            double Fx = fdx, Fy = fdy, T = tdr;
            // the floe's contact history (TSP): partners and displacements
            // after the previous step, rewritten below with this step's contacts
            uint4 hj = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
            double hx[SP_SPRING_CAP];
            uint16_t* const tj = TSP ? reinterpret_cast<uint16_t*>(a.tsp_j + s + l) : nullptr;
            double* const tx = TSP ? a.tsp_x + (size_t)(s + l) * SP_SPRING_CAP : nullptr;
            bool had = false;   // the floe was in contact after the previous step
            if (TSP) {
                hj = a.tsp_j[s + l];
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
                if (!contact_terms<TSP>((int)(pj.x - xl), (int)(pj.y - yl), rld, uld, vld, wld,
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
                ncontact += (l < j) ? 1ull : 0ull;
            }
            if (TSP && (had || nh > 0))   // a floe out of contact before and now keeps its empty table
                for (int e = nh; e < SP_SPRING_CAP; ++e) {
                    tj[e] = 0xffffu;
                    tx[e] = 0.0;
                }

            // ---- time update (semi-implicit Euler by default), FP64 arithmetic,
            // FP32 / fixed-point storage
            const double inv_m = 1.0 / md;
            const double dt = a.dtd;
            const double und = uld + dt * (Fx * inv_m);
            const double vnd = vld + dt * (Fy * inv_m);
            const double inv_i = 1.0 / (md * (rld * rld));
            const double wnd = wld + dt * (T * inv_i);
            const bool fe = (a.flags & SP_FORWARD_EULER) != 0;
            const double ux = fe ? uld : und, vx = fe ? vld : vnd, wx = fe ? wld : wnd;
            const int sx = __double2int_rn(dt * ux * a.inv_qxd);
            const int sy = __double2int_rn(dt * vx * a.inv_qyd);
            {
                const float ddx = (float)sx * a.qx, ddy = (float)sy * a.qy;
                maxdisp = fmaxf(maxdisp, sqrtf(ddx * ddx + ddy * ddy));
            }
            const float un = (float)und, vn = (float)vnd, wn = (float)wnd;
            a.xi[s + l] = xl + (uint32_t)sx;
            a.yi[s + l] = yl + (uint32_t)sy;
            a.u[s + l] = un;
            a.v[s + l] = vn;
            a.w[s + l] = wn;
            a.th[s + l] = (float)((double)__uint_as_float(pl.w) + dt * wx);
            if (!(isfinite(un) && isfinite(vn) && isfinite(wn))) atomicOr(a.err, kErrNaN);

            // ---- statistics of the pre-step state (FP64)
            acc[0] += md * uld;
            acc[1] += md * vld;
            acc[2] += md * rld * rld * wld;
            acc[3] += uld;
            acc[4] += vld;
            acc[5] += fdx;
            acc[6] += fdy;
            acc[7] += tdr;
        }

        // ---- group reduction through LDS: lane partials -> 16 segment sums per
        // quantity -> DPP row sum (fixed order, deterministic)
        const unsigned long long cs = wave_sum_u64(ncontact);
        const float wd = wave_max_f32(maxdisp);
        if ((tid & 63) == 0) {
            csum[tid >> 6] = cs;
            wdisp[tid >> 6] = wd;
        }
        __syncthreads();   // every lane is done with the cell's LDS data
        if (valid && gt == 0) {
            float d = 0.0f;
            for (int q = 0; q < W; ++q) d = fmaxf(d, wdisp[g * W + q]);
            // the bound grows by the largest displacement of this step (rounded up)
            a.vdisp[c] = (build ? 0.0f : vd) + d * 1.0001f + 1e-3f;
        }
#pragma unroll
        for (int k = 0; k < kDyn; ++k) red[k * G + gt] = acc[k];
        if (gt < kLfOps) lfops[g][gt] = lfo;
        __syncthreads();
        constexpr int SEG = G / 16;                 // values per segment
        for (int kq = gt >> 4; kq < kDyn; kq += G / 16) {
            // segment seg sums lanes seg, seg + 16, ... in order (neighbouring
            // lanes read neighbouring words: no bank conflicts)
            const int seg = gt & 15;
            const double* src = red + kq * G + seg;
            double x = 0.0;
#pragma unroll
            for (int i = 0; i < SEG; ++i) x += src[16 * i];
            x = row_sum(x);
            if (seg == 15 && valid) {
                const int slot = dyn_slot(kq);
                double* const mo = wk.w ? a.mom_alt : a.mom;
                mo[(size_t)c * kMomStride + slot] = x;
                if (slot == M_UX || slot == M_UY)   // continuum coefficient <v> = U / n
                    mo[(size_t)c * kMomStride + (slot == M_UX ? M_UBAR : M_VBAR)] =
                        n > 0 ? x / (double)n : 0.0;
            }
        }
        if (valid && gt == 0) {
            // per-cell running count, written by the cell's own group only (one
            // shared counter would serialise every workgroup on one address)
            unsigned long long t = 0;
            for (int q = 0; q < W; ++q) t += csum[g * W + q];
            a.contacts[c] = ccell + t;
        }
        // continuum update of the previous level for this cell (operands loaded
        // at the start of the cell)
        if (valid && a.lf && gt == G - 1)
            lf_from_ops(c, lfops[g], a.Qn, a.nx * a.ny, a.dtd, a.dX, a.dY, a.inv_area, a.max_cfl_bits, a.err);
        if (!PERSIST) break;
        __syncthreads();   // the cell's LDS data is free
    }
}

// ------------------------------------------------------- cell statistics
// All 11 statistics of the current state, one 256-thread workgroup per cell
// (cell c0 + blockIdx.x, or cells[blockIdx.x] with a cell list), written to
// row c - c0 of a.mom.
__global__ __launch_bounds__(256) void stats_kernel(StepArgs a, const int32_t* cells, int c0)
{
    __shared__ double red11[SP_NMOM][16];
    __shared__ ModeC mode_c[SP_MAX_MODES];
    const int c = cells ? cells[blockIdx.x] : c0 + (int)blockIdx.x;
    const int tid = threadIdx.x;
    const int s = a.cell_start[c];
    const int n = a.cell_start[c + 1] - s;
    if (tid < a.nmodes) mode_consts(a.modes, tid, a.phase[(size_t)c * a.nmodes + tid], mode_c);
    __syncthreads();
    double acc[SP_NMOM];
#pragma unroll
    for (int k = 0; k < SP_NMOM; ++k) acc[k] = 0.0;
    for (int l = tid; l < n; l += 256) {
        const uint32_t xl = a.xi[s + l], yl = a.yi[s + l];
        const double rld = a.r[s + l], uld = a.u[s + l], vld = a.v[s + l], wld = a.w[s + l];
        double fdx = 0.0, fdy = 0.0, tdr = 0.0;
        if (!(a.flags & SP_OCEAN_OFF)) {
            const float fx = (float)(int)(xl - 0x80000000u) * 2.3283064365386963e-10f;
            const float fy = (float)(int)(yl - 0x80000000u) * 2.3283064365386963e-10f;
            double uo = a.u0, vo = a.v0, zeta = 0.0;
            ocean_modes(fx, fy, mode_c, a.nmodes, a.modes.direct != 0, uo, vo, zeta);
            const double du = uo - uld, dv = vo - vld;
            const double sp = sqrt_nonneg(du * du + dv * dv);
            const double alpha = a.cdrho * kPi * rld * rld;
            fdx = alpha * du * sp;
            fdy = alpha * dv * sp;
            const double dW = 0.5 * zeta - wld;
            const double r2 = rld * rld;
            tdr = a.cdrho * kPi * r2 * r2 * rld * dW * fabs(dW);
        }
        const double md = a.rho_ice_d * (double)a.h[s + l] * kPi * rld * rld;
        acc[M_N] += 1.0;
        acc[M_MASS] += md;
        acc[M_PX] += md * uld;
        acc[M_PY] += md * vld;
        acc[M_L] += md * rld * rld * wld;
        acc[M_UX] += uld;
        acc[M_UY] += vld;
        acc[M_SVX] += fdx;
        acc[M_SVY] += fdy;
        acc[M_SW] += tdr;
        acc[M_AICE] += kPi * rld * rld;
    }
    const int lane = tid & 63, rowid = tid >> 4;
#pragma unroll
    for (int k = 0; k < SP_NMOM; ++k) {
        const double x = row_sum(acc[k]);
        if ((lane & 15) == 15) red11[k][rowid] = x;
    }
    __syncthreads();
    if (tid < SP_NMOM) {
        double x = red11[tid][0];
#pragma unroll
        for (int q = 1; q < 16; ++q) x += red11[tid][q];
        double* const row = a.mom + (size_t)(c - c0) * kMomStride;
        row[tid] = x;
        if (tid == M_UX || tid == M_UY) row[tid == M_UX ? M_UBAR : M_VBAR] = n > 0 ? x / (double)n : 0.0;
    }
}

// ------------------------------------------------ standalone continuum step
__global__ __launch_bounds__(64) void lf_kernel(const double* mom, const double* Q, double* Qn, int nx,
                                                int ny, double dT, double dX, double dY,
                                                double inv_area, unsigned long long* max_cfl_bits,
                                                uint32_t* err, int wall)
{
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C < nx * ny) lf_cell(C, mom, Q, Qn, nx, ny, dT, dX, dY, inv_area, max_cfl_bits, err, wall != 0);
}

// The same update for the listed cells only (the cells without floes, which
// stay out of the DEM launches).
__global__ __launch_bounds__(64) void lf_list_kernel(const int32_t* cells, int ncl, const double* mom, const double* Q,
                                                     double* Qn, int nx, int ny, double dT, double dX, double dY,
                                                     double inv_area, unsigned long long* max_cfl_bits,
                                                     uint32_t* err, int wall)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncl) lf_cell(cells[i], mom, Q, Qn, nx, ny, dT, dX, dY, inv_area, max_cfl_bits, err, wall != 0);
}

__global__ void q_from_moments_kernel(const double* mom, double* Q, int nc, double inv_area)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double* s = mom + (size_t)c * kMomStride;
    Q[c] = s[M_MASS] * inv_area;
    Q[(size_t)nc + c] = s[M_PX] * inv_area;
    Q[(size_t)2 * nc + c] = s[M_PY] * inv_area;
    Q[(size_t)3 * nc + c] = s[M_L] * inv_area;
}

// ------------------------------------------------------- pair export (debug)
__global__ __launch_bounds__(256) void pairs_kernel(StepArgs a, int32_t* pl, int32_t* pj,
                                                    unsigned long long* count, long long cap)
{
    const int c = blockIdx.x;
    const int s = a.cell_start[c];
    const int n = a.cell_start[c + 1] - s;
    for (int l = threadIdx.x; l < n; l += 256) {
        const uint32_t xl = a.xi[s + l], yl = a.yi[s + l];
        const float rl = a.r[s + l];
        for (int j = l + 1; j < n; ++j) {
            const int dxi = (int)(a.xi[s + j] - xl), dyi = (int)(a.yi[s + j] - yl);
            float diff, R2;
            screen(dxi, dyi, rl, a.r[s + j], a.qx, a.qy, diff, R2);
            if (!(diff < kGuard * R2)) continue;
            if (!decide(dxi, dyi, rl, a.r[s + j], a)) continue;
            const unsigned long long k = atomicAdd(count, 1ull);
            if ((long long)k < cap) {
                pl[k] = s + l;
                pj[k] = s + j;
            }
        }
    }
}

}  // namespace spdem
