// spdem: superparameterised sea-ice floe DEM for MI355X (gfx950, CDNA4).
//
// Method: Deng, Stechmann & Chen, "Particle-continuum multiscale modeling of
// sea ice floes".  One doubly periodic DEM per coarse cell (Sec. 3.1); the DEM
// system and contact law of Sec. 2.1; cell statistics feeding the moment
// equations of Sec. 2.3; Lax-Friedrichs with the Oseen momentum advection
// (Sec. 3.2).
//
// Layout and schedule:
//   * floe state is SoA in HBM, sorted by cell, updated in place: xi, yi
//     (u32 cell fractions), u, v, w, th, r, h (f32);
//   * one workgroup owns one cell per step: it stages the cell's positions,
//     radii, velocities and spins in LDS, evaluates the ocean and drag in
//     registers, enumerates contact candidates from LDS (all pairs, or square
//     sub-bins of side >= 2 r_max built by an LDS counting sort), records each
//     floe's contacts in an LDS list, then sums the contact forces in
//     ascending partner index (the result does not depend on the candidate
//     order), integrates, writes the floe back and reduces the FP64 cell
//     statistics with wavefront shuffles;
//   * the continuum update is a separate small kernel over the coarse grid.
//
// Contact decision: contact iff |x_j - x_l| < r_l + r_j.  The step screens in
// FP32 and decides pairs within a relative guard band of 2^-19 (far wider than
// the FP32 rounding of the screen) with the FP64 expression
// (dx*dx + dy*dy) < R*R, dx = dxi * (Lx 2^-32), R = r_l + r_j, evaluated
// without contraction, so the contact set is the one the FP64 expression gives.
//
// Precision: positions are fixed point (2^-32 of the cell: < 6e-6 m at 25 km),
// per-contact separation and overlap are FP64 (the overlap d - R cancels),
// forces and the floe state are FP32, cell statistics and the continuum FP64.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/spdem.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMomStride = 16;          // doubles per cell in the statistics buffer (128 B)
constexpr int kListCap = SP_CONTACT_CAP;
constexpr int kMaxBinsSide = 32;
constexpr double kPi = 3.14159265358979323846;
constexpr float kPiF = 3.14159265358979323846f;
constexpr float kGuard = 1.0f / 524288.0f;  // 2^-19

// device fault bits
constexpr uint32_t kErrOverlap = 1u;
constexpr uint32_t kErrNaN = 2u;
constexpr uint32_t kErrCFL = 4u;
constexpr uint32_t kErrCapacity = 8u;

enum { M_N = 0, M_MASS, M_PX, M_PY, M_L, M_UX, M_UY, M_SVX, M_SVY, M_SW, M_AICE, M_UBAR, M_VBAR };

struct Modes {
    float kxL[SP_MAX_MODES];  // kx * Lx: phase per cell fraction
    float kyL[SP_MAX_MODES];
    float au[SP_MAX_MODES];
    float av[SP_MAX_MODES];
    float cz[SP_MAX_MODES];   // curl coefficient av kx - au ky
};

struct StepArgs {
    uint32_t* xi;
    uint32_t* yi;
    float* u;
    float* v;
    float* w;
    float* th;
    const float* r;
    const float* h;
    const int32_t* cell_start;
    const float2* phase;       // [ncells][nmodes]: (sin, cos) of kx Xc + ky Yc + phase at the cell centre
    double* mom;               // [ncells][kMomStride]
    uint32_t* err;
    unsigned long long* contacts;
    int32_t ncells;
    int32_t nmodes;
    int32_t cap;               // LDS floe capacity
    int32_t nbx, nby;          // sub-bins per side (1: all pairs along that axis)
    uint32_t flags;
    float qx, qy;              // Lx 2^-32, Ly 2^-32
    double qxd, qyd;
    double inv_qxd, inv_qyd;
    double dtd;
    double Ed, Gd, mud;
    double cdrho;              // Cd rho_o
    double rho_ice_d;
    float u0, v0;
    Modes modes;
};

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
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

// Block-wide exclusive scan of cnt[0..nb) into start[0..nb], nb <= 4 * kBlock.
__device__ void block_exclusive_scan(const int* cnt, int* start, int nb, int* wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int loc[4];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int b = tid * 4 + k;
        loc[k] = b < nb ? cnt[b] : 0;
        tot += loc[k];
    }
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = 0;
    for (int k = 0; k < wave; ++k) base += wsum[k];
    int run = base + incl - tot;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int b = tid * 4 + k;
        if (b < nb) start[b] = run;
        run += loc[k];
    }
    if (tid == kBlock - 1) start[nb] = run;
    __syncthreads();
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

// Sum over a row of 16 lanes with DPP row shifts (deterministic order); the
// row total lands in the row's last lane.
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, true);
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

// ------------------------------------------------------------ cell kernel
// Statistics reduced by every step.  n, M and A_ice depend only on the radii
// and thicknesses; the statistics kernel writes them when the floes are set.
constexpr int kDyn = 8;
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

// SCHED: 1 all pairs, 2 binned half shell.  STEP: false = statistics of the
// current state only (no contacts, no update, all 11 statistics).
template <int SCHED, bool STEP>
__global__ __launch_bounds__(kBlock) void dem_cell_kernel(StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red11[SP_NMOM][kBlock / 16];
    __shared__ int wsum[kBlock / 64];
    __shared__ unsigned long long csum[kBlock / 64];

    __shared__ float4 mode_k[SP_MAX_MODES];   // kx Lx, ky Ly, au, av
    __shared__ float4 mode_c[SP_MAX_MODES];   // curl coefficient, sin and cos of the centre phase, -

    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int s = a.cell_start[c];
    const int n = a.cell_start[c + 1] - s;
    const int cap = a.cap;

    if (tid < a.nmodes) {
        const float2 sc = a.phase[(size_t)c * a.nmodes + tid];
        mode_k[tid] = make_float4(a.modes.kxL[tid], a.modes.kyL[tid], a.modes.au[tid], a.modes.av[tid]);
        mode_c[tid] = make_float4(a.modes.cz[tid], sc.x, sc.y, 0.0f);
    }
    if (!STEP) __syncthreads();

    uint4* P = reinterpret_cast<uint4*>(smem);                // xi, yi, r bits, -
    float4* V = reinterpret_cast<float4*>(P + cap);           // u, v, w, -
    uint4* S = reinterpret_cast<uint4*>(V + cap);             // sorted copy: xi, yi, r bits, index | bin << 16
    uint16_t* lst = reinterpret_cast<uint16_t*>(S + (SCHED == 2 ? cap : 0));  // [cap][kListCap]
    int* cnt = reinterpret_cast<int*>(lst + (size_t)cap * kListCap);
    int* binof = cnt + cap;
    int* rank = binof + (SCHED == 2 ? cap : 0);
    int* bcnt = rank + (SCHED == 2 ? cap : 0);
    int* bstart = bcnt + (SCHED == 2 ? a.nbx * a.nby : 0);

    if (STEP) {
        for (int i = tid; i < n; i += kBlock) {
            P[i] = make_uint4(a.xi[s + i], a.yi[s + i], __float_as_uint(a.r[s + i]), 0u);
            V[i] = make_float4(a.u[s + i], a.v[s + i], a.w[s + i], 0.0f);
            cnt[i] = 0;
        }
        if (SCHED == 2) {
            const int nb = a.nbx * a.nby;
            for (int b = tid; b < nb; b += kBlock) bcnt[b] = 0;
            __syncthreads();
            for (int i = tid; i < n; i += kBlock) {
                const int bx = (int)__umulhi(P[i].x, (uint32_t)a.nbx);
                const int by = (int)__umulhi(P[i].y, (uint32_t)a.nby);
                const int b = by * a.nbx + bx;
                binof[i] = b;
                rank[i] = atomicAdd(&bcnt[b], 1);
            }
            __syncthreads();
            block_exclusive_scan(bcnt, bstart, nb, wsum);
            for (int i = tid; i < n; i += kBlock) {
                uint4 p = P[i];
                p.w = (uint32_t)i | ((uint32_t)binof[i] << 16);
                S[bstart[binof[i]] + rank[i]] = p;
            }
        }
        __syncthreads();

        // ---- phase 1: contact candidates -> per-floe lists
        if (SCHED == 1) {
            // every floe against every floe (itself included, skipped later);
            // the list comes out in ascending partner order
            for (int l = tid; l < n; l += kBlock) {
                const uint4 pl = P[l];
                const float rl = __uint_as_float(pl.z);
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
            for (int t = tid; t < n; t += kBlock) {
                const uint4 own = S[t];
                const int o = (int)(own.w & 0xffffu);
                const int b = (int)(own.w >> 16);
                const int bx = b % a.nbx, by = b / a.nbx;
                const float rl = __uint_as_float(own.z);
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
    }

    double acc[SP_NMOM];
#pragma unroll
    for (int k = 0; k < SP_NMOM; ++k) acc[k] = 0.0;
    unsigned long long ncontact = 0;

    for (int l = tid; l < n; l += kBlock) {
        uint32_t xl, yl;
        float rl, ul, vl, wl;
        if (STEP) {
            const uint4 pl = P[l];
            const float4 vv = V[l];
            xl = pl.x;
            yl = pl.y;
            rl = __uint_as_float(pl.z);
            ul = vv.x;
            vl = vv.y;
            wl = vv.z;
        } else {
            xl = a.xi[s + l];
            yl = a.yi[s + l];
            rl = a.r[s + l];
            ul = a.u[s + l];
            vl = a.v[s + l];
            wl = a.w[s + l];
        }

        // ---- ocean current and curl at the floe centre (angle addition around
        // the cell centre keeps the FP32 arguments below (|kx| Lx + |ky| Ly) / 2),
        // then drag and drag torque in FP64
        const double rld = (double)rl, uld = (double)ul, vld = (double)vl, wld = (double)wl;
        double fdx = 0.0, fdy = 0.0, tdr = 0.0;
        if (!(a.flags & SP_OCEAN_OFF)) {
            const float fx = (float)(int)(xl - 0x80000000u) * 2.3283064365386963e-10f;
            const float fy = (float)(int)(yl - 0x80000000u) * 2.3283064365386963e-10f;
            float uo = a.u0, vo = a.v0, zeta = 0.0f;
#pragma unroll 2
            for (int m = 0; m < a.nmodes; ++m) {
                const float4 mk = mode_k[m];
                const float4 mc = mode_c[m];
                const float dth = mk.x * fx + mk.y * fy;
                float sd, cd;
                sincos_small(dth, sd, cd);
                const float sn = mc.y * cd + mc.z * sd;    // sin and cos of the full phase
                const float cn = mc.z * cd - mc.y * sd;
                uo += mk.z * sn;
                vo += mk.w * sn;
                zeta += mc.x * cn;
            }
            const double du = (double)uo - uld, dv = (double)vo - vld;
            const double sp = sqrt(du * du + dv * dv);
            const double alpha = a.cdrho * kPi * rld * rld;
            fdx = alpha * du * sp;
            fdy = alpha * dv * sp;
            const double dW = 0.5 * (double)zeta - wld;
            const double r2 = rld * rld;
            const double beta = a.cdrho * kPi * r2 * r2 * rld;
            tdr = beta * dW * fabs(dW);
        }
        const double hld = (double)a.h[s + l];
        const double md = a.rho_ice_d * hld * kPi * rld * rld;

        if (STEP) {
            uint16_t* my = lst + (size_t)l * kListCap;
            int k = cnt[l];
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

            // ---- phase 2: contact forces and torques in ascending partner order (FP64)
            double Fx = fdx, Fy = fdy, T = tdr;
            for (int q = 0; q < k; ++q) {
                const int j = my[q];
                if (j == l) continue;
                const uint4 pj = P[j];
                const int dxi = (int)(pj.x - xl), dyi = (int)(pj.y - yl);
                const float rj = __uint_as_float(pj.z);
                if (!decide(dxi, dyi, rl, rj, a)) continue;
                const double dx = (double)dxi * a.qxd, dy = (double)dyi * a.qyd;
                const double d2 = dx * dx + dy * dy;
                if (!(d2 > 0.0)) {
                    atomicOr(a.err, kErrOverlap);
                    continue;
                }
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
                const float4 vj = V[j];
                const double wjd = (double)vj.z;
                // spin sum in a fixed operand order (lower floe index first) so that
                // the pair forces are exactly antisymmetric
                const double spin = (l < j) ? (wld * rld + wjd * rjd) : (wjd * rjd + wld * rld);
                const double vt = (((double)vj.x - uld) * tx + ((double)vj.y - vld) * ty) - spin;
                const double capf = a.mud * fabs(Fn);
                const double Ft = fmin(fmax(cc * a.Gd * vt, -capf), capf);
                Fx += Fn * nx + Ft * tx;
                Fy += Fn * ny + Ft * ty;
                T += rld * Ft;
                ncontact += (l < j) ? 1ull : 0ull;
            }

            // ---- time update (semi-implicit Euler by default), FP64 arithmetic,
            // FP32 / fixed-point storage
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
            a.xi[s + l] = xl + (uint32_t)sx;
            a.yi[s + l] = yl + (uint32_t)sy;
            a.u[s + l] = un;
            a.v[s + l] = vn;
            a.w[s + l] = wn;
            a.th[s + l] = (float)((double)a.th[s + l] + dt * wx);
            if (!(isfinite(un) && isfinite(vn) && isfinite(wn))) atomicOr(a.err, kErrNaN);
        } else {
            acc[M_N] += 1.0;
            acc[M_MASS] += md;
            acc[M_AICE] += kPi * rld * rld;
        }

        // ---- cell statistics of the pre-step state (FP64)
        acc[M_PX] += md * uld;
        acc[M_PY] += md * vld;
        acc[M_L] += md * rld * rld * wld;
        acc[M_UX] += uld;
        acc[M_UY] += vld;
        acc[M_SVX] += fdx;
        acc[M_SVY] += fdy;
        acc[M_SW] += tdr;
    }

    const int lane = tid & 63;
    if (STEP) {
        // ---- block reduction of the 8 step statistics through LDS: lane
        // partials -> 16 segment sums per quantity -> DPP row sum (fixed order)
        unsigned long long cs = wave_sum_u64(ncontact);
        if (lane == 0) csum[tid >> 6] = cs;
        __syncthreads();   // every lane is done with the cell's LDS data
        double* red = reinterpret_cast<double*>(smem);     // [kDyn][kBlock]
#pragma unroll
        for (int k = 0; k < kDyn; ++k) red[k * kBlock + tid] = acc[dyn_slot(k)];
        __syncthreads();
        if (tid < kDyn * 16) {
            const int k = tid >> 4, seg = tid & 15;
            const double* src = red + k * kBlock + seg * 16;
            double x = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) x += src[i];
            x = row_sum(x);
            if (seg == 15) {
                const int slot = dyn_slot(k);
                a.mom[(size_t)c * kMomStride + slot] = x;
                if (slot == M_UX || slot == M_UY)   // continuum coefficient <v> = U / n
                    a.mom[(size_t)c * kMomStride + (slot == M_UX ? M_UBAR : M_VBAR)] =
                        n > 0 ? x / (double)n : 0.0;
            }
        }
        if (tid == 0) {
            const unsigned long long t = csum[0] + csum[1] + csum[2] + csum[3];
            if (t) atomicAdd(a.contacts, t);
        }
    } else {
        // ---- all 11 statistics: DPP row sums, then 16 row partials per quantity
        const int rowid = tid >> 4;
#pragma unroll
        for (int k = 0; k < SP_NMOM; ++k) {
            const double x = row_sum(acc[k]);
            if ((lane & 15) == 15) red11[k][rowid] = x;
        }
        __syncthreads();
        if (tid < SP_NMOM) {
            double x = red11[tid][0];
#pragma unroll
            for (int q = 1; q < kBlock / 16; ++q) x += red11[tid][q];
            a.mom[(size_t)c * kMomStride + tid] = x;
            if (tid == M_UX || tid == M_UY)
                a.mom[(size_t)c * kMomStride + (tid == M_UX ? M_UBAR : M_VBAR)] = n > 0 ? x / (double)n : 0.0;
        }
    }
}

// ------------------------------------------------------ continuum update
struct LfArgs {
    const double* mom;   // [ncells][kMomStride]
    const double* Q;     // [4][ncells]
    double* Qn;          // [4][ncells]
    unsigned long long* max_cfl_bits;
    uint32_t* err;
    int32_t nx, ny;
    double dT, dX, dY, inv_area;
};

__device__ __forceinline__ double ubar(const double* mom, int c, int f)
{
    return mom[(size_t)c * kMomStride + (f == M_UX ? M_UBAR : M_VBAR)];
}

__global__ __launch_bounds__(64) void lf_kernel(LfArgs a)
{
    const int nc = a.nx * a.ny;
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    double cfl = 0.0;
    if (C < nc) {
        const int ix = C % a.nx, iy = C / a.nx;
        const int E = iy * a.nx + (ix + 1 == a.nx ? 0 : ix + 1);
        const int W = iy * a.nx + (ix == 0 ? a.nx - 1 : ix - 1);
        const int N = (iy + 1 == a.ny ? 0 : iy + 1) * a.nx + ix;
        const int S = (iy == 0 ? a.ny - 1 : iy - 1) * a.nx + ix;
        const double uE = ubar(a.mom, E, M_UX), uW = ubar(a.mom, W, M_UX);
        const double vN = ubar(a.mom, N, M_UY), vS = ubar(a.mom, S, M_UY);
        const double uC = ubar(a.mom, C, M_UX), vC = ubar(a.mom, C, M_UY);
        const double cx = a.dT / (2.0 * a.dX), cy = a.dT / (2.0 * a.dY);
        cfl = fabs(uC) * a.dT / a.dX + fabs(vC) * a.dT / a.dY;
        const double* sC = a.mom + (size_t)C * kMomStride;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double qE = a.Q[(size_t)f * nc + E], qW = a.Q[(size_t)f * nc + W];
            const double qN = a.Q[(size_t)f * nc + N], qS = a.Q[(size_t)f * nc + S];
            const double avg = 0.25 * (qE + qW + qN + qS);
            double q;
            if (f == 0) {
                q = avg - cx * (uE * qE - uW * qW) - cy * (vN * qN - vS * qS);
            } else if (f == 3) {
                q = avg - cx * (uE * qE - uW * qW) - cy * (vN * qN - vS * qS) +
                    a.dT * sC[M_SW] * a.inv_area;
            } else {
                q = avg - a.dT * (uC * (qE - qW) / (2.0 * a.dX) + vC * (qN - qS) / (2.0 * a.dY)) +
                    a.dT * sC[f == 1 ? M_SVX : M_SVY] * a.inv_area;
            }
            a.Qn[(size_t)f * nc + C] = q;
        }
    }
    // wavefront max of the CFL number, one atomic per wavefront
    double x = cfl;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    if ((threadIdx.x & 63) == 0) {
        atomicMax(a.max_cfl_bits, (unsigned long long)__double_as_longlong(x));
        if (x > 1.0) atomicOr(a.err, kErrCFL);
    }
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
__global__ __launch_bounds__(kBlock) void pairs_kernel(StepArgs a, int32_t* pl, int32_t* pj,
                                                       unsigned long long* count, long long cap)
{
    const int c = blockIdx.x;
    const int s = a.cell_start[c];
    const int n = a.cell_start[c + 1] - s;
    for (int l = threadIdx.x; l < n; l += kBlock) {
        const uint32_t xl = a.xi[s + l], yl = a.yi[s + l];
        const float rl = a.r[s + l];
        for (int j = l + 1; j < n; ++j) {
            const int dxi = (int)(a.xi[s + j] - xl), dyi = (int)(a.yi[s + j] - yl);
            float diff, R2;
            screen(dxi, dyi, rl, a.r[s + j], a.qx, a.qy, diff, R2);
            if (!(diff < kGuard * R2)) continue;
            if (!decide(dxi, dyi, rl, a.r[s + j], a)) continue;
            unsigned long long k = atomicAdd(count, 1ull);
            if ((long long)k < cap) {
                pl[k] = s + l;
                pj[k] = s + j;
            }
        }
    }
}

}  // namespace

// =================================================================== host
struct sp_ctx {
    sp_params p;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int device = 0;

    // ocean
    double u0 = 0, v0 = 0;
    int nmodes = 0;
    double kx[SP_MAX_MODES], ky[SP_MAX_MODES], au[SP_MAX_MODES], av[SP_MAX_MODES],
        ph[SP_MAX_MODES];
    bool phase_dirty = true;

    // floes
    int64_t n = 0;
    int32_t ncells = 0;
    int32_t cap = 0;
    int32_t nbx = 1, nby = 1;
    int32_t sched = SP_SCHED_ALLPAIRS;
    bool have_floes = false;
    std::vector<int32_t> start_h;

    // device buffers
    uint32_t *xi = nullptr, *yi = nullptr;
    float *u = nullptr, *v = nullptr, *w = nullptr, *th = nullptr, *r = nullptr, *h = nullptr;
    int32_t* cell_start = nullptr;
    float2* phase = nullptr;
    double* mom = nullptr;    // statistics written by the step
    double* mom2 = nullptr;   // statistics of the current state (read_moments)
    double* Q[2] = {nullptr, nullptr};
    int qcur = 0;
    uint32_t* err_d = nullptr;
    unsigned long long* contacts_d = nullptr;
    unsigned long long* cfl_bits_d = nullptr;
    int64_t steps = 0;
};

namespace {

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

#define HIP_TRY(ctx, expr)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), SP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));            \
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

void free_all(sp_ctx* c)
{
    void* ps[] = {c->xi, c->yi, c->u, c->v, c->w, c->th, c->r, c->h, c->cell_start, c->phase,
                  c->mom, c->mom2, c->Q[0], c->Q[1], c->err_d, c->contacts_d, c->cfl_bits_d};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    c->xi = c->yi = nullptr;
    c->u = c->v = c->w = c->th = c->r = c->h = nullptr;
    c->cell_start = nullptr;
    c->phase = nullptr;
    c->mom = c->mom2 = nullptr;
    c->Q[0] = c->Q[1] = nullptr;
    c->err_d = nullptr;
    c->contacts_d = c->cfl_bits_d = nullptr;
}

size_t lds_bytes(int sched, int cap, int nb)
{
    size_t b = (size_t)cap * (16 + 16 + 2 * kListCap + 4);
    if (sched == SP_SCHED_BINNED) b += (size_t)cap * (16 + 4 + 4) + (size_t)(2 * nb + 1) * 4;
    b = std::max(b, (size_t)kDyn * kBlock * sizeof(double));   // reduction buffer
    return (b + 15) & ~(size_t)15;
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
    a.mom = c->mom;
    a.err = c->err_d;
    a.contacts = c->contacts_d;
    a.ncells = c->ncells;
    a.nmodes = c->nmodes;
    a.cap = c->cap;
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
    a.u0 = (float)c->u0;
    a.v0 = (float)c->v0;
    for (int m = 0; m < c->nmodes; ++m) {
        a.modes.kxL[m] = (float)(c->kx[m] * c->p.cell_lx);
        a.modes.kyL[m] = (float)(c->ky[m] * c->p.cell_ly);
        a.modes.au[m] = (float)c->au[m];
        a.modes.av[m] = (float)c->av[m];
        a.modes.cz[m] = (float)(c->av[m] * c->kx[m] - c->au[m] * c->ky[m]);
    }
    return a;
}

sp_status upload_phase(sp_ctx* c)
{
    if (!c->phase_dirty || c->ncells == 0) return SP_OK;
    const int nm = c->nmodes > 0 ? c->nmodes : 1;
    std::vector<float2> tab((size_t)c->ncells * nm, make_float2(0.0f, 1.0f));
    for (int cell = 0; cell < c->ncells; ++cell) {
        const double Xc = ((double)(cell % c->p.nx) + 0.5) * c->p.cell_lx;
        const double Yc = ((double)(cell / c->p.nx) + 0.5) * c->p.cell_ly;
        for (int m = 0; m < c->nmodes; ++m) {
            const double t = c->kx[m] * Xc + c->ky[m] * Yc + c->ph[m];
            tab[(size_t)cell * nm + m] = make_float2((float)sin(t), (float)cos(t));
        }
    }
    sp_status st = dalloc(c, &c->phase, tab.size());
    if (st) return st;
    HIP_TRY(c, hipMemcpyAsync(c->phase, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->phase_dirty = false;
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
    return fail(c, SP_ECFL, "continuum CFL number exceeded 1");
}

template <class K>
sp_status allow_lds(sp_ctx* c, K kernel, size_t bytes)
{
    if (bytes <= 65536) return SP_OK;
    HIP_TRY(c, hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes));
    return SP_OK;
}

sp_status launch_cell_kernel(sp_ctx* c, const StepArgs& a, bool step)
{
    if (c->ncells == 0) return SP_OK;
    const int nb = c->nbx * c->nby;
    dim3 grid(c->ncells), block(kBlock);
    if (step) {
        sp_status st = c->sched == SP_SCHED_BINNED
                           ? allow_lds(c, dem_cell_kernel<2, true>, lds_bytes(SP_SCHED_BINNED, c->cap, nb))
                           : allow_lds(c, dem_cell_kernel<1, true>, lds_bytes(SP_SCHED_ALLPAIRS, c->cap, 1));
        if (st) return st;
    }
    if (!step) {
        hipLaunchKernelGGL((dem_cell_kernel<1, false>), grid, block, 0, c->stream, a);
    } else if (c->sched == SP_SCHED_BINNED) {
        hipLaunchKernelGGL((dem_cell_kernel<2, true>), grid, block,
                           lds_bytes(SP_SCHED_BINNED, c->cap, nb), c->stream, a);
    } else {
        hipLaunchKernelGGL((dem_cell_kernel<1, true>), grid, block,
                           lds_bytes(SP_SCHED_ALLPAIRS, c->cap, 1), c->stream, a);
    }
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

sp_status reset_continuum(sp_ctx* c)
{
    StepArgs a = make_args(c, 0.0);
    sp_status st = launch_cell_kernel(c, a, false);
    if (st) return st;
    const double inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    hipLaunchKernelGGL(q_from_moments_kernel, dim3((c->ncells + 255) / 256), dim3(256), 0, c->stream,
                       c->mom, c->Q[0], c->ncells, inv_area);
    HIP_TRY(c, hipGetLastError());
    c->qcur = 0;
    return SP_OK;
}

sp_status install_floes(sp_ctx* c, int64_t n, const int32_t* counts)
{
    // host-side validation of the counts; buffers already sized by the caller
    (void)n;
    c->start_h.assign((size_t)c->ncells + 1, 0);
    int32_t mx = 0;
    for (int i = 0; i < c->ncells; ++i) {
        c->start_h[i + 1] = c->start_h[i] + counts[i];
        mx = std::max(mx, counts[i]);
    }
    c->cap = std::max(64, (mx + 63) / 64 * 64);
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
    (void)hipGetDevice(&c->device);
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
    if (!st) st = dalloc(c, &c->contacts_d, 1);
    if (!st) st = dalloc(c, &c->cfl_bits_d, 1);
    if (!st) st = dalloc(c, &c->mom, (size_t)c->ncells * kMomStride);
    if (!st) st = dalloc(c, &c->mom2, (size_t)c->ncells * kMomStride);
    if (!st) st = dalloc(c, &c->Q[0], (size_t)c->ncells * 4);
    if (!st) st = dalloc(c, &c->Q[1], (size_t)c->ncells * 4);
    if (!st && hipMemsetAsync(c->err_d, 0, sizeof(uint32_t), c->stream) != hipSuccess) st = SP_EDEVICE;
    if (!st && hipMemsetAsync(c->contacts_d, 0, 8, c->stream) != hipSuccess) st = SP_EDEVICE;
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
    c->u0 = u0;
    c->v0 = v0;
    c->nmodes = nmodes;
    for (int m = 0; m < nmodes; ++m) {
        c->kx[m] = kx[m];
        c->ky[m] = ky[m];
        c->au[m] = au[m];
        c->av[m] = av[m];
        c->ph[m] = phase[m];
        if (!std::isfinite(kx[m]) || !std::isfinite(ky[m]) || !std::isfinite(au[m]) ||
            !std::isfinite(av[m]) || !std::isfinite(phase[m]))
            return fail(c, SP_EINVAL, "non-finite mode %d", m);
    }
    c->phase_dirty = true;
    return upload_phase(c);
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

    sp_status st = SP_OK;
    const size_t N = (size_t)n;
    if (!st) st = dalloc(c, &c->xi, N);
    if (!st) st = dalloc(c, &c->yi, N);
    if (!st) st = dalloc(c, &c->u, N);
    if (!st) st = dalloc(c, &c->v, N);
    if (!st) st = dalloc(c, &c->w, N);
    if (!st) st = dalloc(c, &c->th, N);
    if (!st) st = dalloc(c, &c->r, N);
    if (!st) st = dalloc(c, &c->h, N);
    if (!st) st = dalloc(c, &c->cell_start, (size_t)c->ncells + 1);
    if (st) return st;
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

    install_floes(c, n, counts);
    HIP_TRY(c, hipMemcpyAsync(c->cell_start, c->start_h.data(), ((size_t)c->ncells + 1) * 4,
                              hipMemcpyHostToDevice, c->stream));
    // sub-bins of side >= 2 r_max
    int bx = n > 0 ? (int)floor(c->p.cell_lx / (2.0 * (double)rmax)) : 1;
    int by = n > 0 ? (int)floor(c->p.cell_ly / (2.0 * (double)rmax)) : 1;
    bx = std::min(bx, kMaxBinsSide);
    by = std::min(by, kMaxBinsSide);
    if (bx < 3) bx = 1;
    if (by < 3) by = 1;
    int sched = c->p.schedule;
    if (sched == SP_SCHED_AUTO) sched = (bx >= 3 && by >= 3) ? SP_SCHED_BINNED : SP_SCHED_ALLPAIRS;
    c->sched = sched;
    if (sched == SP_SCHED_BINNED) {
        c->nbx = bx;
        c->nby = by;
    } else {
        c->nbx = c->nby = 1;
    }
    c->n = n;
    HIP_TRY(c, hipMemsetAsync(c->err_d, 0, 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->contacts_d, 0, 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->cfl_bits_d, 0, 8, c->stream));
    c->steps = 0;
    st = upload_phase(c);
    if (st) return st;
    c->have_floes = true;
    st = reset_continuum(c);
    if (st) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
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

static sp_status sp_step_lf(sp_ctx* c, double dt)
{
    LfArgs la;
    la.mom = c->mom;
    la.max_cfl_bits = c->cfl_bits_d;
    la.err = c->err_d;
    la.nx = c->p.nx;
    la.ny = c->p.ny;
    la.dT = dt;
    la.dX = c->p.cell_lx;
    la.dY = c->p.cell_ly;
    la.inv_area = 1.0 / (c->p.cell_lx * c->p.cell_ly);
    la.Q = c->Q[c->qcur];
    la.Qn = c->Q[c->qcur ^ 1];
    hipLaunchKernelGGL(lf_kernel, dim3((c->ncells + 63) / 64), dim3(64), 0, c->stream, la);
    HIP_TRY(c, hipGetLastError());
    c->qcur ^= 1;
    return SP_OK;
}

sp_status sp_step(sp_ctx* c, double dt, int64_t nsteps)
{
    if (!c) return SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_step before sp_set_floes");
    if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0)
        return fail(c, SP_EINVAL, "dt must be positive and nsteps non-negative");
    sp_status st = upload_phase(c);
    if (st) return st;
    StepArgs a = make_args(c, dt);
    const bool cont = !(c->p.flags & SP_NO_CONTINUUM);
    for (int64_t k = 0; k < nsteps; ++k) {
        st = launch_cell_kernel(c, a, true);
        if (st) return st;
        if (cont) {
            st = sp_step_lf(c, dt);
            if (st) return st;
        }
        c->steps++;
    }
    return SP_OK;
}

sp_status sp_profile_steps(sp_ctx* c, double dt, int64_t nsteps, double* dem_ms, double* lf_ms)
{
    if (!c) return SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_profile_steps before sp_set_floes");
    if (!(dt > 0.0) || nsteps < 1) return fail(c, SP_EINVAL, "dt must be positive and nsteps >= 1");
    const bool cont = !(c->p.flags & SP_NO_CONTINUUM);
    std::vector<hipEvent_t> ev((size_t)nsteps * 3);
    for (auto& e : ev) HIP_TRY(c, hipEventCreate(&e));
    sp_status st = SP_OK;
    for (int64_t k = 0; k < nsteps && !st; ++k) {
        HIP_TRY(c, hipEventRecord(ev[3 * k], c->stream));
        st = launch_cell_kernel(c, make_args(c, dt), true);
        HIP_TRY(c, hipEventRecord(ev[3 * k + 1], c->stream));
        if (!st && cont) st = sp_step_lf(c, dt);
        HIP_TRY(c, hipEventRecord(ev[3 * k + 2], c->stream));
        c->steps++;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double sd = 0, sl = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        float a = 0, b = 0;
        HIP_TRY(c, hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]));
        HIP_TRY(c, hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]));
        sd += a;
        sl += b;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (st) return st;
    if (dem_ms) *dem_ms = sd / (double)nsteps;
    if (lf_ms) *lf_ms = cont ? sl / (double)nsteps : 0.0;
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
        sp_status st = launch_cell_kernel(c, a, false);
        if (st) return st;
        std::vector<double> buf((size_t)nc * kMomStride);
        HIP_TRY(c, hipMemcpyAsync(buf.data(), c->mom2, buf.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < nc; ++i)
            for (int k = 0; k < SP_NMOM; ++k) out[(size_t)i * SP_NMOM + k] = buf[(size_t)i * kMomStride + k];
    } else if (which == SP_MOMENTS_CONTINUUM) {
        std::vector<double> buf((size_t)nc * 4);
        HIP_TRY(c, hipMemcpyAsync(buf.data(), c->Q[c->qcur], buf.size() * 8, hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < nc; ++i)
            for (int f = 0; f < 4; ++f) out[(size_t)i * 4 + f] = buf[(size_t)f * nc + i];
    } else {
        return fail(c, SP_EINVAL, "unknown moments selector %d", which);
    }
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
    if (!c || !count || cap < 0 || (cap > 0 && (!l || !j))) return c ? fail(c, SP_EINVAL, "bad pair buffers") : SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    // first pass counts, second pass stores everything, host sorts
    unsigned long long* cnt_d = nullptr;
    sp_status st = dalloc(c, &cnt_d, 1);
    if (st) return st;
    StepArgs a = make_args(c, 0.0);
    HIP_TRY(c, hipMemsetAsync(cnt_d, 0, 8, c->stream));
    hipLaunchKernelGGL(pairs_kernel, dim3(c->ncells), dim3(kBlock), 0, c->stream, a, (int32_t*)nullptr,
                       (int32_t*)nullptr, cnt_d, 0ll);
    unsigned long long tot = 0;
    HIP_TRY(c, hipMemcpyAsync(&tot, cnt_d, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int32_t *pl = nullptr, *pj = nullptr;
    if (tot > 0) {
        st = dalloc(c, &pl, tot);
        if (!st) st = dalloc(c, &pj, tot);
        if (st) {
            (void)hipFree(cnt_d);
            if (pl) (void)hipFree(pl);
            return st;
        }
        HIP_TRY(c, hipMemsetAsync(cnt_d, 0, 8, c->stream));
        hipLaunchKernelGGL(pairs_kernel, dim3(c->ncells), dim3(kBlock), 0, c->stream, a, pl, pj, cnt_d,
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
    unsigned long long cnt = 0, bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&cnt, c->contacts_d, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&bits, c->cfl_bits_d, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
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

}  // extern "C"
