// Host side of the learned closure (included at the end of spdem.hip, where
// sp_ctx and its helpers are visible): the network object (parameters, Adam
// state, normalisation, workspaces), inference, gradients and training, the
// per-cell feature gather and the (feature, tendency) sampler.
#pragma once

#include "mlp_kernels.h"
#include "train_kernels.h"

namespace spdem {

// ---------------------------------------------------------------------------
// The closure replaces a cell's DEM by a reduced one plus a learned residual.
//
// Reduced DEM.  Without contacts every floe relaxes towards the ocean under
// the quadratic drag laws of Sec. 2.1, dw/dt = -k |w| w for its velocity
// relative to the current (k = C_d rho_o / (rho_ice h)) and likewise for its
// spin relative to the half-curl; that equation has the closed form
// w(t) = w0 / (1 + k |w0| t).  The reduced DEM of a cell is one such body with
// the cell's summed drag: its relative velocity and spin at the time t0 they
// were last taken from the cell's floes, red = (du0_x, du0_y, dW0, t0), relax
// in closed form with the cell's mean-field rates
//     kappa_v = C_d rho_o sum pi r^2 / sum m,   kappa_w / r2m,
//     kappa_w = C_d rho_o sum pi r^5 / sum m,   r2m = sum m r^2 / sum m,
// and give the statistics the continuum update consumes: the coefficient
// <v> = u_o - du and the sources per unit area S_v / A = rho_f kappa_v |du| du,
// S_w / A = rho_f kappa_w |dW| dW, rho_f = sum m / A (u_o, curl at the cell
// centre).  As in the plain method, these do not depend on the continuum state.
//
// Base update (base_cell): the Lax-Friedrichs step of lf_cell with every cell's
// statistics taken from its reduced DEM.  The network adds the rest of the
// plain method's update (the residual), as a function of the features of the
// base-updated state; the residual then acts on the new state, so that a
// relaxation it has learned damps the checkerboard mode the averaging of the
// Lax-Friedrichs step maps to its negative instead of amplifying it.
// ---------------------------------------------------------------------------

// Static data of each cell's floes: desc = (A_ice / A, mean h, r2m, n, mean r,
// mean r^2) as float, mf = (kappa_v, kappa_w, r2m, rho_f) as double.  One
// workgroup per cell (blockIdx.x, or cells[blockIdx.x] with a list),
// fixed-order FP64 sums.
__global__ __launch_bounds__(256) void descriptors_kernel(const int32_t* cells, const int32_t* cell_start,
                                                          const float* r, const float* h, double inv_area,
                                                          double rho_ice, double cdrho, float* desc, double* mf)
{
    __shared__ double part[8][256];
    const int c = cells ? cells[blockIdx.x] : (int)blockIdx.x;
    const int s = cell_start[c], n = cell_start[c + 1] - s;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int l = threadIdx.x; l < n; l += 256) {
        const double rl = r[s + l], hl = h[s + l];
        const double m = hl * rl * rl;   // the mass over rho_ice pi
        acc[0] += 1.0;
        acc[1] += rl * rl;
        acc[2] += rl;
        acc[3] += hl;
        acc[4] += m * rl * rl;
        acc[5] += m;
        acc[6] += rl * rl * rl * rl * rl;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) part[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 8; ++k) part[k][threadIdx.x] += part[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nn = part[0][0], hm = part[5][0];
        const double r2m = hm > 0 ? part[4][0] / hm : 0.0;
        float* d = desc + (size_t)c * 6;
        d[0] = (float)(kPi * part[1][0] * inv_area);
        d[1] = nn > 0 ? (float)(part[3][0] / nn) : 0.0f;
        d[2] = (float)r2m;
        d[3] = (float)nn;
        d[4] = nn > 0 ? (float)(part[2][0] / nn) : 0.0f;
        d[5] = nn > 0 ? (float)(part[1][0] / nn) : 0.0f;
        double* q = mf + (size_t)c * 4;
        // sum m = rho_ice pi sum h r^2
        q[0] = hm > 0 ? cdrho * part[1][0] / (rho_ice * hm) : 0.0;
        q[1] = hm > 0 ? cdrho * part[6][0] / (rho_ice * hm) : 0.0;
        q[2] = r2m;
        q[3] = rho_ice * kPi * hm * inv_area;
    }
}

struct CellOcean {
    double u, v, zeta;
};

// Ocean current and curl at the centre of cell C (from its phase table).
__device__ __forceinline__ CellOcean ocean_centre(int C, const double2* phase, int nmodes, const Modes& modes,
                                                  double u0, double v0)
{
    CellOcean o{u0, v0, 0.0};
    for (int m = 0; m < nmodes; ++m) {
        const double2 sc = phase[(size_t)C * nmodes + m];
        o.u += modes.au[m] * sc.x;
        o.v += modes.av[m] * sc.x;
        o.zeta += modes.cz[m] * sc.y;
    }
    return o;
}

// Ocean current and curl at every cell centre, kept for the closure kernels
// (the ocean is steady: computed once per ocean or grid change).
__global__ void ocean_centre_kernel(int ncells, const double2* phase, int nmodes, Modes modes, double u0, double v0,
                                    double* oc)
{
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= ncells) return;
    const CellOcean o = ocean_centre(C, phase, nmodes, modes, u0, v0);
    reinterpret_cast<double4*>(oc)[C] = make_double4(o.u, o.v, o.zeta, 0.0);
}

// Relative velocity and spin of cell C's reduced DEM at time t.
__device__ __forceinline__ void reduced_rel(int C, const double* red, const double* mf, double t, double& dux,
                                            double& duy, double& dw)
{
    const double* q = red + (size_t)C * 4;
    const double* k = mf + (size_t)C * 4;
    const double tr = t > q[3] ? t - q[3] : 0.0;
    const double fu = 1.0 / (1.0 + k[0] * sqrt(q[0] * q[0] + q[1] * q[1]) * tr);
    dux = q[0] * fu;
    duy = q[1] * fu;
    const double kw = k[2] > 0.0 ? k[1] / k[2] : 0.0;
    dw = q[2] / (1.0 + kw * fabs(q[2]) * tr);
}

// Statistics of cell C's reduced DEM at time t: coefficient (u, v), sources
// per unit area (s_x, s_y, s_w).
__device__ __forceinline__ CellOcean centre_of(int C, const double* oc)
{
    const double4 q = reinterpret_cast<const double4*>(oc)[C];
    return CellOcean{q.x, q.y, q.z};
}

__device__ __forceinline__ void reduced_stats(int C, const double* red, const double* mf, const double* oc, double t,
                                              double out[5])
{
    const CellOcean o = centre_of(C, oc);
    double dux, duy, dw;
    reduced_rel(C, red, mf, t, dux, duy, dw);
    const double* k = mf + (size_t)C * 4;
    const double sp = sqrt(dux * dux + duy * duy);
    out[0] = o.u - dux;
    out[1] = o.v - duy;
    out[2] = k[3] * k[0] * sp * dux;
    out[3] = k[3] * k[0] * sp * duy;
    out[4] = k[3] * k[1] * fabs(dw) * dw;
}

struct ClosureArgs {
    const double* red;
    const double* mf;
    const double* oc;   // [ncells][4]: ocean u, v, curl at each cell centre (ocean_centre_kernel)
    int nx, ny;
    double dX, dY;
    double t;       // time of the pre-step state
    const double* rs;   // [ncells][5] reduced_stats of every cell at t, or null: computed where needed
};

// The base update of cell C (lf_cell with the reduced DEM statistics of every cell).
__device__ __forceinline__ void cell_rstats(int C, const ClosureArgs& a, double out[5])
{
    if (a.rs) {
#pragma unroll
        for (int k = 0; k < 5; ++k) out[k] = a.rs[(size_t)C * 5 + k];
    } else {
        reduced_stats(C, a.red, a.mf, a.oc, a.t, out);
    }
}

__device__ __forceinline__ void base_cell(int C, const double* Q, const ClosureArgs& a, double dT, double out[4])
{
    const int nx = a.nx, ny = a.ny, nc = nx * ny;
    const int ix = C % nx, iy = C / nx;
    const int E = iy * nx + (ix + 1 == nx ? 0 : ix + 1);
    const int W = iy * nx + (ix == 0 ? nx - 1 : ix - 1);
    const int N = (iy + 1 == ny ? 0 : iy + 1) * nx + ix;
    const int S = (iy == 0 ? ny - 1 : iy - 1) * nx + ix;
    double sC[5], sE[5], sW[5], sN[5], sS[5];
    cell_rstats(C, a, sC);
    cell_rstats(E, a, sE);
    cell_rstats(W, a, sW);
    cell_rstats(N, a, sN);
    cell_rstats(S, a, sS);
    const double cx = dT / (2.0 * a.dX), cy = dT / (2.0 * a.dY);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const double qE = Q[(size_t)f * nc + E], qW = Q[(size_t)f * nc + W];
        const double qN = Q[(size_t)f * nc + N], qS = Q[(size_t)f * nc + S];
        const double avg = 0.25 * (qE + qW + qN + qS);
        if (f == 0 || f == 3)
            out[f] = avg - cx * (sE[0] * qE - sW[0] * qW) - cy * (sN[1] * qN - sS[1] * qS) + (f == 3 ? dT * sC[4] : 0.0);
        else
            out[f] = avg - dT * (sC[0] * (qE - qW) / (2.0 * a.dX) + sC[1] * (qN - qS) / (2.0 * a.dY)) +
                     dT * sC[f == 1 ? 2 : 3];
    }
}

// Base-updated state of every cell: Qb [4][nc].
// The reduced DEM statistics of every cell at a.t (a.rs must be null).
// Every cell's reduced statistics into rs; with row and mom, a closure cell
// (row[C] >= 0) also writes its coefficient <v> into its statistics row of mom,
// which its DEM neighbours' continuum stencils read.
__global__ void reduced_stats_kernel(ClosureArgs a, double* rs, const int32_t* row = nullptr,
                                     double* mom = nullptr)
{
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    if (C >= a.nx * a.ny) return;
    double o[5];
    reduced_stats(C, a.red, a.mf, a.oc, a.t, o);
#pragma unroll
    for (int k = 0; k < 5; ++k) rs[(size_t)C * 5 + k] = o[k];
    if (mom && row[C] >= 0) {
        mom[(size_t)C * kMomStride + M_UBAR] = o[0];
        mom[(size_t)C * kMomStride + M_VBAR] = o[1];
    }
}

__global__ void base_kernel(const double* Q, double* Qb, ClosureArgs a, double dT)
{
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = a.nx * a.ny;
    if (C >= nc) return;
    double o[4];
    base_cell(C, Q, a, dT, o);
#pragma unroll
    for (int f = 0; f < 4; ++f) Qb[(size_t)f * nc + C] = o[f];
}

// Reduced DEM of the listed cells (all cells with a null list) taken from
// their floes' statistics `mom` at time t: velocity U / n, spin L / (M r2m).
// Cells whose status entry is RS_INVALID (when a status array is given) keep
// their reduced DEM.
__global__ void reduced_init_kernel(const int32_t* cells, int ncl, const int32_t* status, const double* mom,
                                    ClosureArgs a, double* red)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    if (status && status[i] == 2) return;
    const int C = cells ? cells[i] : i;
    const double* s = mom + (size_t)C * kMomStride;
    const double n = s[M_N], M = s[M_MASS], r2m = a.mf[(size_t)C * 4 + 2];
    const double U = n > 0.0 ? s[M_UX] / n : 0.0, V = n > 0.0 ? s[M_UY] / n : 0.0;
    const double Om = (M > 0.0 && r2m > 0.0) ? s[M_L] / (M * r2m) : 0.0;
    const CellOcean o = centre_of(C, a.oc);
    double* q = red + (size_t)C * 4;
    q[0] = o.u - U;
    q[1] = o.v - V;
    q[2] = 0.5 * o.zeta - Om;
    q[3] = a.t;
}

// The 45 closure inputs of cell C into o: the continuum state Q (rho, P_x, P_y,
// P_w) on the 3 x 3 neighbourhood (row by row from the south-west, periodic),
// the ocean current and curl at the cell centre, A_ice / A, mean h, r2m, and
// the reduced DEM's relative velocity and spin at time t.
__device__ __forceinline__ void cell_features(int c, const double* Q, const ClosureArgs& a, const float* desc,
                                              float* o)
{
    const int nx = a.nx, ny = a.ny, nc = nx * ny;
    const int ix = c % nx, iy = c / nx;
    int k = 0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = (iy + dy + ny) % ny;
        for (int dx = -1; dx <= 1; ++dx) {
            const int nb = yy * nx + (ix + dx + nx) % nx;
#pragma unroll
            for (int f = 0; f < 4; ++f) o[k++] = (float)Q[(size_t)f * nc + nb];
        }
    }
    const CellOcean oc = centre_of(c, a.oc);
    o[36] = (float)oc.u;
    o[37] = (float)oc.v;
    o[38] = (float)oc.zeta;
    o[39] = desc[(size_t)c * 6 + 0];
    o[40] = desc[(size_t)c * 6 + 1];
    o[41] = desc[(size_t)c * 6 + 2];
    double dux, duy, dw;
    reduced_rel(c, a.red, a.mf, a.t, dux, duy, dw);
    o[42] = (float)dux;
    o[43] = (float)duy;
    o[44] = (float)dw;
}

// Features of every cell (cells == null) or of the listed cells into
// consecutive rows of x.
// One row per thread (blocks of at most 128 threads): the rows are built in
// LDS and the block's contiguous span of x is written coalesced.
__global__ __launch_bounds__(128) void features_kernel(const int32_t* cells, int ncl, const double* Q, ClosureArgs a,
                                                       const float* desc, float* x)
{
    __shared__ float tile[128 * spmlp::kIn];
    const int i0 = blockIdx.x * blockDim.x;
    const int i = i0 + threadIdx.x;
    if (i < ncl) cell_features(cells ? cells[i] : i, Q, a, desc, tile + threadIdx.x * spmlp::kIn);
    __syncthreads();
    const int rows = min((int)blockDim.x, ncl - i0);
    for (int e = threadIdx.x; e < rows * spmlp::kIn; e += blockDim.x) x[(size_t)i0 * spmlp::kIn + e] = tile[e];
}

// (Q_now - Q_ref) / dt per cell, [nc][4] FP32.
__global__ void tendency_kernel(const double* Qnow, const double* Qref, int nc, double dt, float* t)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
#pragma unroll
    for (int f = 0; f < 4; ++f)
        t[(size_t)c * 4 + f] = (float)((Qnow[(size_t)f * nc + c] - Qref[(size_t)f * nc + c]) / dt);
}

// Per-column mean and standard deviation of X [n][cols] (FP64, fixed order).
__global__ __launch_bounds__(256) void column_stats_kernel(const float* X, long n, int cols, float* mean,
                                                           float* inv_std, float* stdv)
{
    __shared__ double part[256];
    __shared__ double mu;
    const int col = blockIdx.x;
    double s = 0.0;
    for (long i = threadIdx.x; i < n; i += 256) s += (double)X[i * cols + col];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) mu = n > 0 ? part[0] / (double)n : 0.0;
    __syncthreads();
    double q = 0.0;
    for (long i = threadIdx.x; i < n; i += 256) {
        const double e = (double)X[i * cols + col] - mu;
        q += e * e;
    }
    part[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sd = n > 1 ? sqrt(part[0] / (double)n) : 0.0;
        mean[col] = (float)mu;
        // a constant column carries no information: it is zeroed (inputs) or left unscaled (outputs)
        const bool flat = !(sd > 1e-12 * (fabs(mu) + 1e-30));
        if (inv_std) inv_std[col] = flat ? 0.0f : (float)(1.0 / sd);
        if (stdv) stdv[col] = flat ? 1.0f : (float)sd;
    }
}

}  // namespace spdem

struct sp_mlp {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cus = 256;           // compute units of the device (grid of the fused forward)
    std::string err;
    float* theta = nullptr;      // FP32 master parameters
    uint16_t* theta_h = nullptr; // bfloat16 copy read by the matrix products
    unsigned char* wsw = nullptr; // LDS image of the fused forward (kFwdLds bytes: weight tiles, biases, norm)
    bool wsw_stale = true;        // parameters or normalisation changed since wsw was made
    float* m = nullptr;          // Adam moments
    float* v = nullptr;
    float* grad = nullptr;
    int64_t adam_t = 0;
    // normalisation: x_n = (x - x_mean) x_inv_std; y = y_n y_std + y_mean
    float* norm = nullptr;       // [x_mean 45 | x_inv_std 45 | y_mean 4 | y_inv_std 4 | y_std 4]
    float* loss_d = nullptr;
    // fused training step: two LDS images (current weights, the next step's), per-batch scratch
    unsigned char* timg[2] = {nullptr, nullptr};
    int tcur = 0;
    bool timg_stale = true;      // parameters or normalisation changed outside the fused step
    int64_t tr_rows = 0;         // padded batch the scratch holds
    uint16_t* tr_aT = nullptr;
    uint16_t* tr_dT = nullptr;
    float* tr_bpart = nullptr;
    double* tr_lpart = nullptr;
    float* epoch_loss = nullptr; // per-batch losses of sp_mlp_train_epoch
    int64_t epoch_cap = 0;
    // input noise of training steps (sp_mlp_set_input_noise) and the noisy
    // copy of the rows a call's steps read
    int noise_n = 0;
    uint64_t noise_seed = 0;
    float noise_sd[spmlp::kIn] = {};
    float* aug_x = nullptr;
    float* aug_t = nullptr;
    int64_t aug_cap = 0;
};

namespace {

using namespace spmlp;

sp_status mfail(sp_mlp* m, sp_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (m) m->err = buf;
    return st;
}

#define MLP_HIP(mm, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (void)hipGetLastError();                                                          \
            return mfail((mm), SP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
        }                                                                                     \
    } while (0)

template <class T>
sp_status malloc_m(sp_mlp* mm, T** p, size_t count)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, std::max<size_t>(1, count) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return mfail(mm, SP_ENOMEM, "hipMalloc(%zu): %s", count * sizeof(T), hipGetErrorString(e));
    }
    return SP_OK;
}

// Inference forward pass of M rows in one fused launch (no scratch, nothing
// kept), on `stream`.
sp_status mlp_infer(sp_mlp* mm, const float* x, int64_t M, float* y, hipStream_t stream)
{
    if (M <= 0) return SP_OK;
    if (mm->wsw_stale) {
        hipLaunchKernelGGL(stage_forward_kernel, dim3((kFwdStageThreads + 255) / 256), dim3(256), 0, stream,
                           mm->theta_h, mm->theta, mm->norm, mm->wsw);
        MLP_HIP(mm, hipGetLastError());
        mm->wsw_stale = false;
    }
    const int64_t per_block = (int64_t)kFwdWaves * 16;
    const int64_t blocks = std::min<int64_t>((M + per_block - 1) / per_block, 2 * (int64_t)mm->num_cus);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(64 * kFwdWaves), kFwdLds, stream, x,
                       (long)M, mm->wsw, y);
    MLP_HIP(mm, hipGetLastError());
    return SP_OK;
}

// Scratch of the fused training step for a batch of B rows (padded to a
// multiple of kTrRowAlign); the deltas start zeroed (the output deltas use 4
// of their 16 rows, the rest stay zero).
sp_status ensure_train(sp_mlp* mm, int B, int* Bp_out)
{
    const int Bp = (B + kTrRowAlign - 1) / kTrRowAlign * kTrRowAlign;
    *Bp_out = Bp;
    if (Bp <= mm->tr_rows) return SP_OK;
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    const size_t P = (size_t)Bp;
    sp_status st = malloc_m(mm, &mm->tr_aT, P * kTrARows);
    if (!st) st = malloc_m(mm, &mm->tr_dT, P * kTrDRows);
    if (!st) st = malloc_m(mm, &mm->tr_bpart, P / 16 * kTrBias);
    if (!st) st = malloc_m(mm, &mm->tr_lpart, P / 16);
    if (st) {
        mm->tr_rows = 0;
        return st;
    }
    MLP_HIP(mm, hipMemsetAsync(mm->tr_dT, 0, P * kTrDRows * 2, mm->stream));
    mm->tr_rows = Bp;
    return SP_OK;
}

// The noisy copy of n training rows (gathered by `rows` if not null) for the
// next Adam steps (step s = the number of steps taken before it), `batch`
// rows per step; *X, *T then point at the copy.
sp_status augment_rows(sp_mlp* mm, const float** X, const float** T, const int32_t* rows, int64_t n, int batch)
{
    if (n > mm->aug_cap) {
        MLP_HIP(mm, hipStreamSynchronize(mm->stream));
        SP_TRY(malloc_m(mm, &mm->aug_x, (size_t)n * kIn));
        SP_TRY(malloc_m(mm, &mm->aug_t, (size_t)n * kOut));
        mm->aug_cap = n;
    }
    NoiseArgs na;
    memset(&na, 0, sizeof na);
    na.n = mm->noise_n;
    na.seed = mm->noise_seed;
    for (int f = 0; f < mm->noise_n; ++f) na.sd[f] = mm->noise_sd[f];
    hipLaunchKernelGGL(tr_augment_kernel, dim3((unsigned)((n * 24 + 255) / 256)), dim3(256), 0, mm->stream, *X, *T, rows,
                       (long)n, (long long)mm->adam_t, batch, na, mm->aug_x, mm->aug_t);
    MLP_HIP(mm, hipGetLastError());
    *X = mm->aug_x;
    *T = mm->aug_t;
    return SP_OK;
}

// One fused step on B rows (gathered by `rows` if not null): the gradient into
// mm->grad (adam false), or an Adam step at rate lr; the summed squared error
// into *loss_d (device).
sp_status fused_step(sp_mlp* mm, const float* X, const float* T, const int32_t* rows, int B, bool adam, float lr,
                     float* loss_d)
{
    int Bp = 0;
    SP_TRY(ensure_train(mm, B, &Bp));
    if (mm->timg_stale) {
        for (int b = 0; b < 2; ++b) {
            hipLaunchKernelGGL(tr_stage_kernel, dim3((kTrStageThreads + 255) / 256), dim3(256), 0, mm->stream,
                               mm->theta_h, mm->theta, mm->norm, mm->timg[b]);
            MLP_HIP(mm, hipGetLastError());
        }
        mm->tcur = 0;
        mm->timg_stale = false;
    }
    TrainArgs ta;
    ta.X = X;
    ta.T = T;
    ta.rows = rows;
    ta.B = B;
    ta.Bp = Bp;
    ta.img = mm->timg[mm->tcur];
    ta.aT = mm->tr_aT;
    ta.dT = mm->tr_dT;
    ta.bpart = mm->tr_bpart;
    ta.lpart = mm->tr_lpart;
    hipLaunchKernelGGL(tr_rows_kernel, dim3((unsigned)(Bp / 16)), dim3(64 * kTrSplit), kTrLdsAll, mm->stream,
                       ta);
    MLP_HIP(mm, hipGetLastError());
    GradArgs ga;
    memset(&ga, 0, sizeof ga);
    ga.aT = mm->tr_aT;
    ga.dT = mm->tr_dT;
    ga.bpart = mm->tr_bpart;
    ga.lpart = mm->tr_lpart;
    ga.ntile = Bp / 16;
    ga.Bp = Bp;
    ga.loss = loss_d;
    if (adam) {
        mm->adam_t++;
        const double b1 = 0.9, b2 = 0.999;
        ga.theta = mm->theta;
        ga.m = mm->m;
        ga.v = mm->v;
        ga.theta_h = mm->theta_h;
        ga.img_next = mm->timg[mm->tcur ^ 1];
        ga.lr = lr;
        ga.b1 = (float)b1;
        ga.b2 = (float)b2;
        ga.eps = 1e-8f;
        ga.c1 = (float)(1.0 - pow(b1, (double)mm->adam_t));
        ga.c2 = (float)(1.0 - pow(b2, (double)mm->adam_t));
    } else {
        ga.grad = mm->grad;
    }
    hipLaunchKernelGGL(tr_grad_kernel, dim3(kTrGradTiles), dim3(64 * kTrGradWaves), 0, mm->stream, ga);
    MLP_HIP(mm, hipGetLastError());
    if (adam) {
        mm->tcur ^= 1;
        mm->wsw_stale = true;   // the inference image follows the new weights when next used
    }
    return SP_OK;
}

}  // namespace

extern "C" {

sp_status sp_mlp_create(void* stream, sp_mlp** out)
{
    if (!out) return SP_EINVAL;
    *out = nullptr;
    sp_mlp* mm = new sp_mlp();
    if (stream) {
        mm->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&mm->stream, hipStreamNonBlocking) != hipSuccess) {
            delete mm;
            return SP_EDEVICE;
        }
        mm->own_stream = true;
    }
    sp_status st = SP_OK;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        mm->num_cus = cus;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(mlp_forward_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFwdLds) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(tr_rows_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kTrLdsAll) != hipSuccess)
        st = SP_EDEVICE;
    if (!st) st = malloc_m(mm, &mm->theta, kNParams);
    if (!st) st = malloc_m(mm, &mm->theta_h, kNParams);
    if (!st) st = malloc_m(mm, &mm->wsw, kFwdLds);
    if (!st) st = malloc_m(mm, &mm->timg[0], kTrLds);
    if (!st) st = malloc_m(mm, &mm->timg[1], kTrLds);
    if (!st) st = malloc_m(mm, &mm->m, kNParams);
    if (!st) st = malloc_m(mm, &mm->v, kNParams);
    if (!st) st = malloc_m(mm, &mm->grad, kNParams);
    if (!st) st = malloc_m(mm, &mm->norm, 2 * kIn + 3 * kOut);
    if (!st) st = malloc_m(mm, &mm->loss_d, 1);
    if (!st) {
        std::vector<float> nrm(2 * kIn + 3 * kOut, 0.0f);
        for (int i = 0; i < kIn; ++i) nrm[kIn + i] = 1.0f;
        for (int i = 0; i < kOut; ++i) nrm[2 * kIn + kOut + i] = nrm[2 * kIn + 2 * kOut + i] = 1.0f;
        if (hipMemcpy(mm->norm, nrm.data(), nrm.size() * 4, hipMemcpyHostToDevice) != hipSuccess) st = SP_EDEVICE;
        if (!st && hipMemset(mm->theta, 0, kNParams * 4) != hipSuccess) st = SP_EDEVICE;
        if (!st && hipMemset(mm->theta_h, 0, kNParams * 2) != hipSuccess) st = SP_EDEVICE;
        if (!st && hipMemset(mm->m, 0, kNParams * 4) != hipSuccess) st = SP_EDEVICE;
        if (!st && hipMemset(mm->v, 0, kNParams * 4) != hipSuccess) st = SP_EDEVICE;
    }
    if (st) {
        sp_mlp_destroy(mm);
        return st;
    }
    *out = mm;
    return SP_OK;
}

void sp_mlp_destroy(sp_mlp* mm)
{
    if (!mm) return;
    if (mm->stream) (void)hipStreamSynchronize(mm->stream);
    void* ps[] = {mm->theta, mm->theta_h, mm->wsw, mm->m, mm->v, mm->grad, mm->norm, mm->loss_d, mm->timg[0],
                  mm->timg[1], mm->tr_aT, mm->tr_dT, mm->tr_bpart, mm->tr_lpart, mm->epoch_loss,
                  mm->aug_x, mm->aug_t};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (mm->own_stream && mm->stream) (void)hipStreamDestroy(mm->stream);
    delete mm;
}

const char* sp_mlp_last_error(const sp_mlp* mm) { return mm ? mm->err.c_str() : "null network"; }

sp_status sp_mlp_set_params(sp_mlp* mm, const float* params)
{
    if (!mm || !params) return mm ? mfail(mm, SP_EINVAL, "null parameters") : SP_EINVAL;
    for (int i = 0; i < kNParams; ++i)
        if (!std::isfinite(params[i])) return mfail(mm, SP_EINVAL, "non-finite parameter %d", i);
    MLP_HIP(mm, hipMemcpyAsync(mm->theta, params, kNParams * 4, hipMemcpyHostToDevice, mm->stream));
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, mm->stream, mm->theta, kNParams,
                       mm->theta_h);
    mm->wsw_stale = true;
    mm->timg_stale = true;
    MLP_HIP(mm, hipGetLastError());
    MLP_HIP(mm, hipMemsetAsync(mm->m, 0, kNParams * 4, mm->stream));
    MLP_HIP(mm, hipMemsetAsync(mm->v, 0, kNParams * 4, mm->stream));
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    mm->adam_t = 0;
    return SP_OK;
}

sp_status sp_mlp_get_params(sp_mlp* mm, float* params)
{
    if (!mm || !params) return mm ? mfail(mm, SP_EINVAL, "null output") : SP_EINVAL;
    MLP_HIP(mm, hipMemcpyAsync(params, mm->theta, kNParams * 4, hipMemcpyDeviceToHost, mm->stream));
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    return SP_OK;
}

sp_status sp_mlp_set_norm(sp_mlp* mm, const float* x_mean, const float* x_std, const float* y_mean,
                          const float* y_std)
{
    if (!mm || !x_mean || !x_std || !y_mean || !y_std) return mm ? mfail(mm, SP_EINVAL, "null arrays") : SP_EINVAL;
    std::vector<float> nrm(2 * kIn + 3 * kOut);
    for (int i = 0; i < kIn; ++i) {
        nrm[i] = x_mean[i];
        nrm[kIn + i] = x_std[i] > 0.0f ? 1.0f / x_std[i] : 0.0f;
    }
    for (int i = 0; i < kOut; ++i) {
        if (!(y_std[i] > 0.0f)) return mfail(mm, SP_EINVAL, "output scale %d not positive", i);
        nrm[2 * kIn + i] = y_mean[i];
        nrm[2 * kIn + kOut + i] = 1.0f / y_std[i];
        nrm[2 * kIn + 2 * kOut + i] = y_std[i];
    }
    MLP_HIP(mm, hipMemcpyAsync(mm->norm, nrm.data(), nrm.size() * 4, hipMemcpyHostToDevice, mm->stream));
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    mm->wsw_stale = true;
    mm->timg_stale = true;
    return SP_OK;
}

sp_status sp_mlp_get_norm(sp_mlp* mm, float* x_mean, float* x_inv_std, float* y_mean, float* y_std)
{
    if (!mm) return SP_EINVAL;
    std::vector<float> nrm(2 * kIn + 3 * kOut);
    MLP_HIP(mm, hipMemcpyAsync(nrm.data(), mm->norm, nrm.size() * 4, hipMemcpyDeviceToHost, mm->stream));
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    for (int i = 0; i < kIn; ++i) {
        if (x_mean) x_mean[i] = nrm[i];
        if (x_inv_std) x_inv_std[i] = nrm[kIn + i];
    }
    for (int i = 0; i < kOut; ++i) {
        if (y_mean) y_mean[i] = nrm[2 * kIn + i];
        if (y_std) y_std[i] = nrm[2 * kIn + 2 * kOut + i];
    }
    return SP_OK;
}

sp_status sp_mlp_fit_norm(sp_mlp* mm, const float* X, const float* T, int64_t n)
{
    if (!mm || !X || !T || n < 2) return mm ? mfail(mm, SP_EINVAL, "need device data and n >= 2") : SP_EINVAL;
    hipLaunchKernelGGL(column_stats_kernel, dim3(kIn), dim3(256), 0, mm->stream, X, (long)n, kIn, mm->norm,
                       mm->norm + kIn, (float*)nullptr);
    MLP_HIP(mm, hipGetLastError());
    hipLaunchKernelGGL(column_stats_kernel, dim3(kOut), dim3(256), 0, mm->stream, T, (long)n, kOut,
                       mm->norm + 2 * kIn, mm->norm + 2 * kIn + kOut, mm->norm + 2 * kIn + 2 * kOut);
    MLP_HIP(mm, hipGetLastError());
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    // outputs with no spread keep unit scale (inv_std = 1 / 1)
    std::vector<float> nrm(2 * kIn + 3 * kOut);
    MLP_HIP(mm, hipMemcpy(nrm.data(), mm->norm, nrm.size() * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < kOut; ++i)
        if (nrm[2 * kIn + kOut + i] == 0.0f) nrm[2 * kIn + kOut + i] = 1.0f;
    MLP_HIP(mm, hipMemcpy(mm->norm, nrm.data(), nrm.size() * 4, hipMemcpyHostToDevice));
    mm->wsw_stale = true;
    mm->timg_stale = true;
    return SP_OK;
}

sp_status sp_mlp_forward(sp_mlp* mm, const float* x, int64_t M, float* y)
{
    if (!mm || (M > 0 && (!x || !y)) || M < 0 || M > INT32_MAX / kHid)
        return mm ? mfail(mm, SP_EINVAL, "bad forward arguments") : SP_EINVAL;
    if (M == 0) return SP_OK;
    return mlp_infer(mm, x, M, y, mm->stream);
}

sp_status sp_mlp_gradient(sp_mlp* mm, const float* X, const float* T, int32_t B, float* grad_host, float* loss)
{
    if (!mm || !X || !T || B < 1 || !grad_host) return mm ? mfail(mm, SP_EINVAL, "bad gradient arguments") : SP_EINVAL;
    SP_TRY(fused_step(mm, X, T, nullptr, B, false, 0.0f, mm->loss_d));
    MLP_HIP(mm, hipMemcpyAsync(grad_host, mm->grad, kNParams * 4, hipMemcpyDeviceToHost, mm->stream));
    float ls = 0.0f;
    MLP_HIP(mm, hipMemcpyAsync(&ls, mm->loss_d, 4, hipMemcpyDeviceToHost, mm->stream));
    MLP_HIP(mm, hipStreamSynchronize(mm->stream));
    if (loss) *loss = ls / (float)(B * kOut);
    return SP_OK;
}

sp_status sp_mlp_train_step(sp_mlp* mm, const float* X, const float* T, const int32_t* rows, int32_t B, float lr,
                            float* loss)
{
    if (!mm || !X || !T || B < 1 || !(lr > 0)) return mm ? mfail(mm, SP_EINVAL, "bad training arguments") : SP_EINVAL;
    if (mm->noise_n > 0) {
        SP_TRY(augment_rows(mm, &X, &T, rows, B, B));
        rows = nullptr;
    }
    SP_TRY(fused_step(mm, X, T, rows, B, true, lr, mm->loss_d));
    if (loss) {
        float ls = 0.0f;
        MLP_HIP(mm, hipMemcpyAsync(&ls, mm->loss_d, 4, hipMemcpyDeviceToHost, mm->stream));
        MLP_HIP(mm, hipStreamSynchronize(mm->stream));
        *loss = ls / (float)(B * kOut);
    }
    return SP_OK;
}

sp_status sp_mlp_set_input_noise(sp_mlp* mm, int32_t nfeat, const float* sd, uint64_t seed)
{
    if (!mm) return SP_EINVAL;
    if (nfeat < 0 || nfeat > kIn || (nfeat > 0 && !sd)) return mfail(mm, SP_EINVAL, "bad input noise arguments");
    for (int f = 0; f < nfeat; ++f)
        if (!(sd[f] >= 0.0f) || !std::isfinite(sd[f])) return mfail(mm, SP_EINVAL, "noise scale of input %d", f);
    mm->noise_n = nfeat;
    mm->noise_seed = seed;
    for (int f = 0; f < kIn; ++f) mm->noise_sd[f] = f < nfeat ? sd[f] : 0.0f;
    return SP_OK;
}

sp_status sp_mlp_train_epoch(sp_mlp* mm, const float* X, const float* T, const int32_t* perm, int64_t n,
                             int32_t batch, float lr, float* mean_loss)
{
    if (!mm || !X || !T || !perm || n < 1 || batch < 1 || !(lr > 0))
        return mm ? mfail(mm, SP_EINVAL, "bad epoch arguments") : SP_EINVAL;
    const int64_t nb = n / batch;   // full batches only
    std::vector<float> losses;
    if (nb > mm->epoch_cap) {
        MLP_HIP(mm, hipStreamSynchronize(mm->stream));
        SP_TRY(malloc_m(mm, &mm->epoch_loss, (size_t)nb));
        mm->epoch_cap = nb;
    }
    float* const lbuf = mm->epoch_loss;
    sp_status st = SP_OK;
    if (mm->noise_n > 0 && nb > 0) {
        // the epoch's rows with their noise, in the order the steps read them
        SP_TRY(augment_rows(mm, &X, &T, perm, nb * batch, batch));
        for (int64_t b = 0; b < nb && !st; ++b)
            st = fused_step(mm, X + b * batch * kIn, T + b * batch * kOut, nullptr, batch, true, lr, lbuf + b);
    } else {
        for (int64_t b = 0; b < nb && !st; ++b) st = fused_step(mm, X, T, perm + b * batch, batch, true, lr, lbuf + b);
    }
    if (!st && mean_loss) {
        losses.resize((size_t)std::max<int64_t>(nb, 1));
        if (hipMemcpyAsync(losses.data(), lbuf, losses.size() * 4, hipMemcpyDeviceToHost, mm->stream) != hipSuccess ||
            hipStreamSynchronize(mm->stream) != hipSuccess)
            st = SP_EDEVICE;
        double s = 0.0;
        for (int64_t b = 0; b < nb; ++b) s += losses[b];
        *mean_loss = nb > 0 ? (float)(s / (double)nb / (double)(batch * kOut)) : 0.0f;
    }
    (void)hipStreamSynchronize(mm->stream);
    if (st == SP_EDEVICE) return mfail(mm, st, "epoch copy failed");
    return st;
}

// ------------------------------------------------- closure <-> simulation
}  // extern "C"

namespace {

// Static cell data of every cell, computed once per floe set (cells
// re-synchronised later refresh their own).
sp_status ensure_cell_data(sp_ctx* c)
{
    if (c->desc && c->mf && !c->desc_stale) return SP_OK;
    if (!c->desc) SP_TRY(dalloc(c, &c->desc, (size_t)c->ncells * 6));
    if (!c->mf) SP_TRY(dalloc(c, &c->mf, (size_t)c->ncells * 4));
    c->desc_stale = false;
    hipLaunchKernelGGL(descriptors_kernel, dim3(c->ncells), dim3(256), 0, c->stream, nullptr, c->cell_start, c->r,
                       c->h, 1.0 / (c->p.cell_lx * c->p.cell_ly), c->p.rho_ice, c->p.cd * c->p.rho_ocean, c->desc,
                       c->mf);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

sp_status upload_ocean_centres(sp_ctx* c)
{
    SP_TRY(dalloc(c, &c->ocen, (size_t)c->ncells * 4));
    const StepArgs s = make_args(c, 0.0);
    hipLaunchKernelGGL(ocean_centre_kernel, dim3((c->ncells + 255) / 256), dim3(256), 0, c->stream, c->ncells,
                       c->phase, c->nmodes, s.modes, s.u0, s.v0, c->ocen);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

ClosureArgs closure_args(const sp_ctx* c, double t)
{
    ClosureArgs a;
    memset(&a, 0, sizeof a);
    a.red = c->red;
    a.mf = c->mf;
    a.oc = c->ocen;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.dX = c->p.cell_lx;
    a.dY = c->p.cell_ly;
    a.t = t;
    return a;
}

// Reduced DEM of every cell from the statistics `mom` of the current floes.
sp_status init_reduced_all(sp_ctx* c, const double* mom)
{
    SP_TRY(ensure_cell_data(c));
    if (!c->red) SP_TRY(dalloc(c, &c->red, (size_t)c->ncells * 4));
    hipLaunchKernelGGL(reduced_init_kernel, dim3((c->ncells + 255) / 256), dim3(256), 0, c->stream, nullptr,
                       c->ncells, nullptr, mom, closure_args(c, c->t_now), c->red);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

// The same from freshly computed statistics (after the ocean changed).
sp_status refresh_reduced_all(sp_ctx* c)
{
    StepArgs a = make_args(c, 0.0);
    a.mom = c->mom2;
    hipLaunchKernelGGL(stats_kernel, dim3(c->ncells), dim3(256), 0, c->stream, a, nullptr, 0);
    HIP_TRY(c, hipGetLastError());
    return init_reduced_all(c, c->mom2);
}

}  // namespace

extern "C" {

sp_status sp_closure_features(sp_ctx* c, float* x)
{
    if (!c || !x) return c ? fail(c, SP_EINVAL, "null features buffer") : SP_EINVAL;
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    SP_TRY(flush_lf(c));
    SP_TRY(upload_phase(c));
    SP_TRY(ensure_cell_data(c));
    hipLaunchKernelGGL(features_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, nullptr, c->ncells,
                       c->Q[c->kstep & 1], closure_args(c, c->t_now), c->desc, x);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

sp_status sp_closure_sample(sp_ctx* c, double dt, int32_t mode, float* x, float* t)
{
    if (!c || !x || !t) return c ? fail(c, SP_EINVAL, "null sample buffers") : SP_EINVAL;
    if (mode != SP_TEND_FULL && mode != SP_TEND_RESIDUAL) return fail(c, SP_EINVAL, "unknown tendency mode %d", mode);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, SP_EINVAL, "dt must be positive");
    if (c->p.flags & SP_NO_CONTINUUM) return fail(c, SP_ESTATE, "sampling needs the continuum update");
    if (c->p.flags & SP_TANGENTIAL_SPRING) return fail(c, SP_ESTATE, "sampling runs the viscous contact law");
    if (c->p.flags & SP_WALL_X) return fail(c, SP_ESTATE, "sampling runs on the periodic coarse grid");
    if (c->N0 > 1) return fail(c, SP_ESTATE, "sampling takes one-step tendencies (N0 = 1)");
    if (!c->have_floes) return fail(c, SP_ESTATE, "no floes");
    SP_TRY(flush_lf(c));
    SP_TRY(upload_phase(c));
    SP_TRY(ensure_cell_data(c));
    if (!c->qprev) SP_TRY(dalloc(c, &c->qprev, (size_t)c->ncells * 4));
    const double* Q = c->Q[c->kstep & 1];
    const ClosureArgs a = closure_args(c, c->t_now);
    if (mode == SP_TEND_RESIDUAL) {
        hipLaunchKernelGGL(base_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, Q, c->qprev, a, dt);
        HIP_TRY(c, hipGetLastError());
    } else {
        HIP_TRY(c, hipMemcpyAsync(c->qprev, Q, (size_t)c->ncells * 4 * 8, hipMemcpyDeviceToDevice, c->stream));
    }
    hipLaunchKernelGGL(features_kernel, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, nullptr, c->ncells,
                       c->qprev, a, c->desc, x);
    HIP_TRY(c, hipGetLastError());
    SP_TRY(sp_step(c, dt, 1));
    SP_TRY(flush_lf(c));
    hipLaunchKernelGGL(tendency_kernel, dim3((c->ncells + 255) / 256), dim3(256), 0, c->stream, c->Q[c->kstep & 1],
                       c->qprev, c->ncells, dt, t);
    HIP_TRY(c, hipGetLastError());
    return SP_OK;
}

}  // extern "C"
