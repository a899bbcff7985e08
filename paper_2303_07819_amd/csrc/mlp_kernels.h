// Device code of the learned closure: a 45 -> 128 -> 128 -> 128 -> 4 GELU
// network run with bfloat16 MFMA (v_mfma_f32_16x16x16_bf16) and FP32
// accumulation, its backward pass, Adam, and the per-cell feature gather.
//
// Every matrix product goes through one tiled kernel: C = A B with A(m, k) and
// B(k, n) addressed through strides, so the transposed products of the
// backward pass need no copies.  A 256-thread workgroup computes a 64 x 64
// output tile; each wavefront owns a 32 x 32 quarter as 2 x 2 MFMA tiles and
// the K loop stages 64 x 16 and 16 x 64 bfloat16 tiles in LDS.  Products with
// few output tiles and a long K (the weight gradients, K = batch) split K over
// the grid's z dimension into partial tiles that a second kernel sums in a
// fixed order.  The epilogue
// adds the bias and applies GELU (forward), the GELU derivative (backward) or
// an affine output map, and writes FP32 and/or bfloat16 results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmlp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 45, kHid = 128, kOut = 4;
constexpr int kNParams = kHid * kIn + kHid + 2 * (kHid * kHid + kHid) + kOut * kHid + kOut;   // 39,428
// offsets of W1, b1, W2, b2, W3, b3, W4, b4 in the flat parameter vector
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid, kOffB4 = kOffW4 + kOut * kHid;

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum { EPI_STORE = 0, EPI_HIDDEN = 1, EPI_AFFINE = 2, EPI_GELU_BACK = 3 };

struct GemmArgs {
    const uint16_t* A;
    long sam, sak;          // A(m, k) = A[m sam + k sak]
    const uint16_t* B;
    long sbk, sbn;          // B(k, n) = B[k sbk + n sbn]
    int M, N, K;
    int mode;
    const float* bias;      // [N] (EPI_HIDDEN, EPI_AFFINE)
    const float* scale;     // [N] (EPI_AFFINE): out = (C + bias) scale + shift
    const float* shift;
    float* outF;            // FP32 result (may be null)
    long ldf;
    uint16_t* outH;         // bfloat16 result (may be null)
    long ldh;
    const float* zsaved;    // EPI_GELU_BACK: pre-activations [M][ldz]
    long ldz;
    int kchunk;             // split K: workgroup z covers k in [z kchunk, (z + 1) kchunk) (EPI_STORE into
    long part_stride;       // outF + z part_stride; 0: one slice)
};

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ uint16_t As[64][16];
    __shared__ uint16_t Bs[16][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kbeg = g.kchunk > 0 ? (int)blockIdx.z * g.kchunk : 0;
    const int kend = g.kchunk > 0 ? min(g.K, kbeg + g.kchunk) : g.K;
    if (g.kchunk > 0) g.outF += (long)blockIdx.z * g.part_stride;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        {
            const int r = tid >> 2, kk = (tid & 3) * 4;
            const int m = m0 + r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + kk + q;
                As[r][kk + q] = (m < g.M && k < kend) ? g.A[(long)m * g.sam + (long)k * g.sak] : (uint16_t)0;
            }
        }
        {
            const int kk = tid >> 4, cc = (tid & 15) * 4;
            const int k = k0 + kk;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = n0 + cc + q;
                Bs[kk][cc + q] = (k < kend && n < g.N) ? g.B[(long)k * g.sbk + (long)n * g.sbn] : (uint16_t)0;
            }
        }
        __syncthreads();
        const int kq = 4 * (lane >> 4), li = lane & 15;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x4 a;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = (short)As[wm + i * 16 + li][kq + q];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bf16x4 b;
#pragma unroll
                for (int q = 0; q < 4; ++q) b[q] = (short)Bs[kq + q][wn + j * 16 + li];
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // output element (row, col) of lane / register: row = 4 (lane / 16) + r, col = lane % 16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                float v = acc[i][j][r];
                if (g.mode == EPI_HIDDEN) {
                    const float z = v + g.bias[col];
                    if (g.outF) g.outF[(long)row * g.ldf + col] = z;
                    g.outH[(long)row * g.ldh + col] = f2bf(gelu_f(z));
                } else if (g.mode == EPI_AFFINE) {
                    const float y = v + g.bias[col];
                    g.outF[(long)row * g.ldf + col] = g.scale ? y * g.scale[col] + g.shift[col] : y;
                } else if (g.mode == EPI_GELU_BACK) {
                    const float d = v * gelu_grad_f(g.zsaved[(long)row * g.ldz + col]);
                    if (g.outF) g.outF[(long)row * g.ldf + col] = d;
                    if (g.outH) g.outH[(long)row * g.ldh + col] = f2bf(d);
                } else {
                    if (g.outF) g.outF[(long)row * g.ldf + col] = v;
                    if (g.outH) g.outH[(long)row * g.ldh + col] = f2bf(v);
                }
            }
}

// ------------------------------------------------ fused forward (inference)
// Normalisation, the three GELU layers and the output map in one launch, for
// inference (nothing is kept for a backward pass).  Each product runs
// transposed, H^T = W X^T, with the weights as the MFMA A operand and the
// activations as the B operand: the output tile of a 16 x 16 x 16 step holds in
// each lane four consecutive output features of row lane % 16, which is exactly
// the B operand of the next layer's step, so activations stay in registers.
// A wavefront carries 16 rows through all layers; the workgroup stages every
// weight tile in LDS once, swizzled so that each lane's four A values are one
// 8-byte read (80 KB: two workgroups per CU).
constexpr int kFwdWaves = 8;
constexpr int kFwdT1 = 8 * 3, kFwdT2 = 64, kFwdT3 = 64, kFwdT4 = 8;   // 16 x 16 tiles: W1 (K 45 -> 48), W2, W3,
constexpr int kFwdTiles = kFwdT1 + kFwdT2 + kFwdT3 + kFwdT4;          // W4 (4 outputs -> 16)
constexpr size_t kFwdLds = (size_t)kFwdTiles * 64 * sizeof(bf16x4);   // 160 tiles: 81,920 B

// A operand of weight tile (ob, kb) of a layer with nin inputs and nout
// outputs: lane l holds W[ob 16 + l % 16][kb 16 + 4 (l / 16) + q], q < 4 (zero
// outside the matrix); W row-major [nout][nin].
__device__ __forceinline__ bf16x4 weight_tile_operand(const uint16_t* W, int nin, int nout, int ob, int kb,
                                                      int lane)
{
    const int o = ob * 16 + (lane & 15);
    const int k0 = kb * 16 + 4 * (lane >> 4);
    bf16x4 a;
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = (short)((o < nout && k0 + q < nin) ? W[o * nin + k0 + q] : 0);
    return a;
}

// Bias, GELU and bfloat16 rounding of an output tile: element r of ob's tile
// is feature ob 16 + 4 (lane / 16) + r.
__device__ __forceinline__ bf16x4 hidden_operand(const f32x4 acc, const float* bias, int ob, int lane)
{
    const int f0 = ob * 16 + 4 * (lane >> 4);
    bf16x4 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = (short)f2bf(gelu_f(acc[r] + bias[f0 + r]));
    return h;
}

// One hidden layer: out[ob] = sum over kb of W(ob, kb) in[kb], 8 x 8 steps,
// weight tiles from LDS (tile index base + ob 8 + kb).
__device__ __forceinline__ void hidden_layer(const bf16x4* wt, int base, const bf16x4 in[8], const float* bias,
                                             int lane, bf16x4 out[8])
{
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wt[(base + ob * 8 + kb) * 64 + lane], in[kb], acc, 0, 0,
                                                             0);
        out[ob] = hidden_operand(acc, bias, ob, lane);
        __builtin_amdgcn_sched_barrier(0);   // keep each tile row's weight reads next to its steps
    }
}

// The weight tiles in the order and lane layout the fused forward stages in
// LDS (tile t, lane l at wsw[t 64 + l]), from the bfloat16 parameters.
__global__ void swizzle_weights_kernel(const uint16_t* th, bf16x4* wsw)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kFwdTiles * 64) return;
    const int t = e >> 6, l = e & 63;
    bf16x4 a;
    if (t < kFwdT1)
        a = weight_tile_operand(th + kOffW1, kIn, kHid, t / 3, t % 3, l);
    else if (t < kFwdT1 + kFwdT2)
        a = weight_tile_operand(th + kOffW2, kHid, kHid, (t - kFwdT1) >> 3, (t - kFwdT1) & 7, l);
    else if (t < kFwdT1 + kFwdT2 + kFwdT3)
        a = weight_tile_operand(th + kOffW3, kHid, kHid, (t - kFwdT1 - kFwdT2) >> 3, (t - kFwdT1 - kFwdT2) & 7, l);
    else
        a = weight_tile_operand(th + kOffW4, kHid, kOut, 0, t - kFwdT1 - kFwdT2 - kFwdT3, l);
    wsw[e] = a;
}

// wsw: weight tiles from swizzle_weights_kernel; theta: FP32 parameters (biases); norm: x_mean[45],
// x_inv_std[45], y_mean[4], (target inverse std)[4], y_std[4]; y [M][4].
__global__ __launch_bounds__(64 * kFwdWaves) __attribute__((amdgpu_waves_per_eu(4))) void mlp_forward_kernel(const float* x, long M, const bf16x4* wsw,
                                                                     const float* theta, const float* norm,
                                                                     float* y)
{
    extern __shared__ __align__(16) unsigned char fwd_smem[];
    bf16x4* wt = reinterpret_cast<bf16x4*>(fwd_smem);   // [kFwdTiles][64]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        const uint4* src = reinterpret_cast<const uint4*>(wsw);   // two tile lanes per 16 bytes
        uint4* dst = reinterpret_cast<uint4*>(wt);
        for (int e = tid; e < kFwdTiles * 32; e += blockDim.x) dst[e] = src[e];
    }
    __syncthreads();

    const float* xm = norm;
    const float* xis = norm + kIn;
    const float* ym = norm + 2 * kIn;
    const float* ys = norm + 2 * kIn + 2 * kOut;
    const long step = (long)gridDim.x * kFwdWaves * 16;
    for (long r0 = ((long)blockIdx.x * kFwdWaves + wave) * 16; r0 < M; r0 += step) {
        const long row = r0 + (lane & 15);
        const bool ok = row < M;
        // layer 1: inputs 4 (lane / 16) + q of each 16-feature block, normalised
        bf16x4 xb[3];
#pragma unroll
        for (int kb = 0; kb < 3; ++kb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = kb * 16 + 4 * (lane >> 4) + q;
                xb[kb][q] = (short)((ok && f < kIn) ? f2bf((x[row * kIn + f] - xm[f]) * xis[f]) : 0);
            }
        bf16x4 h1[8];
#pragma unroll
        for (int ob = 0; ob < 8; ++ob) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < 3; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wt[(ob * 3 + kb) * 64 + lane], xb[kb], acc, 0, 0, 0);
            h1[ob] = hidden_operand(acc, theta + kOffB1, ob, lane);
            __builtin_amdgcn_sched_barrier(0);
        }
        bf16x4 h2[8], h3[8];
        hidden_layer(wt, kFwdT1, h1, theta + kOffB2, lane, h2);
        hidden_layer(wt, kFwdT1 + kFwdT2, h2, theta + kOffB3, lane, h3);
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wt[(kFwdT1 + kFwdT2 + kFwdT3 + kb) * 64 + lane], h3[kb],
                                                             acc, 0, 0, 0);
        // lanes 0-15 hold outputs 0-3 of row lane
        if (lane < 16 && ok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) y[row * kOut + r] = (acc[r] + theta[kOffB4 + r]) * ys[r] + ym[r];
        }
    }
}

// Sum of the `slices` partial products of a split-K product, in slice order:
// out[i] = sum_z part[z stride + i], i < n.
__global__ void splitk_reduce_kernel(const float* part, int slices, long stride, long n, float* out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int z = 0; z < slices; ++z) s += part[(long)z * stride + i];
    out[i] = s;
}

// x [M][kIn] FP32 -> bfloat16 of (x - mean) / std; optional row gather.
__global__ void normalize_input_kernel(const float* x, const int32_t* rows, long M, const float* mean,
                                       const float* inv_std, uint16_t* out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * kIn) return;
    const long m = i / kIn;
    const int f = (int)(i % kIn);
    const long src = rows ? (long)rows[m] : m;
    out[i] = f2bf((x[src * kIn + f] - mean[f]) * inv_std[f]);
}

// Mean-squared-error gradient on normalised targets: d = 2 (y - (t - mean) / std) / (B kOut),
// written in FP32 and bfloat16; per-element squared errors for the loss.
__global__ void mse_grad_kernel(const float* y, const float* t, const int32_t* rows, int B, const float* tmean,
                                const float* tinv_std, float* dF, uint16_t* dH, float* sq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kOut) return;
    const int m = i / kOut, o = i % kOut;
    const long src = rows ? (long)rows[m] : m;
    const float tn = (t[src * kOut + o] - tmean[o]) * tinv_std[o];
    const float e = y[i] - tn;
    const float d = 2.0f * e / (float)(B * kOut);
    dF[i] = d;
    dH[i] = f2bf(d);
    sq[i] = e * e;
}

// Column sums of d [rows][cols] (bias gradients), one workgroup per column,
// fixed reduction order.
__global__ __launch_bounds__(256) void colsum_kernel(const float* d, int rows, int cols, float* out)
{
    __shared__ float part[256];
    const int col = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < rows; r += 256) s += d[(long)r * cols + col];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = part[0];
}

// Sum of n floats in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void sum_kernel(const float* x, int n, float* out)
{
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += (double)x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)part[0];
}

// Adam (bias-corrected) on the FP32 master parameters; refreshes the
// bfloat16 copy the matrix products read.
__global__ void adam_kernel(float* theta, float* m, float* v, const float* grad, int n, float lr, float b1,
                            float b2, float eps, float c1, float c2, uint16_t* theta_h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float th = theta[i] - lr * mh / (sqrtf(vh) + eps);
    theta[i] = th;
    theta_h[i] = f2bf(th);
}

__global__ void to_bf16_kernel(const float* x, int n, uint16_t* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(x[i]);
}

}  // namespace spmlp
