// Device code of the learned closure's inference: a 45 -> 128 -> 128 -> 128
// -> 4 GELU network run with bfloat16 MFMA (v_mfma_f32_16x16x32_bf16 and
// 16x16x16 steps) and FP32 accumulation, in one fused launch per batch of
// rows; the GELU used by inference and training; the per-cell feature gather
// helpers.  The training step (forward, backward, Adam) is in
// train_kernels.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmlp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
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

// Four floats to bfloat16, round to nearest even (the gfx950 conversion
// instruction, two values per instruction).
__device__ __forceinline__ bf16x4 to_bf16x4(float a, float b, float c, float d)
{
    bf16x4 h;
    h[0] = __builtin_bit_cast(short, (__bf16)a);
    h[1] = __builtin_bit_cast(short, (__bf16)b);
    h[2] = __builtin_bit_cast(short, (__bf16)c);
    h[3] = __builtin_bit_cast(short, (__bf16)d);
    return h;
}

// E(z) = erfc(|z| / sqrt 2) = 2 Phi(-|z|), twice the lower tail of the normal
// distribution, without branches or division.  Writing erfc(x) = exp(-x^2 +
// P(x)) with P smooth and P(0) = 0, and taking s = |z| sqrt(log2(e) / 2), the
// tail is E = 2^(-s^2 + R(s)) with R(s) = log2(e) P(s / sqrt(log2 e)).  R here
// is a degree-7 least-squares fit of our own in Chebyshev nodes on x in
// [0, 4], reweighted towards equal ripple, with R(0) = 0 kept exact: relative
// error of erfc 4e-6 on [0, 4].  Its leading coefficient is negative, so past
// the fit range (|z| > 5.66, where E < 2e-8) the exponent only falls and E
// goes to zero without a clamp.  Evaluated in FP32, GELU below is within
// 7e-7 of its exact value for every z.
__device__ __forceinline__ float erfc_tail(float z)
{
    const float s = fabsf(z) * 0.8493217825889587f;
    float q = -5.538857749343151e-06f;
    q = fmaf(q, s, 0.00016052437422331423f);
    q = fmaf(q, s, -0.0020819962956011295f);
    q = fmaf(q, s, 0.01627247780561447f);
    q = fmaf(q, s, -0.08793872594833374f);
    q = fmaf(q, s, 0.36431241035461426f);
    q = fmaf(q, s, -1.3554487228393555f);
    return __builtin_amdgcn_exp2f(s * (q - s));
}

// Twice GELU in its erf form: 2 z Phi(z) = z + |z| - |z| E(z).
__device__ __forceinline__ float twice_gelu(float z) { return fmaf(-fabsf(z), erfc_tail(z), z + fabsf(z)); }

// GELU = z Phi(z) (half of twice_gelu) and its derivative Phi(z) + z phi(z),
// phi(z) = exp(-z^2 / 2) / sqrt(2 pi), from one evaluation of the tail.
__device__ __forceinline__ void gelu_and_grad(float z, float& g, float& dg)
{
    const float e = erfc_tail(z);
    g = 0.5f * fmaf(-fabsf(z), e, z + fabsf(z));
    const float h = 0.5f * e;
    const float phi = z >= 0.0f ? 1.0f - h : h;
    const float dens = 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * z * z);
    dg = fmaf(z, dens, phi);
}

// ------------------------------------------------ fused forward (inference)
// Normalisation, the three GELU layers and the output map in one launch, for
// inference (nothing is kept for a backward pass).  Each product runs
// transposed, H^T = W X^T, with the weights as the MFMA A operand and the
// activations as the B operand.  The output tile of a step holds in each lane
// four consecutive output features of row lane % 16 (features 4 (lane / 16)
// + r of the tile); the hidden layers take their inputs 32 at a time with
// v_mfma_f32_16x16x32_bf16, whose B operand gives each lane 8 input slots, and
// slot q of lane group g = lane / 16 is read as feature 4 g + q (q < 4) or
// 16 + 4 g + q - 4 (q >= 4) of the 32: exactly the two output tiles of the
// previous layer that lane holds, so activations never leave registers (the
// weight tiles are stored in the same permuted order; a product's sum does not
// depend on the order of its terms).  Layer 1 (45 inputs, padded to 48) runs
// 16x16x16 steps on the normalised inputs.  Biases start the accumulators.
// A wavefront carries 16 rows through all layers.  The workgroup stages one
// image in LDS: every weight tile swizzled so that each lane's A values are
// one read, the biases and the normalisation (79 KB: two workgroups per CU).
constexpr int kFwdWaves = 8;
constexpr int kFwdT1 = 8 * 3;                  // W1: 8 output x 3 input tiles of 16 x 16 (K 45 -> 48)
constexpr int kFwdT2 = 8 * 4, kFwdT3 = 8 * 4;  // W2, W3: 8 output x 4 input tiles of 16 x 32
constexpr int kFwdT4 = 4;                      // W4: 4 input tiles of 16 x 32, output rows 0-3 stored
constexpr int kFwdNormLen = 48 + 48 + 2 * kOut;  // x mean, x inverse std (each padded to 48), y mean, y std
// byte offsets in the staged image
constexpr size_t kFwdOffW32 = (size_t)kFwdT1 * 64 * sizeof(bf16x4);
constexpr size_t kFwdOffW4 = kFwdOffW32 + (size_t)(kFwdT2 + kFwdT3) * 64 * sizeof(bf16x8);
constexpr size_t kFwdOffBias = kFwdOffW4 + (size_t)kFwdT4 * 16 * sizeof(bf16x8);  // b1, b2, b3, b4
constexpr size_t kFwdOffNorm = kFwdOffBias + (size_t)(3 * kHid + kOut) * sizeof(float);
constexpr size_t kFwdLds = kFwdOffNorm + kFwdNormLen * sizeof(float);
constexpr int kFwdStageThreads = (kFwdT1 + kFwdT2 + kFwdT3) * 64 + kFwdT4 * 16 + 3 * kHid + kOut + kFwdNormLen;
static_assert(kFwdOffBias % 16 == 0 && kFwdOffNorm % 16 == 0 && kFwdLds % 16 == 0, "aligned LDS reads");
static_assert(2 * kFwdLds <= 160 * 1024, "two forward workgroups per compute unit");

// A operand of 16 x 16 weight tile (ob, kb) of a layer with nin inputs and
// nout outputs: lane l holds W[ob 16 + l % 16][kb 16 + 4 (l / 16) + q], q < 4
// (zero outside the matrix); W row-major [nout][nin].
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

// A operand of 16 x 32 weight tile (ob, kb) in the permuted input order, the
// weights halved (exact in bfloat16): lane l holds W[ob 16 + l % 16][kb 32 +
// 4 (l / 16) + q] / 2 for q < 4 and W[ob 16 + l % 16][kb 32 + 16 + 4 (l / 16)
// + q - 4] / 2 for q >= 4.
__device__ __forceinline__ bf16x8 weight_tile_operand32(const uint16_t* W, int nin, int nout, int ob, int kb,
                                                        int lane)
{
    const int o = ob * 16 + (lane & 15);
    const int g = lane >> 4;
    bf16x8 a;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = kb * 32 + (q < 4 ? 4 * g + q : 16 + 4 * g + q - 4);
        const float w = (o < nout && k < nin) ? 0.5f * bf2f(W[o * nin + k]) : 0.0f;
        a[q] = __builtin_bit_cast(short, (__bf16)w);
    }
    return a;
}

// Twice GELU, rounded to bfloat16, of an output tile (bias already in acc).
// The layer it feeds takes half its weights: scaling by a power of two
// commutes with the rounding, so the products are those of GELU and the
// weights themselves.
__device__ __forceinline__ bf16x4 hidden_operand(const f32x4 acc)
{
    return to_bf16x4(twice_gelu(acc[0]), twice_gelu(acc[1]), twice_gelu(acc[2]), twice_gelu(acc[3]));
}

__device__ __forceinline__ bf16x8 join(bf16x4 a, bf16x4 b)
{
    return bf16x8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

__device__ __forceinline__ f32x4 mfma_step(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma_step(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One GELU layer of 8 output tiles, out[ob] = GELU(bias + sum over kb of
// W(ob, kb) b[kb]) (twice GELU, see hidden_operand), weight tile (ob, kb) at
// wt[(ob KB + kb) 64 + lane] in LDS, biases at bias[0 .. 127] in LDS.
// Software-pipelined: while the vector ALUs take the GELU of tile ob, the
// matrix core runs the KB steps of tile ob + 1, whose operands were read from
// LDS one tile earlier, and the reads for tile ob + 2 are in flight.
template <int KB, typename T>
__device__ __forceinline__ void gelu_layer(const T* wt, const float* bias, const T b[KB], int lane, bf16x4 out[8])
{
    T a[2][KB];
    f32x4 bs[2];
    const int g4 = 4 * (lane >> 4);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        a[0][kb] = wt[kb * 64 + lane];
        a[1][kb] = wt[(KB + kb) * 64 + lane];
    }
    bs[0] = *reinterpret_cast<const f32x4*>(bias + g4);
    bs[1] = *reinterpret_cast<const f32x4*>(bias + 16 + g4);
    f32x4 acc = bs[0];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = mfma_step(a[0][kb], b[kb], acc);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        f32x4 nxt = acc;
        if (ob + 1 < 8) {
            const int s = (ob + 1) & 1;
            nxt = bs[s];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) nxt = mfma_step(a[s][kb], b[kb], nxt);
        }
        if (ob + 2 < 8) {
            const int s = ob & 1;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) a[s][kb] = wt[((ob + 2) * KB + kb) * 64 + lane];
            bs[s] = *reinterpret_cast<const f32x4*>(bias + (ob + 2) * 16 + g4);
        }
        bf16x4 o = hidden_operand(acc);
        asm volatile("" : "+v"(o));   // computed here, not sunk to the next layer's first use
        out[ob] = o;
        acc = nxt;
        // interleave: the reads first, then each step of tile ob + 1 between GELU instructions
        __builtin_amdgcn_sched_group_barrier(0x100, KB + 1, 0);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The image the fused forward stages in LDS (kFwdLds bytes): the 16 x 16
// tiles of W1 (tile t = ob 3 + kb, lane l, at bf16x4 index t 64 + l), the
// 16 x 32 tiles of W2 and W3 (from kFwdOffW32, bf16x8 index t 64 + l, t = ob 4
// + kb), the 16 x 32 tiles of W4 with only the lanes of output rows 0-3 (from
// kFwdOffW4, bf16x8 index kb 16 + 4 (l / 16) + l % 16 for l % 16 < 4), the
// FP32 biases b1, b2, b3, b4 and the normalisation (x mean and x inverse std
// each padded with zeros to 48, y mean, y std); from the bfloat16 and FP32
// parameters and the normalisation [x mean 45 | x inverse std 45 | y mean 4 |
// y inverse std 4 | y std 4].
__global__ void stage_forward_kernel(const uint16_t* th, const float* theta, const float* norm, unsigned char* img)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kFwdT1 * 64) {
        const int t = e >> 6;
        reinterpret_cast<bf16x4*>(img)[e] = weight_tile_operand(th + kOffW1, kIn, kHid, t / 3, t % 3, e & 63);
        return;
    }
    e -= kFwdT1 * 64;
    if (e < (kFwdT2 + kFwdT3) * 64) {
        const int u = e >> 6, l = e & 63;
        const uint16_t* W = u < kFwdT2 ? th + kOffW2 : th + kOffW3;
        const int v = u < kFwdT2 ? u : u - kFwdT2;
        reinterpret_cast<bf16x8*>(img + kFwdOffW32)[e] = weight_tile_operand32(W, kHid, kHid, v >> 2, v & 3, l);
        return;
    }
    e -= (kFwdT2 + kFwdT3) * 64;
    if (e < kFwdT4 * 16) {
        const int kb = e >> 4, j = e & 15;
        reinterpret_cast<bf16x8*>(img + kFwdOffW4)[e] =
            weight_tile_operand32(th + kOffW4, kHid, kOut, 0, kb, 16 * (j >> 2) + (j & 3));
        return;
    }
    e -= kFwdT4 * 16;
    if (e < 3 * kHid + kOut) {
        const int off = e < kHid ? kOffB1 + e
                      : e < 2 * kHid ? kOffB2 + e - kHid
                      : e < 3 * kHid ? kOffB3 + e - 2 * kHid : kOffB4 + e - 3 * kHid;
        reinterpret_cast<float*>(img + kFwdOffBias)[e] = theta[off];
        return;
    }
    e -= 3 * kHid + kOut;
    if (e >= kFwdNormLen) return;
    float v;
    if (e < 96) {
        const int f = e % 48;
        v = f < kIn ? norm[(e < 48 ? 0 : kIn) + f] : 0.0f;
    } else {
        v = e < 96 + kOut ? norm[2 * kIn + e - 96] : norm[2 * kIn + 2 * kOut + e - 96 - kOut];
    }
    reinterpret_cast<float*>(img + kFwdOffNorm)[e] = v;
}

// img: the staged image (stage_forward_kernel); x [M][45] raw inputs, y [M][4]
// outputs in physical units.
__global__ __launch_bounds__(64 * kFwdWaves) __attribute__((amdgpu_waves_per_eu(4))) void mlp_forward_kernel(const float* x, long M, const unsigned char* img,
                                                                     float* y)
{
    extern __shared__ __align__(16) unsigned char fwd_smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g4 = 4 * (lane >> 4);
    const long step = (long)gridDim.x * kFwdWaves * 16;
    // raw inputs 4 (lane / 16) + q of each 16-feature block of row r0 + lane % 16,
    // every read in bounds (row and feature clamped; the padding is zeroed later)
    float xv[12];
    auto load_inputs = [&](long r0) {
        const long row = r0 + (lane & 15);
        const float* xr = x + (row < M ? row : M - 1) * kIn;
#pragma unroll
        for (int i = 0; i < 12; ++i) xv[i] = xr[min((i >> 2) * 16 + g4 + (i & 3), kIn - 1)];
    };
    long r0 = ((long)blockIdx.x * kFwdWaves + wave) * 16;
    if (r0 < M) load_inputs(r0);   // in flight with the staging
    {
        // all reads in flight before the first write
        constexpr int kVec = (int)(kFwdLds / 16), kIter = (kVec + 64 * kFwdWaves - 1) / (64 * kFwdWaves);
        const uint4* src = reinterpret_cast<const uint4*>(img);
        uint4* dst = reinterpret_cast<uint4*>(fwd_smem);
        uint4 t[kIter];
#pragma unroll
        for (int i = 0; i < kIter; ++i) t[i] = src[min(tid + i * 64 * kFwdWaves, kVec - 1)];
#pragma unroll
        for (int i = 0; i < kIter; ++i) {
            const int e = tid + i * 64 * kFwdWaves;
            if (e < kVec) dst[e] = t[i];
        }
    }
    __syncthreads();
    const bf16x4* w1 = reinterpret_cast<const bf16x4*>(fwd_smem);
    const bf16x8* w32 = reinterpret_cast<const bf16x8*>(fwd_smem + kFwdOffW32);
    const bf16x8* w4 = reinterpret_cast<const bf16x8*>(fwd_smem + kFwdOffW4);
    const float* bias = reinterpret_cast<const float*>(fwd_smem + kFwdOffBias);
    const float* nrm = reinterpret_cast<const float*>(fwd_smem + kFwdOffNorm);
    const float* xm = nrm;
    const float* xis = nrm + 48;
    const float* ym = nrm + 96;
    const float* ys = nrm + 96 + kOut;
    for (; r0 < M; r0 += step) {
        const long row = r0 + (lane & 15);
        const bool ok = row < M;   // rows past M compute on a copy of row M - 1 and are not stored
        // layer 1 on the normalised inputs
        bf16x4 xb[3];
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) {
            const int f0 = kb * 16 + g4;
            const f32x4 m = *reinterpret_cast<const f32x4*>(xm + f0);
            const f32x4 is = *reinterpret_cast<const f32x4*>(xis + f0);
            // padding features: a finite input times the zero inverse std of the padding
            xb[kb] = to_bf16x4((xv[kb * 4] - m[0]) * is[0], (xv[kb * 4 + 1] - m[1]) * is[1],
                               (xv[kb * 4 + 2] - m[2]) * is[2], (xv[kb * 4 + 3] - m[3]) * is[3]);
        }
        bf16x4 h1[8], h2[8], h3[8];
        gelu_layer<3, bf16x4>(w1, bias, xb, lane, h1);
        bf16x8 b[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) b[kb] = join(h1[2 * kb], h1[2 * kb + 1]);
        gelu_layer<4, bf16x8>(w32, bias + kHid, b, lane, h2);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) b[kb] = join(h2[2 * kb], h2[2 * kb + 1]);
        gelu_layer<4, bf16x8>(w32 + kFwdT2 * 64, bias + 2 * kHid, b, lane, h3);
        // output map: A rows 0-3 (lanes with lane % 16 < 4) are the output
        // weights; the other lanes read some stored row, and the output rows they
        // make (features 4-15, each from its own A row) are never stored
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const int ai = g4 + (lane & 3);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_step(w4[kb * 16 + ai], join(h3[2 * kb], h3[2 * kb + 1]), acc);
        // lanes 0-15 hold outputs 0-3 of row lane
        if (lane < 16 && ok) {
            const float* b4 = bias + 3 * kHid;
#pragma unroll
            for (int r = 0; r < 4; ++r) y[row * kOut + r] = (acc[r] + b4[r]) * ys[r] + ym[r];
        }
        if (r0 + step < M) load_inputs(r0 + step);
    }
}

__global__ void to_bf16_kernel(const float* x, int n, uint16_t* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(x[i]);
}

}  // namespace spmlp
