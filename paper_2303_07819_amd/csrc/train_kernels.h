// Fused training step of the closure network: two launches per Adam step.
//
// tr_rows_kernel: one workgroup per 16 rows of the batch, the network's
// weights staged in LDS as MFMA operand tiles (forward tiles as in the
// inference forward, unhalved, and the transposed tiles of W2, W3 and W4 for
// the backward products).  Each of its eight wavefronts takes one 16-unit
// tile of every hidden layer: forward through the four layers, each layer's
// output tiles exchanged through LDS to form the next product's B operand;
// the GELU derivatives of the wavefront's own tiles kept in registers; the
// loss gradient of the mean squared error on normalised targets (every
// wavefront forms it); then backward through W4^T, W3^T and W2^T, exchanged
// the same way (the transposed products dH^T = W^T dZ^T take W^T as the A
// operand, so the output tile of one is the B operand of the next).  Written
// out for the weight gradients: every layer's input activations and deltas in
// bfloat16 (blocks of 16 features x 8 rows), and per 16-row tile the FP32
// column sums of the deltas (bias gradients) and the squared error (loss).
// Every value is computed as by one wavefront carrying the whole tile.
//
// tr_grad_kernel: one workgroup per 16 x 16 tile of a weight gradient
// (160 tiles, those of one output block of a layer on one XCD), dW = sum over
// rows of d^T a as 16x16x32 MFMA steps over the batch, split over eight
// wavefronts and added in a fixed order; the bias gradients from the tile
// partials (stored column by column) in tile order; then either the gradient
// written out, or the Adam update of the tile's parameters with the new
// bfloat16 weights written into the other of two LDS images for the next step.
//
// Rounding points: bfloat16 inputs and weights of every product, FP32
// accumulation, FP32 pre-activations and deltas, activations and deltas
// rounded to bfloat16 for the next product and the weight gradients, FP32
// bias gradients from the FP32 deltas (the bfloat16 mode of the reference
// network rounds at the same points).
#pragma once

namespace spmlp {

constexpr int kTrSplit = 8;            // wavefronts sharing one 16-row tile in tr_rows_kernel
constexpr int kTrTiles = 8 / kTrSplit; // 16-unit tiles of each hidden layer per wavefront
static_assert(kTrTiles * kTrSplit == 8, "the eight tiles of a hidden layer split evenly");
constexpr int kTrRowAlign = 256;       // padded batch: 32-row steps for each wavefront of tr_grad_kernel
constexpr int kTrGradWaves = 8;        // wavefronts splitting the rows of one weight-gradient tile
// LDS image of tr_rows_kernel (bytes)
constexpr size_t kTrOffF1 = 0;                                   // W1: 8 x 3 tiles of 16 x 16 (bf16x4 per lane)
constexpr size_t kTrOffF2 = kTrOffF1 + (size_t)24 * 64 * 8;      // W2: 8 x 4 tiles of 16 x 32, K permuted (bf16x8)
constexpr size_t kTrOffF3 = kTrOffF2 + (size_t)32 * 64 * 16;     // W3
constexpr size_t kTrOffF4 = kTrOffF3 + (size_t)32 * 64 * 16;     // W4: 4 tiles of 16 x 32, the lanes of rows 0-3
constexpr size_t kTrOffB4 = kTrOffF4 + (size_t)4 * 16 * 16;      // W4^T: 8 tiles of 16 x 16 (K = outputs, 4 of 16)
constexpr size_t kTrOffB3 = kTrOffB4 + (size_t)8 * 64 * 8;       // W3^T: 8 x 4 tiles of 16 x 32, K permuted
constexpr size_t kTrOffB2 = kTrOffB3 + (size_t)32 * 64 * 16;     // W2^T
constexpr size_t kTrOffBias = kTrOffB2 + (size_t)32 * 64 * 16;  // b1, b2, b3 [128], b4 [4] (FP32)
constexpr size_t kTrOffNorm = kTrOffBias + (size_t)(3 * kHid + kOut) * 4;   // x mean, x inv std [48 each], t mean, t inv std [4 each]
constexpr size_t kTrLds = kTrOffNorm + (size_t)104 * 4;
constexpr size_t kTrOffX = kTrLds;                               // layer exchange: 2 x 8 tiles x 64 lanes x bf16x4
constexpr size_t kTrLdsAll = kTrOffX + (size_t)2 * 8 * 64 * 8;
static_assert(kTrLdsAll <= 160 * 1024, "one training workgroup per compute unit");
static_assert(kTrOffBias % 16 == 0 && kTrOffNorm % 16 == 0, "aligned LDS reads");
constexpr int kTrBias = 3 * kHid + kOut;   // bias partials per tile: d1, d2, d3 [128], d4 [4]
// activation and delta regions (offsets in features; a region of F features holds F x Bp values)
constexpr int kTrA0 = 0, kTrA1 = 48, kTrA2 = 176, kTrA3 = 304, kTrARows = 432;
constexpr int kTrD1 = 0, kTrD2 = 128, kTrD3 = 256, kTrD4 = 384, kTrDRows = 400;
constexpr int kTrGradTiles = 24 + 64 + 64 + 8;

// A operand of the transposed 16 x 32 tile (ib, kb) of W ([nout][nin]) for
// dH^T = W^T dZ^T: lane l holds W[kb 32 + s(q)][ib 16 + l % 16], s(q) the
// permuted K slot of group g = l / 16 (4 g + q, or 16 + 4 g + q - 4 for q >= 4).
__device__ __forceinline__ bf16x8 wt_tile_operand32(const uint16_t* W, int nin, int nout, int ib, int kb, int lane)
{
    const int i = ib * 16 + (lane & 15);
    const int g = lane >> 4;
    bf16x8 a;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int o = kb * 32 + (q < 4 ? 4 * g + q : 16 + 4 * g + q - 4);
        a[q] = (short)((o < nout && i < nin) ? W[o * nin + i] : 0);
    }
    return a;
}

// Unhalved forward 16 x 32 tile (ob, kb), K permuted as in the inference forward.
__device__ __forceinline__ bf16x8 w_tile_operand32(const uint16_t* W, int nin, int nout, int ob, int kb, int lane)
{
    const int o = ob * 16 + (lane & 15);
    const int g = lane >> 4;
    bf16x8 a;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = kb * 32 + (q < 4 ? 4 * g + q : 16 + 4 * g + q - 4);
        a[q] = (short)((o < nout && k < nin) ? W[o * nin + k] : 0);
    }
    return a;
}

// The whole training image from the bfloat16 and FP32 parameters and the
// normalisation [x mean 45 | x inv std 45 | y mean 4 | y inv std 4 | y std 4].
constexpr int kTrStageThreads = 24 * 64 + 64 * 64 + 4 * 16 + 8 * 64 + 64 * 64 + kTrBias + 104;

__global__ void tr_stage_kernel(const uint16_t* th, const float* theta, const float* norm, unsigned char* img)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 24 * 64) {
        const int t = e >> 6;
        reinterpret_cast<bf16x4*>(img + kTrOffF1)[e] = weight_tile_operand(th + kOffW1, kIn, kHid, t / 3, t % 3, e & 63);
        return;
    }
    e -= 24 * 64;
    if (e < 64 * 64) {   // W2 then W3 forward
        const int u = e >> 6, l = e & 63;
        const uint16_t* W = u < 32 ? th + kOffW2 : th + kOffW3;
        const int v = u & 31;
        reinterpret_cast<bf16x8*>(img + (u < 32 ? kTrOffF2 : kTrOffF3))[(v << 6) | l] =
            w_tile_operand32(W, kHid, kHid, v >> 2, v & 3, l);
        return;
    }
    e -= 64 * 64;
    if (e < 4 * 16) {    // W4 forward, lanes of rows 0-3
        const int kb = e >> 4, j = e & 15;
        reinterpret_cast<bf16x8*>(img + kTrOffF4)[e] =
            w_tile_operand32(th + kOffW4, kHid, kOut, 0, kb, 16 * (j >> 2) + (j & 3));
        return;
    }
    e -= 4 * 16;
    if (e < 8 * 64) {    // W4^T: lane l of tile ib holds W4[q][ib 16 + l % 16] in group 0
        const int ib = e >> 6, l = e & 63;
        bf16x4 a;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = (short)((l >> 4) == 0 ? th[kOffW4 + q * kHid + ib * 16 + (l & 15)] : 0);
        reinterpret_cast<bf16x4*>(img + kTrOffB4)[e] = a;
        return;
    }
    e -= 8 * 64;
    if (e < 64 * 64) {   // W3^T then W2^T
        const int u = e >> 6, l = e & 63;
        const uint16_t* W = u < 32 ? th + kOffW3 : th + kOffW2;
        const int v = u & 31;
        reinterpret_cast<bf16x8*>(img + (u < 32 ? kTrOffB3 : kTrOffB2))[(v << 6) | l] =
            wt_tile_operand32(W, kHid, kHid, v >> 2, v & 3, l);
        return;
    }
    e -= 64 * 64;
    if (e < kTrBias) {
        const int off = e < kHid ? kOffB1 + e
                      : e < 2 * kHid ? kOffB2 + e - kHid
                      : e < 3 * kHid ? kOffB3 + e - 2 * kHid : kOffB4 + e - 3 * kHid;
        reinterpret_cast<float*>(img + kTrOffBias)[e] = theta[off];
        return;
    }
    e -= kTrBias;
    if (e >= 104) return;
    float v;
    if (e < 96) {
        const int f = e % 48;
        v = f < kIn ? norm[(e < 48 ? 0 : kIn) + f] : 0.0f;
    } else {
        v = norm[2 * kIn + (e - 96)];   // y mean [4], y inv std [4]
    }
    reinterpret_cast<float*>(img + kTrOffNorm)[e] = v;
}

// Index of feature f, batch row r in the activation and delta arrays: blocks
// of 16 features x 8 rows (256 B), by feature tile and then by row group, so
// that the 64 lanes of one gradient step read 1 KB in one piece (lane l:
// features l % 16 of a tile, rows 8 (l / 16) .. + 7).
__device__ __forceinline__ long tr_at(int f, long r, int Bp)
{
    return ((long)(f >> 4) * (Bp >> 3) + (r >> 3)) * 128 + (f & 15) * 8 + (r & 7);
}

struct TrainArgs {
    const float* X;           // [*][45] inputs
    const float* T;           // [*][4] targets
    const int32_t* rows;      // batch row r is X row rows[r] (identity if null)
    int B, Bp;                // batch, padded batch (multiple of kTrRowAlign)
    const unsigned char* img; // training image (kTrLds bytes)
    uint16_t* aT;             // kTrARows x Bp activations (tr_at)
    uint16_t* dT;             // kTrDRows x Bp deltas (tr_at)
    float* bpart;             // [kTrBias][Bp / 16] column sums of the FP32 deltas, by column then tile
    double* lpart;            // [Bp / 16] squared errors
};

// Input noise of training steps: feature f < n of row i (of the caller's X)
// consumed by Adam step s gets sd[f] times a standard normal of (seed, s, i,
// f / 2).
struct NoiseArgs {
    int n;
    unsigned long long seed;
    float sd[48];
};

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the output function of one step.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x)
{
    unsigned long long z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Two standard normals from 64 random bits by the Box-Muller transform
// (two 24-bit uniforms, the first in (0, 1]).
__device__ __forceinline__ void box_muller(unsigned long long h, float& z0, float& z1)
{
    const float u1 = (float)((h >> 40) + 1) * 5.9604644775390625e-8f;
    const float u2 = (float)(h & 0xffffffull) * 5.9604644775390625e-8f;
    const float r = sqrtf(-2.0f * __logf(u1));
    float sn, cs;
    __sincosf(6.283185307179586f * u2, &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
}

// Training rows with their input noise, in the order the steps read them:
// row k of the output is row rows[k] of X (k if rows is null) plus its noise
// for Adam step step0 + k / batch; targets copied alongside.  24 threads per
// row, neighbouring threads on neighbouring words: thread p < 23 takes
// features 2p and 2p + 1 (the two normals of pair p), thread 23 the targets.
__global__ __launch_bounds__(256) void tr_augment_kernel(const float* X, const float* T, const int32_t* rows,
                                                         long n, long long step0, int batch, NoiseArgs na,
                                                         float* Xo, float* To)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long k = t / 24;
    const int p = (int)(t - k * 24);
    if (k >= n) return;
    const long i = rows ? (long)rows[k] : k;
    if (p == 23) {
#pragma unroll
        for (int o = 0; o < kOut; ++o) To[k * kOut + o] = T[i * kOut + o];
        return;
    }
    const int f = 2 * p;
    float a = X[i * kIn + f];
    float b = f + 1 < kIn ? X[i * kIn + f + 1] : 0.0f;
    if (f < na.n) {
        const unsigned long long base =
            splitmix64(splitmix64(na.seed ^ (unsigned long long)(step0 + k / batch)) ^ (unsigned long long)i);
        float z0, z1;
        box_muller(splitmix64(base ^ (unsigned long long)p), z0, z1);
        a += na.sd[f] * z0;
        if (f + 1 < na.n) b += na.sd[f + 1] * z1;
    }
    Xo[k * kIn + f] = a;
    if (f + 1 < kIn) Xo[k * kIn + f + 1] = b;
}

// FP32 sum over each row of 16 lanes by DPP row shifts (fixed order); the
// total lands in the row's last lane.
__device__ __forceinline__ float row16_sum(float x)
{
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xf, 0xf, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xf, 0xf, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xf, 0xf, true));
    return x;
}

// Delta tile of a hidden layer: dz = dh * GELU'(z) (zero for rows past the
// batch), its column sums over the 16 rows into the bias partials, and the
// bfloat16 copy stored (tr_at) and returned as the next B operand.
__device__ __forceinline__ bf16x4 tr_delta(const f32x4 dh, const f32x4 gpz, bool ok, int lane, int f0, long rr, int Bp,
                                          uint16_t* dT, float* bp, int bstride)
{
    float d[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = ok ? dh[r] * gpz[r] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float s = row16_sum(d[r]);
        if ((lane & 15) == 15) bp[(size_t)(f0 + r) * bstride] = s;
    }
    const bf16x4 h = to_bf16x4(d[0], d[1], d[2], d[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) dT[tr_at(f0 + r, rr, Bp)] = (uint16_t)h[r];
    return h;
}

__global__ __launch_bounds__(64 * kTrSplit) void tr_rows_kernel(TrainArgs ta)
{
    extern __shared__ __align__(16) unsigned char tr_smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x;
    const int g4 = 4 * (lane >> 4);
    const long rr = (long)tile * 16 + (lane & 15);
    const bool ok = rr < ta.B;
    const long src = ta.rows ? (long)ta.rows[ok ? rr : ta.B - 1] : (ok ? rr : ta.B - 1);
    // the row's raw inputs and targets (every wavefront of the tile), in flight with the staging
    float xr[12], tr[4];
#pragma unroll
    for (int i = 0; i < 12; ++i) xr[i] = ta.X[src * kIn + min((i >> 2) * 16 + g4 + (i & 3), kIn - 1)];

#pragma unroll
    for (int o = 0; o < 4; ++o) tr[o] = ta.T[src * kOut + o];
    {
        // eight reads in flight before their writes, the image in rounds of eight
        constexpr int kVec = (int)(kTrLds / 16), kStride = 64 * kTrSplit;
        const uint4* srcv = reinterpret_cast<const uint4*>(ta.img);
        uint4* dst = reinterpret_cast<uint4*>(tr_smem);
        for (int base = 0; base < kVec; base += 8 * kStride) {
            uint4 t[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) t[i] = srcv[min(base + tid + i * kStride, kVec - 1)];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = base + tid + i * kStride;
                if (e < kVec) dst[e] = t[i];
            }
        }
    }
    __syncthreads();
    const bf16x4* F1 = reinterpret_cast<const bf16x4*>(tr_smem + kTrOffF1);
    const bf16x8* F2 = reinterpret_cast<const bf16x8*>(tr_smem + kTrOffF2);
    const bf16x8* F3 = reinterpret_cast<const bf16x8*>(tr_smem + kTrOffF3);
    const bf16x8* F4 = reinterpret_cast<const bf16x8*>(tr_smem + kTrOffF4);
    const bf16x4* B4 = reinterpret_cast<const bf16x4*>(tr_smem + kTrOffB4);
    const bf16x8* B3 = reinterpret_cast<const bf16x8*>(tr_smem + kTrOffB3);
    const bf16x8* B2 = reinterpret_cast<const bf16x8*>(tr_smem + kTrOffB2);
    const float* bias = reinterpret_cast<const float*>(tr_smem + kTrOffBias);
    const float* nrm = reinterpret_cast<const float*>(tr_smem + kTrOffNorm);
    // exchange of a layer's output tiles: buffer q holds tile t of lane l as
    // the (t % 2) half of bf16x8 slot (q 4 + t / 2) 64 + l, so that one read
    // gives the next product's B operand of K block t / 2
    bf16x4* xw = reinterpret_cast<bf16x4*>(tr_smem + kTrOffX);
    const bf16x8* xr8 = reinterpret_cast<const bf16x8*>(tr_smem + kTrOffX);
    auto put = [&](int q, int t, const bf16x4 h) { xw[2 * ((q * 4 + (t >> 1)) * 64 + lane) + (t & 1)] = h; };
    auto get = [&](int q, bf16x8* b) {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) b[kb] = xr8[(q * 4 + kb) * 64 + lane];
    };
    const int Bp = ta.Bp;
    const int ntile = Bp >> 4;
    float* bp = ta.bpart + tile;   // bias partial of column c at bp[c ntile]

    // ---- inputs: features 4 (lane / 16) + q of each 16-feature block, normalised
    bf16x4 xb[3];
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) {
        const int f0 = kb * 16 + g4;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = ok ? (xr[kb * 4 + q] - nrm[f0 + q]) * nrm[48 + f0 + q] : 0.0f;
        }
        xb[kb] = to_bf16x4(v[0], v[1], v[2], v[3]);
        if (kb % kTrSplit == wave) {
#pragma unroll
            for (int q = 0; q < 4; ++q) ta.aT[tr_at(kTrA0 + f0 + q, rr, Bp)] = (uint16_t)xb[kb][q];
        }
    }
    // ---- forward: z = bias + W a, a' = GELU(z) in bfloat16, GELU'(z) kept in
    // registers; this wavefront takes output tiles wave kTrTiles .. + kTrTiles - 1
    f32x4 gz[3][kTrTiles];
    auto hidden = [&](const f32x4 z, int layer, int ob, bf16x4& out, f32x4& gd) {
        float a[4], d[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float gl;
            gelu_and_grad(z[r], gl, d[r]);
            a[r] = ok ? gl : 0.0f;
        }
        out = to_bf16x4(a[0], a[1], a[2], a[3]);
        gd = f32x4{d[0], d[1], d[2], d[3]};
        const int arow = (layer == 0 ? kTrA1 : layer == 1 ? kTrA2 : kTrA3) + ob * 16 + g4;
#pragma unroll
        for (int r = 0; r < 4; ++r) ta.aT[tr_at(arow + r, rr, Bp)] = (uint16_t)out[r];
    };
    bf16x8 b[4];
#pragma unroll
    for (int j = 0; j < kTrTiles; ++j) {
        const int ob = wave * kTrTiles + j;
        f32x4 acc = *reinterpret_cast<const f32x4*>(bias + ob * 16 + g4);
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) acc = mfma_step(F1[(ob * 3 + kb) * 64 + lane], xb[kb], acc);
        bf16x4 h;
        hidden(acc, 0, ob, h, gz[0][j]);
        put(0, ob, h);
    }
    __syncthreads();
    get(0, b);
#pragma unroll
    for (int j = 0; j < kTrTiles; ++j) {
        const int ob = wave * kTrTiles + j;
        f32x4 acc = *reinterpret_cast<const f32x4*>(bias + kHid + ob * 16 + g4);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_step(F2[(ob * 4 + kb) * 64 + lane], b[kb], acc);
        bf16x4 h;
        hidden(acc, 1, ob, h, gz[1][j]);
        put(1, ob, h);
    }
    __syncthreads();
    get(1, b);
#pragma unroll
    for (int j = 0; j < kTrTiles; ++j) {
        const int ob = wave * kTrTiles + j;
        f32x4 acc = *reinterpret_cast<const f32x4*>(bias + 2 * kHid + ob * 16 + g4);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_step(F3[(ob * 4 + kb) * 64 + lane], b[kb], acc);
        bf16x4 h;
        hidden(acc, 2, ob, h, gz[2][j]);
        put(0, ob, h);
    }
    __syncthreads();
    get(0, b);
    // ---- output, loss and its gradient (lanes 0-15 hold the 4 outputs of row
    // lane); every wavefront forms the output gradient, the first stores it
    // with the loss and the output bias partials
    bf16x4 dy = bf16x4{0, 0, 0, 0};
    {
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const int ai = g4 + (lane & 3);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_step(F4[kb * 16 + ai], b[kb], acc);
        const bool out_lane = lane < 16 && ok;
        float d[4];
        double sq = 0.0;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const float y = acc[o] + bias[3 * kHid + o];
            const float tn = (tr[o] - nrm[96 + o]) * nrm[100 + o];
            const float e = y - tn;
            d[o] = out_lane ? 2.0f * e / (float)(ta.B * kOut) : 0.0f;
            sq += out_lane ? (double)(e * e) : 0.0;
        }
        if (lane < 16) dy = to_bf16x4(d[0], d[1], d[2], d[3]);
        if (wave == 0) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
            if (lane == 0) ta.lpart[tile] = sq;
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                float s = d[o];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
                if (lane == 0) bp[(size_t)(3 * kHid + o) * ntile] = s;
            }
            if (lane < 16) {
#pragma unroll
                for (int o = 0; o < 4; ++o) ta.dT[tr_at(kTrD4 + o, rr, Bp)] = (uint16_t)dy[o];
            }
        }
    }
    // ---- backward: dh3 = W4^T dy, then W3^T d3 and W2^T d2, this wavefront's
    // tiles of each, exchanged like the forward's
#pragma unroll
    for (int j = 0; j < kTrTiles; ++j) {
        const int ib = wave * kTrTiles + j;
        const f32x4 dh = mfma_step(B4[ib * 64 + lane], dy, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        put(1, ib, tr_delta(dh, gz[2][j], ok, lane, ib * 16 + g4, rr, Bp, ta.dT + (long)kTrD3 * Bp,
                                     bp + (size_t)2 * kHid * ntile, ntile));
    }
    __syncthreads();
    get(1, b);
#pragma unroll
    for (int j = 0; j < kTrTiles; ++j) {
        const int ib = wave * kTrTiles + j;
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_step(B3[(ib * 4 + kb) * 64 + lane], b[kb], acc);
        put(0, ib, tr_delta(acc, gz[1][j], ok, lane, ib * 16 + g4, rr, Bp, ta.dT + (long)kTrD2 * Bp,
                                     bp + (size_t)kHid * ntile, ntile));
    }
    __syncthreads();
    get(0, b);
#pragma unroll
    for (int j = 0; j < kTrTiles; ++j) {
        const int ib = wave * kTrTiles + j;
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma_step(B2[(ib * 4 + kb) * 64 + lane], b[kb], acc);
        (void)tr_delta(acc, gz[0][j], ok, lane, ib * 16 + g4, rr, Bp, ta.dT + (long)kTrD1 * Bp, bp, ntile);
    }
}

struct GradArgs {
    const uint16_t* aT;       // [kTrARows][Bp]
    const uint16_t* dT;       // [kTrDRows][Bp]
    const float* bpart;       // [kTrBias][ntile]
    const double* lpart;      // [ntile]
    int ntile, Bp;
    float* grad;              // gradient mode: [kNParams] out
    // Adam mode (grad == null): FP32 parameters, moments, bfloat16 copy, the next image
    float* theta;
    float* m;
    float* v;
    uint16_t* theta_h;
    unsigned char* img_next;
    float lr, b1, b2, eps, c1, c2;
    float* loss;              // sum of the squared errors
};

// Adam (bias-corrected, on the FP32 master copy, the bfloat16 copy refreshed)
// on one parameter from its moments m0, v0 and value
// th0 read before; returns the new value.
__device__ __forceinline__ float tr_adam(const GradArgs& g, int idx, float gi, float m0, float v0, float th0)
{
    const float mi = g.b1 * m0 + (1.0f - g.b1) * gi;
    const float vi = g.b2 * v0 + (1.0f - g.b2) * gi * gi;
    g.m[idx] = mi;
    g.v[idx] = vi;
    const float mh = mi / g.c1, vh = vi / g.c2;
    const float th = th0 - g.lr * mh / (sqrtf(vh) + g.eps);
    g.theta[idx] = th;
    g.theta_h[idx] = f2bf(th);
    return th;
}

__global__ __launch_bounds__(64 * kTrGradWaves) void tr_grad_kernel(GradArgs g)
{
    __shared__ f32x4 red[kTrGradWaves][64];
    __shared__ uint16_t Wn[16][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware tiles: workgroups are dealt to the eight XCDs in turn, so the
    // workgroups of XCD x = blockIdx % 8 take the tiles of output block ot = x
    // of W1, W2 and W3 (their deltas read once into that XCD's L2) and input
    // block it = x of W4
    const int t = blockIdx.x;
    const int x = t & 7, jt = t >> 3;
    int layer, ot, it;
    if (jt < 3) {
        layer = 0; ot = x; it = jt;
    } else if (jt < 11) {
        layer = 1; ot = x; it = jt - 3;
    } else if (jt < 19) {
        layer = 2; ot = x; it = jt - 11;
    } else {
        layer = 3; ot = 0; it = x;
    }
    const int nin = layer == 0 ? kIn : kHid, nout = layer == 3 ? kOut : kHid;
    const int offW = layer == 0 ? kOffW1 : layer == 1 ? kOffW2 : layer == 2 ? kOffW3 : kOffW4;
    const int offB = layer == 0 ? kOffB1 : layer == 1 ? kOffB2 : layer == 2 ? kOffB3 : kOffB4;
    const int arow = layer == 0 ? kTrA0 : layer == 1 ? kTrA1 : layer == 2 ? kTrA2 : kTrA3;
    const int drow = layer == 0 ? kTrD1 : layer == 1 ? kTrD2 : layer == 2 ? kTrD3 : kTrD4;
    const bool adam = g.grad == nullptr;
    // ---- everything read before the products: the Adam state of wave 0's
    // four parameters, the bias partials (workgroups of the first input
    // block) and the loss partials (workgroup 0)
    const int i_par = it * 16 + (lane & 15);
    float m0[4] = {0, 0, 0, 0}, v0[4] = {0, 0, 0, 0}, th0[4] = {0, 0, 0, 0};
    if (adam && wave == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = ot * 16 + 4 * (lane >> 4) + r;
            if (o < nout && i_par < nin) {
                const int idx = offW + o * nin + i_par;
                m0[r] = g.m[idx];
                v0[r] = g.v[idx];
                th0[r] = g.theta[idx];
            }
        }
    }
    __shared__ float bsum[16][33];
    const int bf = tid >> 5, bj = tid & 31;         // 32 threads per output of the tile
    const int bo = ot * 16 + bf;
    const int boff = layer * kHid + bo;             // partial column (b4 after the three hidden layers)
    if (it == 0) {
        float sb = 0.0f;
        if (bf < 16 && bo < nout)
            for (int q0 = bj; q0 < g.ntile; q0 += 32 * 8) {   // eight reads in flight, added in tile order
                float pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + 32 * u;
                    pv[u] = q < g.ntile ? g.bpart[(size_t)boff * g.ntile + q] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) sb += pv[u];
            }
        if (bf < 16) bsum[bf][bj] = sb;
    }
    __shared__ double lsum[64 * kTrGradWaves];
    if (t == 0) {
        double sl = 0.0;
        for (int q = tid; q < g.ntile; q += 64 * kTrGradWaves) sl += g.lpart[q];
        lsum[tid] = sl;
    }
    // ---- dW tile: A = d^T (16 outputs x rows), B = a (rows x 16 inputs); rows split over the waves
    const int Bp = g.Bp, per = Bp / kTrGradWaves;
    const bf16x8* Ap = reinterpret_cast<const bf16x8*>(g.dT + tr_at(drow + ot * 16, 0, Bp));   // tile start
    const bf16x8* Bq = reinterpret_cast<const bf16x8*>(g.aT + tr_at(arow + it * 16, 0, Bp));
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int k0 = wave * per, kend = k0 + per;
    const bf16x8 zero8 = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = k0; k < kend; k += 16 * 32) {   // 16 steps of 32 rows, their reads in flight together
        bf16x8 a[16], b[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const bool in = k + q * 32 < kend;
            const int e = ((((k + q * 32) >> 3) + (lane >> 4)) << 4) + (lane & 15);   // row group, feature
            a[q] = in ? Ap[e] : zero8;
            b[q] = in ? Bq[e] : zero8;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = mfma_step(a[q], b[q], acc);
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
        f32x4 s = red[0][lane];
#pragma unroll
        for (int w = 1; w < kTrGradWaves; ++w) s = s + red[w][lane];
        // lane holds dW[ot 16 + 4 (lane / 16) + r][it 16 + lane % 16]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = ot * 16 + 4 * (lane >> 4) + r;
            const bool valid = o < nout && i_par < nin;
            const int idx = offW + o * nin + i_par;
            uint16_t nb = 0;
            if (valid) {
                if (!adam) {
                    g.grad[idx] = s[r];
                } else {
                    nb = f2bf(tr_adam(g, idx, s[r], m0[r], v0[r], th0[r]));
                }
            }
            Wn[4 * (lane >> 4) + r][lane & 15] = nb;
        }
    }
    // ---- bias gradients: a fixed tree over the 32 sums of each output
    if (it == 0) {
        for (int w = 16; w >= 1; w >>= 1) {
            if (bf < 16 && bj < w) bsum[bf][bj] += bsum[bf][bj + w];
            __syncthreads();
        }
        if (bf < 16 && bj == 0 && bo < nout) {
            const int idx = offB + bo;
            if (!adam) {
                g.grad[idx] = bsum[bf][0];
            } else {
                reinterpret_cast<float*>(g.img_next + kTrOffBias)[boff] =
                    tr_adam(g, idx, bsum[bf][0], g.m[idx], g.v[idx], g.theta[idx]);
            }
        }
    }
    if (t == 0) {   // the loss: a fixed tree over the threads' sums
        for (int w = 32 * kTrGradWaves; w >= 1; w >>= 1) {
            if (tid < w) lsum[tid] += lsum[tid + w];
            __syncthreads();
        }
        if (tid == 0) *g.loss = (float)lsum[0];
    }
    if (g.grad) return;
    __syncthreads();
    // ---- the new weights into the next image (this tile's part of every entry holding them)
    if (tid >= 64) return;
    const int gq = tid >> 4, lc = tid & 15;
    unsigned char* img = g.img_next;
    if (layer == 0) {   // W1 forward tile (ot, it): lane holds W[ot 16 + lc][it 16 + 4 gq + q]
        bf16x4 a;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = (short)Wn[lc][4 * gq + q];
        reinterpret_cast<bf16x4*>(img + kTrOffF1)[(ot * 3 + it) * 64 + tid] = a;
        return;
    }
    if (layer == 1 || layer == 2) {
        // forward tile (ot, it / 2), slots of half it % 2: W[ot 16 + lc][it 16 + 4 gq + q]
        bf16x4 f, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f[q] = (short)Wn[lc][4 * gq + q];
            b[q] = (short)Wn[4 * gq + q][lc];
        }
        unsigned char* fw = img + (layer == 1 ? kTrOffF2 : kTrOffF3);
        *reinterpret_cast<bf16x4*>(fw + (size_t)((ot * 4 + (it >> 1)) * 64 + tid) * 16 + (it & 1) * 8) = f;
        // transposed tile (it, ot / 2), slots of half ot % 2: W[ot 16 + 4 gq + q][it 16 + lc]
        unsigned char* bw = img + (layer == 1 ? kTrOffB2 : kTrOffB3);
        *reinterpret_cast<bf16x4*>(bw + (size_t)((it * 4 + (ot >> 1)) * 64 + tid) * 16 + (ot & 1) * 8) = b;
        return;
    }
    // W4: forward entries j < 16 (row j & 3, group j >> 2) of tile it / 2, half it % 2
    if (tid < 16) {
        bf16x4 f;
#pragma unroll
        for (int q = 0; q < 4; ++q) f[q] = (short)Wn[tid & 3][4 * (tid >> 2) + q];
        *reinterpret_cast<bf16x4*>(img + kTrOffF4 + (size_t)((it >> 1) * 16 + tid) * 16 + (it & 1) * 8) = f;
        // W4^T tile it, group 0: W4[q][it 16 + tid]
        bf16x4 b;
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = (short)Wn[q][tid];
        reinterpret_cast<bf16x4*>(img + kTrOffB4)[it * 64 + tid] = b;
    }
}

}  // namespace spmlp
