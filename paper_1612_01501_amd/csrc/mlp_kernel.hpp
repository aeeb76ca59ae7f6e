// Learned surrogate of the cell update: an MLP 16 -> 128 -> 128 -> 16 (SiLU)
// that advances a cell by one macro step of four time steps. Weights are
// BF16 and every product runs on the matrix cores (v_mfma_f32_16x16x16_bf16)
// with FP32 accumulation, batched over cells so each layer is a GEMM.
//
// Layout: a wave owns 16 samples (cells). Activations are kept transposed,
// H^T [features x 16 samples], so the accumulator layout of one layer
// (lane j + 16*(i/4) holds rows i..i+3 of column j) is exactly the B-operand
// layout of the next (lane j + 16*(k/4) holds k..k+3 of column j): no data
// moves between layers. Weights W [out][in] are the A operand, read from LDS
// (row i at lane i%16, four consecutive k per lane).
//
// Parameter order (flat fp32): W1[128][16] b1[128] W2[128][128] b2[128]
// W3[16][128] b3[16].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace infoli {

constexpr int kIn = 16, kHid = 128, kOut = 16, kTargets = 14;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid,
              kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid,
              kNumParams = kOffB3 + kOut;                    // 20,752
// LDS row strides (bf16 elements), padded against bank conflicts
constexpr int kS1 = kIn + 4, kS2 = kHid + 4, kS3 = kHid + 4;
constexpr int kLdsW1 = kHid * kS1, kLdsW2 = kHid * kS2, kLdsW3 = kOut * kS3;
constexpr int kMlpLdsElems = kLdsW1 + kLdsW2 + kLdsW3;     // bf16 elements (42 KB)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16 by the hardware conversion (v_cvt_pk_bf16_f32: round to
// nearest even, two values per instruction; NaN stays NaN)
typedef __bf16 hbf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x4 pack_bf16(f32x4 v) {
    const hbf16x4 h = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
    return __builtin_bit_cast(bf16x4, h);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 hbf16x8 __attribute__((ext_vector_type(8)));

// D += A B over 32 of K (v_mfma_f32_16x16x32_bf16, one instruction for two
// 16x16x16 products). Both operands hold, per lane, eight K slots that the
// instruction pairs up between A and B; the sum over K does not depend on
// which K each slot carries, so the slots take two 16-wide fragments side by
// side: (a0, b0) for K rows k0.. and (a1, b1) for K rows k0 + 16.. in the
// 16x16x16 layout. No activation moves between layers.
__device__ __forceinline__ f32x4 mfma32(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
    const bf16x8s a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const bf16x8s b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(hbf16x8, a),
                                                   __builtin_bit_cast(hbf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float silu_grad_f(float z) {
    const float s = sigmoid_f(z);
    return s * (1.0f + z * (1.0f - s));
}

struct MlpSmem {
    uint16_t* w1;   // [128][kS1]
    uint16_t* w2;   // [128][kS2]
    uint16_t* w3;   // [16][kS3]
};

__device__ __forceinline__ MlpSmem mlp_smem(uint16_t* base) {
    return MlpSmem{base, base + kLdsW1, base + kLdsW1 + kLdsW2};
}

// Copy the bf16 weights (dense [out][in] in global memory) into padded LDS,
// four weights (8 bytes) per access, eight loads in flight per thread before
// their stores. Every matrix offset and padded row start is a multiple of
// four weights.
template <int ROWS, int COLS, int S>
__device__ __forceinline__ void copy_matrix_lds(const uint16_t* __restrict__ src, uint16_t* dst) {
    constexpr int kChunks = ROWS * COLS / 4, kPerRow = COLS / 4, kUnroll = 8;
    const uint2* g = reinterpret_cast<const uint2*>(src);
    for (int e0 = threadIdx.x; e0 < kChunks; e0 += kUnroll * blockDim.x) {
        uint2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int e = e0 + u * blockDim.x;
            if (e < kChunks) v[u] = g[e];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int e = e0 + u * blockDim.x;
            if (e < kChunks) *reinterpret_cast<uint2*>(dst + (e / kPerRow) * S + 4 * (e % kPerRow)) = v[u];
        }
    }
}

__device__ __forceinline__ void load_weights_lds(const uint16_t* __restrict__ wb, MlpSmem s) {
    copy_matrix_lds<kHid, kIn, kS1>(wb + kOffW1, s.w1);
    copy_matrix_lds<kHid, kHid, kS2>(wb + kOffW2, s.w2);
    copy_matrix_lds<kOut, kHid, kS3>(wb + kOffW3, s.w3);
}

// A operand: rows rb*16 .. +15 of W (stride S), columns kb*16 + 4*(lane/16) .. +3
__device__ __forceinline__ bf16x4 a_rows(const uint16_t* w, int S, int rb, int kb) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const bf16x4*>(w + (rb * 16 + (l & 15)) * S + kb * 16 + 4 * (l >> 4));
}

// A operand of the transpose: A[i][k] = W[k][i] for rows ib*16.. of W^T
__device__ __forceinline__ bf16x4 a_cols(const uint16_t* w, int S, int ib, int kb) {
    const int l = threadIdx.x & 63;
    const int i = ib * 16 + (l & 15), k = kb * 16 + 4 * (l >> 4);
    bf16x4 r;
    r[0] = (short)w[(k + 0) * S + i];
    r[1] = (short)w[(k + 1) * S + i];
    r[2] = (short)w[(k + 2) * S + i];
    r[3] = (short)w[(k + 3) * S + i];
    return r;
}

// Bias of the four accumulator rows a lane holds in output block ob.
__device__ __forceinline__ f32x4 bias4(const float* b, int ob) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const f32x4*>(b + ob * 16 + 4 * (l >> 4));
}

// Forward pass of one wave. bx: B operand X^T (features 4*(lane/16).. of
// sample lane%16). Keeps pre-activations z for the backward pass when given.
struct MlpActs {
    f32x4 z1[8], z2[8];
    bf16x4 h1[8], h2[8];
};

__device__ __forceinline__ f32x4 mlp_forward(MlpSmem s, const float* __restrict__ params, bf16x4 bx,
                                             MlpActs* keep, bf16x4* h2_out) {
    bf16x4 h1[8];
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        f32x4 z = mfma16(a_rows(s.w1, kS1, ob, 0), bx, bias4(params + kOffB1, ob));
        f32x4 h;
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = silu_f(z[e]);
        h1[ob] = pack_bf16(h);
        if (keep) {
            keep->z1[ob] = z;
            keep->h1[ob] = h1[ob];
        }
    }
    bf16x4 h2[8];
#pragma unroll
    for (int ob = 0; ob < 8; ++ob) {
        f32x4 z = bias4(params + kOffB2, ob);
#pragma unroll
        for (int kb = 0; kb < 8; kb += 2)
            z = mfma32(a_rows(s.w2, kS2, ob, kb), a_rows(s.w2, kS2, ob, kb + 1), h1[kb], h1[kb + 1], z);
        f32x4 h;
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = silu_f(z[e]);
        h2[ob] = pack_bf16(h);
        if (keep) {
            keep->z2[ob] = z;
            keep->h2[ob] = h2[ob];
        }
    }
    f32x4 y = bias4(params + kOffB3, 0);
#pragma unroll
    for (int kb = 0; kb < 8; kb += 2)
        y = mfma32(a_rows(s.w3, kS3, 0, kb), a_rows(s.w3, kS3, 0, kb + 1), h2[kb], h2[kb + 1], y);
    if (h2_out)
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) h2_out[kb] = h2[kb];
    return y;   // lane holds outputs 4*(lane/16)..+3 of sample lane%16
}

// Weight copies for the matrix cores: bf16 of the fp32 masters.
static __global__ void k_mlp_to_bf16(const float* __restrict__ params, uint16_t* __restrict__ wb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kNumParams) wb[e] = to_bf16(params[e]);
}

// ---------------------------------------------------------------- training
// Transposed activation buffers written by the forward/backward pass, read by
// the weight-gradient GEMMs: [feature][batch] bf16.
struct TrainBufs {
    uint16_t* xT;     // [16][B]
    uint16_t* h1T;    // [128][B]
    uint16_t* h2T;    // [128][B]
    uint16_t* dyT;    // [16][B]
    uint16_t* dz2T;   // [128][B]
    uint16_t* dz1T;   // [128][B]
    float* loss_part; // [B/16] per-wave sums of squared errors
};

// Counter-based index draw: SplitMix64 finaliser (Steele, Lea, Flood 2014)
// of a key mixing the seed, the step and the position in the batch.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// One wave per 16 samples: forward, loss, and back-propagation down to dz1.
// Sample p of the batch is row idx(p) of the normalised data set (xn, tn:
// [N][16] fp32); idx(p) = p when seed == 0, else a hashed draw.
static __global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const float* __restrict__ params,
                                                     const uint16_t* __restrict__ wb,
                                                     const float* __restrict__ xn,
                                                     const float* __restrict__ tn, int64_t n_data,
                                                     int batch, uint64_t seed, uint64_t step,
                                                     TrainBufs buf) {
    __shared__ __align__(16) uint16_t s_w[kMlpLdsElems];
    const MlpSmem s = mlp_smem(s_w);
    load_weights_lds(wb, s);
    __syncthreads();
    const int l = threadIdx.x & 63;
    const int g = l >> 4;                       // feature group of this lane
    const int wave_g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int p = wave_g * 16 + (l & 15);       // position in the batch
    if (wave_g * 16 >= batch) return;           // whole waves only (batch % 16 == 0)
    const int64_t row = seed ? (int64_t)(mix64(seed ^ (step << 32) ^ (uint64_t)p) % (uint64_t)n_data) : p;

    const f32x4 xv = *reinterpret_cast<const f32x4*>(xn + row * 16 + 4 * g);
    const f32x4 tv = *reinterpret_cast<const f32x4*>(tn + row * 16 + 4 * g);
    const bf16x4 bx = pack_bf16(xv);
    MlpActs act;
    const f32x4 y = mlp_forward(s, params, bx, &act, nullptr);

    // loss = mean over batch and the 14 targets of (y - t)^2
    const float scale = 2.0f / (float)(batch * kTargets);
    f32x4 dy;
    float sq = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool on = 4 * g + e < kTargets;
        const float d = on ? y[e] - tv[e] : 0.0f;
        sq += d * d;
        dy[e] = d * scale;
    }
    for (int m = 32; m > 0; m >>= 1) sq += __shfl_xor(sq, m, 64);
    if (l == 0) buf.loss_part[wave_g] = sq;
    const bf16x4 dyq = pack_bf16(dy);

    // dz2 = (W3^T dy) * silu'(z2)
    bf16x4 dz2q[8];
#pragma unroll
    for (int ib = 0; ib < 8; ++ib) {
        f32x4 dh = mfma16(a_cols(s.w3, kS3, ib, 0), dyq, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        f32x4 dz;
#pragma unroll
        for (int e = 0; e < 4; ++e) dz[e] = dh[e] * silu_grad_f(act.z2[ib][e]);
        dz2q[ib] = pack_bf16(dz);
    }
    // dz1 = (W2^T dz2) * silu'(z1)
    bf16x4 dz1q[8];
#pragma unroll
    for (int ib = 0; ib < 8; ++ib) {
        f32x4 dh = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < 8; kb += 2)
            dh = mfma32(a_cols(s.w2, kS2, ib, kb), a_cols(s.w2, kS2, ib, kb + 1), dz2q[kb], dz2q[kb + 1], dh);
        f32x4 dz;
#pragma unroll
        for (int e = 0; e < 4; ++e) dz[e] = dh[e] * silu_grad_f(act.z1[ib][e]);
        dz1q[ib] = pack_bf16(dz);
    }

    // transposed stores: element (feature f, position p)
    auto put = [&](uint16_t* dst, int fb, bf16x4 v) {
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[(int64_t)(fb * 16 + 4 * g + e) * batch + p] = (uint16_t)v[e];
    };
    put(buf.xT, 0, bx);
    put(buf.dyT, 0, dyq);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        put(buf.h1T, b, act.h1[b]);
        put(buf.h2T, b, act.h2[b]);
        put(buf.dz2T, b, dz2q[b]);
        put(buf.dz1T, b, dz1q[b]);
    }
}

// Weight and bias gradients as GEMMs over the batch: one wave per 16x16
// output tile and slice of the batch (split K), each slice summed in order
// into its own partial gradient [kGradSplits][kNumParams]; the partials are
// added in slice order afterwards (deterministic). Tiles: dW1 8, dW2 64,
// dW3 8, then bias rows as products with a ones vector: db1 8, db2 8, db3 1.
constexpr int kGradTiles = 8 + 64 + 8 + 8 + 8 + 1;
constexpr int kGradSplits = 16;

static __global__ __launch_bounds__(64) void k_mlp_wgrad(TrainBufs buf, int batch, float* __restrict__ grad_part,
                                                  float* __restrict__ loss_out) {
    const int t = blockIdx.x % kGradTiles;
    const int split = blockIdx.x / kGradTiles;
    float* grad = grad_part + (int64_t)split * kNumParams;
    const int l = threadIdx.x & 63;
    const int g = l >> 4;
    const uint16_t* A;   // [rows][batch]
    const uint16_t* Bm;  // [cols][batch] or nullptr for the ones vector
    int ib, jb, ncols, off;
    if (t < 8) {                 // dW1 = dz1^T x : [128][16]
        A = buf.dz1T; Bm = buf.xT; ib = t; jb = 0; ncols = kIn; off = kOffW1;
    } else if (t < 72) {         // dW2 = dz2^T h1 : [128][128]
        A = buf.dz2T; Bm = buf.h1T; ib = (t - 8) / 8; jb = (t - 8) % 8; ncols = kHid; off = kOffW2;
    } else if (t < 80) {         // dW3 = dy^T h2 : [16][128]
        A = buf.dyT; Bm = buf.h2T; ib = 0; jb = t - 72; ncols = kHid; off = kOffW3;
    } else if (t < 88) {         // db1
        A = buf.dz1T; Bm = nullptr; ib = t - 80; jb = 0; ncols = 1; off = kOffB1;
    } else if (t < 96) {         // db2
        A = buf.dz2T; Bm = nullptr; ib = t - 88; jb = 0; ncols = 1; off = kOffB2;
    } else {                     // db3
        A = buf.dyT; Bm = nullptr; ib = 0; jb = 0; ncols = 1; off = kOffB3;
    }
    const bf16x4 ones = {(short)0x3f80, (short)0x3f80, (short)0x3f80, (short)0x3f80};
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const uint16_t* arow = A + (int64_t)(ib * 16 + (l & 15)) * batch + 4 * g;
    const uint16_t* brow = Bm ? Bm + (int64_t)(jb * 16 + (l & 15)) * batch + 4 * g : nullptr;
    const int kb = batch / 16;
    const int k0 = (int)((int64_t)split * kb / kGradSplits), k1 = (int)((int64_t)(split + 1) * kb / kGradSplits);
    for (int k = 16 * k0; k < 16 * k1; k += 16) {
        const bf16x4 av = *reinterpret_cast<const bf16x4*>(arow + k);
        const bf16x4 bv = Bm ? *reinterpret_cast<const bf16x4*>(brow + k) : ones;
        acc = mfma16(av, bv, acc);
    }
    // lane holds rows ib*16 + 4g + e, column jb*16 + l%16
    if (ncols == 1) {
        if ((l & 15) == 0)
#pragma unroll
            for (int e = 0; e < 4; ++e) grad[off + ib * 16 + 4 * g + e] = acc[e];
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) grad[off + (ib * 16 + 4 * g + e) * ncols + jb * 16 + (l & 15)] = acc[e];
    }
    if (t == 0 && split == 0 && loss_out) {   // whole wave: strided partial sums, fixed butterfly
        float s = 0.0f;
        for (int w = l; w < batch / 16; w += 64) s += buf.loss_part[w];
        for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
        if (l == 0) *loss_out = s / (float)(batch * kTargets);
    }
}

// Sum of the split-K partial gradients, in slice order.
__device__ __forceinline__ float grad_sum(const float* __restrict__ part, int splits, int e) {
    float gr = part[e];
    for (int sp = 1; sp < splits; ++sp) gr += part[(int64_t)sp * kNumParams + e];
    return gr;
}

static __global__ void k_grad_reduce(const float* __restrict__ part, int splits, float* __restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kNumParams) grad[e] = grad_sum(part, splits, e);
}

// Adam (Kingma and Ba, 2015) on the fp32 masters, then their bf16 copies;
// the gradient is the sum of `splits` partials [splits][kNumParams].
static __global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, int splits, uint16_t* __restrict__ wb, float lr, float b1,
                       float b2, float eps, float corr1, float corr2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNumParams) return;
    const float gr = grad_sum(grad, splits, e);
    const float mm = b1 * m[e] + (1.0f - b1) * gr;
    const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    const float upd = lr * (mm / corr1) / (sqrtf(vv / corr2) + eps);
    const float nw = w[e] - upd;
    w[e] = nw;
    wb[e] = to_bf16(nw);
}

// Plain forward over a batch (x: [B][16] normalised) -> y [B][16].
static __global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params,
                                                     const uint16_t* __restrict__ wb,
                                                     const float* __restrict__ x, int batch,
                                                     float* __restrict__ y) {
    __shared__ __align__(16) uint16_t s_w[kMlpLdsElems];
    const MlpSmem s = mlp_smem(s_w);
    load_weights_lds(wb, s);
    __syncthreads();
    const int l = threadIdx.x & 63;
    const int g = l >> 4;
    const int wave_g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave_g * 16 >= batch) return;
    const int p = wave_g * 16 + (l & 15);
    const f32x4 xv = *reinterpret_cast<const f32x4*>(x + (int64_t)p * 16 + 4 * g);
    const f32x4 out = mlp_forward(s, params, pack_bf16(xv), nullptr, nullptr);
    *reinterpret_cast<f32x4*>(y + (int64_t)p * 16 + 4 * g) = out;
}

}  // namespace infoli
