// Surrogate MLP 4-128-128-3 (SiLU) on gfx950 matrix cores.
//
// The network maps normalised Hamiltonian parameters (beta, Jx, Jy, h) to
// normalised equilibrium observables; it steers the parameter optimisation
// of the paper's optimisation experiments (Results) while Monte Carlo checks
// its answers.  Weights and activations enter the matrix cores as BF16
// (round to nearest even from FP32), products accumulate in FP32
// (gfx950's v_mfma_f32_16x16x32_bf16: a 16x16 tile per wave, K = 32).  Rounding points (the oracle mirrors them):
//   forward : xb = bf16(x); z1 = W1b xb + b1; h1 = bf16(silu z1);
//             z2 = W2b h1 + b2; h2 = bf16(silu z2); y = W3b h2 + b3
//   backward: dY = 2 w (y - t) / B (FP32);  dW3 = sum dY h2, dH2 = W3b^T dY;
//             dz2 = dH2 silu'(z2); dz2b = bf16(dz2);
//             dW2 = sum dz2b h1 (MFMA), dH1 = W2b^T dz2b (MFMA);
//             dz1 = dH1 silu'(z1); dW1 = sum dz1 xb; dx = W1b^T dz1;
//             bias gradients are FP32 sums of the unrounded dz.
// Batch sums are per-workgroup partials reduced in a fixed order, so the
// result does not depend on scheduling.  Each workgroup (4 waves) handles
// 64 samples, 16 per wave.
#include "spinmc_internal.hpp"

namespace spinmc {

namespace {

constexpr int kIn = 4, kH = 128, kOut = 3;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              oW3 = ob2 + kH, ob3 = oW3 + kOut * kH, kNP = ob3 + kOut;
constexpr int kSamplesPerWG = 64;
constexpr int kPadK = 8;             // LDS row padding (bf16 elements) against bank conflicts
constexpr int kK1 = 32;              // layer-1 K (4 inputs, zero-padded to one MFMA step)
constexpr int kS1 = kK1 + kPadK;     // row stride of layer-1 tiles
constexpr int kS2 = kH + kPadK;      // row stride of K=128 tiles
constexpr int kST = kSamplesPerWG + kPadK;  // row stride of sample-major transposed tiles

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

// Operand fragment of a 16 x 32 tile (rows r, k in [k0, k0 + 32)) from a
// row-major bf16 tile: lane l holds row l % 16, k0 + 8 (l / 16) .. + 7, one
// 16-byte load (row strides and k0 keep it 16-byte aligned).
__device__ __forceinline__ bf16x8 frag(const uint16_t* base, int stride, int k0) {
    const int l = threadIdx.x & 63;
    const uint16_t* p = base + (l & 15) * stride + k0 + 8 * (l >> 4);
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ float4v mfma(bf16x8 a, bf16x8 b, float4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Weights into LDS as BF16, [out][in] rows (B^T layout of the matrix cores).
// 16-byte loads, all of a thread's loads issued before their conversions.
__device__ void stage_weights(const float* P, uint16_t* w1, uint16_t* w2, uint16_t* w3,
                              bool need_w2) {
    // W1: 128 x 4 -> rows of kK1 (k >= 4 zero); one float4 per row
    for (int n = threadIdx.x; n < kH; n += blockDim.x) {
        const float4 v = *reinterpret_cast<const float4*>(P + oW1 + n * kIn);
        uint16_t* r = w1 + n * kS1;
        r[0] = f2bf(v.x);
        r[1] = f2bf(v.y);
        r[2] = f2bf(v.z);
        r[3] = f2bf(v.w);
#pragma unroll
        for (int k = kIn; k < kK1; ++k) r[k] = 0;
    }
    if (need_w2) {
        constexpr int kV = kH * kH / 4;  // float4 of W2
        const float4* src = reinterpret_cast<const float4*>(P + oW2);
        for (int i0 = threadIdx.x; i0 < kV; i0 += 16 * blockDim.x) {
            float4 v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                v[u] = i < kV ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i >= kV) break;
                const int n = (4 * i) >> 7, k = (4 * i) & 127;
                const uint32_t lo = (uint32_t)f2bf(v[u].x) | ((uint32_t)f2bf(v[u].y) << 16);
                const uint32_t hi = (uint32_t)f2bf(v[u].z) | ((uint32_t)f2bf(v[u].w) << 16);
                *reinterpret_cast<uint2*>(w2 + n * kS2 + k) = make_uint2(lo, hi);
            }
        }
    }
    // W3: 3 x 128 -> 16 rows (rows >= 3 zero)
    for (int i = threadIdx.x; i < 16 * kH / 4; i += blockDim.x) {
        const int n = (4 * i) >> 7, k = (4 * i) & 127;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (n < kOut) v = *reinterpret_cast<const float4*>(P + oW3 + n * kH + k);
        const uint32_t lo = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
        const uint32_t hi = (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
        *reinterpret_cast<uint2*>(w3 + n * kS2 + k) = make_uint2(lo, hi);
    }
}

// Output layer for the wave's 16 samples from h2 (bf16 tile): lane holds
// y[row = 4(l/16)+i][col = l%16] (cols >= 3 are padding).
__device__ __forceinline__ float4v out_layer(const uint16_t* h2, const uint16_t* w3) {
    float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < kH / 32; ++kt) acc = mfma(frag(h2, kS2, 32 * kt), frag(w3, kS2, 32 * kt), acc);
    return acc;
}

}  // namespace

// --------------------------------------------------------------- forward
__global__ void __launch_bounds__(256) k_mlp_fwd(const float* P, const float* x, int B, float* y,
                                                 float* act) {
    __shared__ __align__(16) uint16_t w1[kH * kS1];
    __shared__ __align__(16) uint16_t w2[kH * kS2];
    __shared__ __align__(16) uint16_t w3[16 * kS2];
    __shared__ __align__(16) uint16_t xa[4][16 * kS1];
    __shared__ __align__(16) uint16_t h1[4][16 * kS2];
    __shared__ __align__(16) uint16_t h2[4][16 * kS2];
    stage_weights(P, w1, w2, w3, true);
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int s0 = blockIdx.x * kSamplesPerWG + wave * 16;
    for (int i = l; i < 16 * kK1; i += 64) {
        const int r = i / kK1, k = i % kK1;
        const int s = s0 + r;
        xa[wave][r * kS1 + k] = (k < kIn && s < B) ? f2bf(x[(size_t)s * kIn + k]) : (uint16_t)0;
    }
    __syncthreads();
    const int col = l & 15, rb = 4 * (l >> 4);
    // layer 1 (K = 4, zero-padded to 32)
#pragma unroll
    for (int nt = 0; nt < kH / 16; ++nt) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag(xa[wave], kS1, 0), frag(w1 + nt * 16 * kS1, kS1, 0), acc);
        const int n = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = acc[i] + P[ob1 + n];
            const int s = s0 + rb + i;
            if (act && s < B) act[(size_t)s * 2 * kH + n] = z;
            h1[wave][(rb + i) * kS2 + n] = f2bf(silu(z));
        }
    }
    __syncthreads();
    // layer 2 (K = 128)
#pragma unroll
    for (int nt = 0; nt < kH / 16; ++nt) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < kH / 32; ++kt)
            acc = mfma(frag(h1[wave], kS2, 32 * kt), frag(w2 + nt * 16 * kS2, kS2, 32 * kt), acc);
        const int n = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = acc[i] + P[ob2 + n];
            const int s = s0 + rb + i;
            if (act && s < B) act[(size_t)s * 2 * kH + kH + n] = z;
            h2[wave][(rb + i) * kS2 + n] = f2bf(silu(z));
        }
    }
    __syncthreads();
    if (!y) return;  // training steps keep only the pre-activations
    const float4v o = out_layer(h2[wave], w3);
    if (col < kOut) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = s0 + rb + i;
            if (s < B) y[(size_t)s * kOut + col] = o[i] + P[ob3 + col];
        }
    }
}

// -------------------------------------------------------------- backward
// Per-workgroup partial gradients into part[wg][kNP + 1] (last: loss), and
// input gradients dx (optional).
__global__ void __launch_bounds__(256) k_mlp_bwd(const float* P, const float* x, const float* act,
                                                 const float* t, const float* w, int B,
                                                 float* part, float* dx) {
    __shared__ __align__(16) uint16_t w2t[kH * kS2];      // W2^T: [in][out]
    __shared__ __align__(16) uint16_t w3[16 * kS2];
    __shared__ __align__(16) uint16_t w1[kH * kS1];
    __shared__ __align__(16) uint16_t h1t[kH * kST];      // h1^T: [neuron][sample]
    __shared__ __align__(16) uint16_t dz2t[kH * kST];     // dz2b^T: [neuron][sample]
    __shared__ __align__(16) uint16_t dz2[kSamplesPerWG * kS2];  // dz2b: [sample][neuron]
    __shared__ __align__(16) uint16_t h2[4][16 * kS2];
    constexpr int kSZ = kH + 4;
    __shared__ __align__(16) float dz1[kSamplesPerWG * kSZ];
    __shared__ float dY[kSamplesPerWG][4];
    __shared__ float xs[kSamplesPerWG][kIn];  // bf16-rounded inputs, as float
    __shared__ float red[256];
    stage_weights(P, w1, nullptr, w3, false);
    {
        constexpr int kV = kH * kH / 4;
        const float4* src = reinterpret_cast<const float4*>(P + oW2);
        for (int i0 = threadIdx.x; i0 < kV; i0 += 16 * blockDim.x) {
            float4 v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                v[u] = i < kV ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i >= kV) break;
                const int o = (4 * i) >> 7, in = (4 * i) & 127;
                w2t[(in + 0) * kS2 + o] = f2bf(v[u].x);
                w2t[(in + 1) * kS2 + o] = f2bf(v[u].y);
                w2t[(in + 2) * kS2 + o] = f2bf(v[u].z);
                w2t[(in + 3) * kS2 + o] = f2bf(v[u].w);
            }
        }
    }
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int base = blockIdx.x * kSamplesPerWG;
    for (int i = threadIdx.x; i < kSamplesPerWG * kIn; i += blockDim.x) {
        const int gs = base + i / kIn;
        xs[i / kIn][i % kIn] = gs < B ? bf2f(f2bf(x[(size_t)gs * kIn + i % kIn])) : 0.f;
    }
    // h1 (transposed) and h2 from the stored pre-activations
    {
        constexpr int kV = kSamplesPerWG * kH / 4;  // float4 per layer
        static_assert(kV % 256 == 0, "act staging assumes 256 threads");
        float4 z1[kV / 256], z2[kV / 256];
#pragma unroll
        for (int u = 0; u < kV / 256; ++u) {
            const int i = threadIdx.x + 256 * u;
            const int sm = (4 * i) >> 7, n = (4 * i) & 127;
            const int gs = base + sm;
            z1[u] = z2[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gs < B) {
                z1[u] = *reinterpret_cast<const float4*>(act + (size_t)gs * 2 * kH + n);
                z2[u] = *reinterpret_cast<const float4*>(act + (size_t)gs * 2 * kH + kH + n);
            }
        }
#pragma unroll
        for (int u = 0; u < kV / 256; ++u) {
            const int i = threadIdx.x + 256 * u;
            const int sm = (4 * i) >> 7, n = (4 * i) & 127;
            const bool in_b = base + sm < B;
            const float a1[4] = {z1[u].x, z1[u].y, z1[u].z, z1[u].w};
            const float a2[4] = {z2[u].x, z2[u].y, z2[u].z, z2[u].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                h1t[(n + c) * kST + sm] = in_b ? f2bf(silu(a1[c])) : (uint16_t)0;
                h2[sm >> 4][(sm & 15) * kS2 + n + c] = in_b ? f2bf(silu(a2[c])) : (uint16_t)0;
            }
        }
    }
    __syncthreads();
    // recompute y for the wave's samples, then dY and the loss
    const int col = l & 15, rb = 4 * (l >> 4);
    const int s0 = wave * 16;
    const float4v o = out_layer(h2[wave], w3);
    float lossp = 0.f;
    if (col < 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = s0 + rb + i, gs = base + s;
            float d = 0.f;
            if (col < kOut && gs < B) {
                const float yv = o[i] + P[ob3 + col];
                const float e = yv - t[(size_t)gs * kOut + col];
                lossp += w[col] * e * e;
                d = 2.0f * w[col] * e / (float)B;
            }
            dY[s][col] = d;
        }
    }
    red[threadIdx.x] = lossp;
    __syncthreads();
    // dH2 = W3b^T dY, dz2 = dH2 silu'(z2); eight pre-activations per lane
    // loaded before their use
    static_assert((kSamplesPerWG * kH) % (8 * 256) == 0, "dz2 batches assume 256 threads");
    for (int i0 = threadIdx.x; i0 < kSamplesPerWG * kH; i0 += 8 * 256) {
        float z2v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 256 * u;
            const int gs = base + (i >> 7);
            z2v[u] = gs < B ? act[(size_t)gs * 2 * kH + kH + (i & 127)] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 256 * u;
            const int s = i >> 7, n = i & 127;
            float d = 0.f;
            if (base + s < B) {
                float dh = 0.f;
#pragma unroll
                for (int j = 0; j < kOut; ++j) dh += dY[s][j] * bf2f(w3[j * kS2 + n]);
                d = dh * dsilu(z2v[u]);
            }
            const uint16_t db = f2bf(d);
            dz2t[n * kST + s] = db;
            dz2[s * kS2 + n] = db;
            dz1[s * kSZ + n] = d;  // unrounded dz2, for db2 (dz1 is computed later)
        }
    }
    __syncthreads();
    float* pg = part + (size_t)blockIdx.x * (kNP + 1);
    // dW2 = dz2b^T h1 (M = out neuron, N = in neuron, K = 64 samples): wave
    // owns out-tiles 2*wave, 2*wave+1
    for (int mt = 2 * wave; mt < 2 * wave + 2; ++mt) {
#pragma unroll
        for (int nt = 0; nt < kH / 16; ++nt) {
            float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < kSamplesPerWG / 32; ++kt)
                acc = mfma(frag(dz2t + mt * 16 * kST, kST, 32 * kt),
                           frag(h1t + nt * 16 * kST, kST, 32 * kt), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                pg[oW2 + (mt * 16 + rb + i) * kH + nt * 16 + col] = acc[i];
        }
    }
    // dW3, db3 (VALU): out j, neuron n
    for (int i = threadIdx.x; i < kOut * kH; i += blockDim.x) {
        const int j = i >> 7, n = i & 127;
        float s = 0.f;
        for (int q = 0; q < kSamplesPerWG; ++q) s += dY[q][j] * bf2f(h2[q >> 4][(q & 15) * kS2 + n]);
        pg[oW3 + j * kH + n] = s;
    }
    if (threadIdx.x < kOut) {
        float s = 0.f;
        for (int q = 0; q < kSamplesPerWG; ++q) s += dY[q][threadIdx.x];
        pg[ob3 + threadIdx.x] = s;
    }
    // db2 = sum of the unrounded dz2 (zero for samples past B)
    if (threadIdx.x < kH) {
        const int n = threadIdx.x;
        float s = 0.f;
        for (int q = 0; q < kSamplesPerWG; ++q) s += dz1[q * kSZ + n];
        pg[ob2 + n] = s;
    }
    __syncthreads();
    // dH1 = dz2b W2b (the wave's 16 samples), dz1 = dH1 silu'(z1)
#pragma unroll
    for (int nt = 0; nt < kH / 16; ++nt) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < kH / 32; ++kt)
            acc = mfma(frag(dz2 + s0 * kS2, kS2, 32 * kt), frag(w2t + nt * 16 * kS2, kS2, 32 * kt),
                       acc);
        const int n = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = s0 + rb + i, gs = base + s;
            dz1[s * kSZ + n] = gs < B ? acc[i] * dsilu(act[(size_t)gs * 2 * kH + n]) : 0.f;
        }
    }
    __syncthreads();
    // dW1, db1 (VALU) and dx
    for (int i = threadIdx.x; i < kH * (kIn + 1); i += blockDim.x) {
        const int n = i / (kIn + 1), k = i % (kIn + 1);
        float s = 0.f;
        for (int q = 0; q < kSamplesPerWG; ++q)  // dz1 is zero for samples past B
            s += dz1[q * kSZ + n] * (k < kIn ? xs[q][k] : 1.0f);
        if (k < kIn)
            pg[oW1 + n * kIn + k] = s;
        else
            pg[ob1 + n] = s;
    }
    if (dx) {
        for (int i = threadIdx.x; i < kSamplesPerWG * kIn; i += blockDim.x) {
            const int q = i >> 2, k = i & 3;
            const int gs = base + q;
            if (gs >= B) continue;
            float s = 0.f;
            for (int n = 0; n < kH; ++n) s += dz1[q * kSZ + n] * bf2f(w1[n * kS1 + k]);
            dx[(size_t)gs * kIn + k] = s;
        }
    }
    // loss partial
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) pg[kNP] = red[0] / (float)B;
}

// Fixed-order sum of the per-workgroup partials.
__global__ void k_mlp_reduce(const float* part, int n_wg, float* grad, float* loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kNP) return;
    float s = 0.f;
    for (int g = 0; g < n_wg; ++g) s += part[(size_t)g * (kNP + 1) + i];
    if (i < kNP)
        grad[i] = s;
    else if (loss)
        *loss = s;
}

__global__ void k_mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// The fixed-order sum of k_mlp_reduce and the Adam update of k_mlp_adam in
// one pass over the parameters (the same arithmetic in the same order).
__global__ void k_mlp_reduce_adam(const float* part, int n_wg, float* grad, float* loss,
                                  float* p, float* m, float* v, float lr, float b1, float b2,
                                  float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kNP) return;
    float gi = 0.f;
    for (int g = 0; g < n_wg; ++g) gi += part[(size_t)g * (kNP + 1) + i];
    if (i == kNP) {
        if (loss) *loss = gi;
        return;
    }
    if (grad) grad[i] = gi;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_mlp_train_step(float* params, const float* x, const float* t, const float* w,
                                 int B, float* grad, float* m, float* v, int step, float lr,
                                 float b1, float b2, float eps, float* loss, float* act,
                                 float* scratch, hipStream_t s) {
    const int g = (B + kSamplesPerWG - 1) / kSamplesPerWG;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(256), 0, s, params, x, B, (float*)nullptr, act);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_bwd, dim3(g), dim3(256), 0, s, params, x, act, t, w, B, scratch,
                       (float*)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, scratch, g,
                       grad, loss, params, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const float* x, int B, float* y, float* act,
                              hipStream_t s) {
    const int g = (B + kSamplesPerWG - 1) / kSamplesPerWG;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(256), 0, s, params, x, B, y, act);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* params, const float* x, const float* act,
                               const float* t, const float* w, int B, float* grad, float* dx,
                               float* loss, float* scratch, hipStream_t s) {
    const int g = (B + kSamplesPerWG - 1) / kSamplesPerWG;
    hipLaunchKernelGGL(k_mlp_bwd, dim3(g), dim3(256), 0, s, params, x, act, t, w, B, scratch, dx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, scratch, g,
                       grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, int n, int step,
                           float lr, float b1, float b2, float eps, hipStream_t s) {
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((n + 255) / 256), dim3(256), 0, s, params, grad, m, v, n,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

int mlp_num_params() { return kNP; }
int mlp_scratch_floats(int B) { return ((B + kSamplesPerWG - 1) / kSamplesPerWG) * (kNP + 1); }

}  // namespace spinmc
