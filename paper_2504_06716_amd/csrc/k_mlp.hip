// Learned freeze proposer: a small MLP (32 -> 64 -> 64 -> 1) over the last
// eight logged gradient-norm averages of each Gaussian, proposing Gaussians
// for the freeze map; the freeze rule of Section 3.2.1 vetoes proposals
// whose averages are far above its thresholds.  (A project extension: the
// paper has no such model.)
//
//   K11a push:      ring[slot][q][i] = bf16(min(ema[q][i], 1e30))
//   K11b stats:     per-feature sum and sum of squares of log10 features
//   K11c features:  x[i][4j+q] = bf16((log10(ring[(head-j)&7][q][i] + 1e-12) - mean) / std)
//   K11d forward:   both hidden layers on bf16 matrix cores (16x16x32 MFMA,
//                   float32 accumulation), bias + ReLU in registers, the
//                   first hidden layer re-rounded to bf16 through LDS, the
//                   output unit as a float32 dot product
//   K11e bce:       dL/dz = (sigmoid(z) - y) / n and the loss (fixed order)
//   K11f backward:  weight gradients on bf16 matrix cores (split-bf16 for
//                   the derivative operands), per-block partials summed in
//                   block order (deterministic)
//   K11g adam:      float32 master weights, bf16 copies of W1 and W2
//   K11h propose:   z > threshold and not vetoed
#include "gsta_internal.h"

namespace gsta {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {   // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ float feature(const uint16_t* __restrict__ ring, int64_t n, int head, int f, int64_t i,
                                        const float* __restrict__ mean, const float* __restrict__ stdv) {
    const int j = f >> 2, q = f & 3;
    const float r = from_bf16(ring[((int64_t)((head - j) & 7) * 4 + q) * n + i]);
    const float lg = log10f(r + 1e-12f);
    return mean ? (lg - mean[f]) / stdv[f] : lg;
}

__global__ __launch_bounds__(256) void k_traj_push(const float* __restrict__ ema, int64_t n,
                                                   uint16_t* __restrict__ ring, int slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) ring[((int64_t)slot * 4 + q) * n + i] = to_bf16(fminf(ema[q * n + i], 1e30f));
}

// Per block: sum and sum of squares of the unstandardised features; thread
// t owns feature t & 31 for the Gaussians t >> 5, +8, +16, ...
__global__ __launch_bounds__(256) void k_mlp_stats(const uint16_t* __restrict__ ring, int64_t n, int head,
                                                   double* __restrict__ part) {
    __shared__ double s_a[256], s_b[256];
    const int f = threadIdx.x & 31, r0 = threadIdx.x >> 5;
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 8 + r0; i < n; i += (int64_t)gridDim.x * 8) {
        const double x = (double)feature(ring, n, head, f, i, nullptr, nullptr);
        a += x;
        b += x * x;
    }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x < 32) {
        double ta = 0.0, tb = 0.0;
        for (int k = 0; k < 8; ++k) {
            ta += s_a[k * 32 + threadIdx.x];
            tb += s_b[k * 32 + threadIdx.x];
        }
        part[(int64_t)blockIdx.x * 64 + threadIdx.x] = ta;
        part[(int64_t)blockIdx.x * 64 + 32 + threadIdx.x] = tb;
    }
}

__global__ __launch_bounds__(64) void k_mlp_stats_final(const double* __restrict__ part, int nblocks,
                                                        double* __restrict__ sums) {
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) acc += part[(int64_t)b * 64 + t];
    sums[t] += acc;
}

__global__ __launch_bounds__(256) void k_mlp_features(const uint16_t* __restrict__ ring, int64_t n, int head,
                                                      const float* __restrict__ mean, const float* __restrict__ stdv,
                                                      uint16_t* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t w[16];
#pragma unroll
    for (int f = 0; f < 32; f += 2) {
        const uint32_t lo = to_bf16(feature(ring, n, head, f, i, mean, stdv));
        const uint32_t hi = to_bf16(feature(ring, n, head, f + 1, i, mean, stdv));
        w[f >> 1] = lo | (hi << 16);
    }
    uint4* dst = reinterpret_cast<uint4*>(x + i * 32);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// One wave per tile of 16 samples.  MFMA 16x16x32 operand layout (lane l):
// A row l & 15, columns 8 (l >> 4) .. +7; B column l & 15, rows
// 8 (l >> 4) .. +7; result column l & 15, rows 4 (l >> 4) .. +3.
__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t* __restrict__ wb, const float* __restrict__ wf,
                                                     const uint16_t* __restrict__ x, int64_t n,
                                                     float* __restrict__ logits, uint16_t* __restrict__ h1_out,
                                                     float* __restrict__ h2_out) {
    __shared__ __attribute__((aligned(16))) uint16_t s_w1[64 * 32];
    __shared__ __attribute__((aligned(16))) uint16_t s_w2[64 * 64];
    __shared__ float s_b1[64], s_b2[64], s_w3[64];
    __shared__ __attribute__((aligned(16))) uint16_t s_h1[4][16 * 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int k = tid; k < 64 * 32 / 8; k += 256)
        reinterpret_cast<uint4*>(s_w1)[k] = reinterpret_cast<const uint4*>(wb)[k];
    for (int k = tid; k < 64 * 64 / 8; k += 256)
        reinterpret_cast<uint4*>(s_w2)[k] = reinterpret_cast<const uint4*>(wb + 2048)[k];
    if (tid < 64) {
        s_b1[tid] = wf[kMlpB1 + tid];
        s_b2[tid] = wf[kMlpB2 + tid];
        s_w3[tid] = wf[kMlpW3 + tid];
    }
    __syncthreads();
    const float b3 = wf[kMlpB3];
    const int row = lane & 15, grp = lane >> 4;
    uint16_t* h1t = s_h1[wid];
    const int64_t ntiles = (n + 15) / 16;
    // every wave of the block runs the same iterations (tiles past the end
    // compute on zeros and write nothing), so block barriers are safe
    for (int64_t t0 = (int64_t)blockIdx.x * 4; t0 < ntiles; t0 += (int64_t)gridDim.x * 4) {
        const int64_t s0 = (t0 + wid) * 16;
        // ---- layer 1: [16 x 32] x [32 x 64] ----
        uint4 av = make_uint4(0u, 0u, 0u, 0u);
        if (s0 + row < n) av = *reinterpret_cast<const uint4*>(x + (s0 + row) * 32 + 8 * grp);
        const bf16x8 a1 = __builtin_bit_cast(bf16x8, av);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int u = 16 * nb + row;
            const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(s_w1 + u * 32 + 8 * grp));
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float h = fmaxf(acc[r] + s_b1[u], 0.f);
                h1t[(4 * grp + r) * 64 + u] = to_bf16(h);
            }
        }
        __syncthreads();
        if (h1_out) {
            // 16 rows of 128 bytes, 8 lanes per row
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int c = lane + 64 * k, sr = c >> 3, part = c & 7;
                if (s0 + sr < n)
                    reinterpret_cast<uint4*>(h1_out + (s0 + sr) * 64)[part] =
                        reinterpret_cast<const uint4*>(h1t + sr * 64)[part];
            }
        }
        // ---- layer 2: [16 x 64] x [64 x 64] ----
        const bf16x8 a20 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(h1t + row * 64 + 8 * grp));
        const bf16x8 a21 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(h1t + row * 64 + 32 + 8 * grp));
        float zp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int u = 16 * nb + row;
            const bf16x8 b0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(s_w2 + u * 64 + 8 * grp));
            const bf16x8 b1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(s_w2 + u * 64 + 32 + 8 * grp));
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a20, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a21, b1, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float h = fmaxf(acc[r] + s_b2[u], 0.f);
                zp[r] += s_w3[u] * h;
                const int64_t s = s0 + 4 * grp + r;
                if (h2_out && s < n) h2_out[s * 64 + u] = h;
            }
        }
        // ---- output unit: sum over the 16 lanes of each row group ----
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) zp[r] += __shfl_xor(zp[r], off, 64);
        }
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t s = s0 + 4 * grp + r;
                if (s < n) logits[s] = zp[r] + b3;
            }
        }
        __syncthreads();   // h1t is rewritten by the next iteration
    }
}

__global__ __launch_bounds__(256) void k_mlp_bce(const float* __restrict__ z, const uint8_t* __restrict__ y,
                                                 int64_t n, float* __restrict__ dz, double2* __restrict__ part) {
    __shared__ double s_l[256];
    const float inv = 1.0f / (float)n;
    double l = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float zi = z[i], yi = y[i] ? 1.f : 0.f;
        const float sg = 1.0f / (1.0f + expf(-zi));
        dz[i] = (sg - yi) * inv;
        l += (double)(fmaxf(zi, 0.f) - zi * yi + log1pf(expf(-fabsf(zi))));
    }
    s_l[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 256; ++k) t += s_l[k];
        part[blockIdx.x] = make_double2(t, 0.0);
    }
}

__global__ __launch_bounds__(64) void k_mlp_bce_final(const double2* __restrict__ part, int nb, int64_t n,
                                                      double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[b].x;
    loss[0] = t / (double)n;
}

// Weight gradients of sum_i dz_i z_i on the matrix cores.  Each block takes
// batches of 32 samples (batch b = block + k * grid) and accumulates in a
// fixed order.  With d2 = dz w3 [h2 > 0] and d1 = (d2 W2) [h1 > 0]:
//   gW2 = d2^T h1   [64 x 64],  gW1 = d1^T x   [64 x 32],  d1 = d2 W2  [32 x 64],
// each a 16x16x32 bf16 MFMA chain with float32 accumulation.  x, h1 and W2
// are bf16 values already (the forward's operands); d2 and d1 are not, so
// each is split into hi = bf16(d) and lo = bf16(d - hi) and both halves are
// multiplied (error ~2^-17 of d instead of the 2^-9 of a single bf16).  The
// bias and w3 gradients are float32 sums on the vector units.
// LDS is [row][32 samples] transposed for the MFMA operands that run over
// samples.  Lane l of an MFMA reads A row l & 15, k 8 (l >> 4) .. +7 and B
// column l & 15, k 8 (l >> 4) .. +7, and holds C rows 4 (l >> 4) .. +3 of
// column l & 15.
__global__ __launch_bounds__(256) void k_mlp_backward(const uint16_t* __restrict__ wb, const float* __restrict__ wf,
                                                      const uint16_t* __restrict__ x, const uint16_t* __restrict__ h1,
                                                      const float* __restrict__ h2, const float* __restrict__ dz,
                                                      int64_t n, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t s_w2t[64][64];     // W2^T: [input v][output u]
    __shared__ __attribute__((aligned(16))) uint16_t s_xt[32][32];      // x^T: [feature][sample]
    __shared__ __attribute__((aligned(16))) uint16_t s_h1t[64][32];     // h1^T: [unit][sample]
    __shared__ __attribute__((aligned(16))) uint16_t s_d2[2][32][64];   // d2 hi / lo: [sample][unit]
    __shared__ __attribute__((aligned(16))) uint16_t s_d2t[2][64][32];  // d2^T hi / lo: [unit][sample]
    __shared__ __attribute__((aligned(16))) uint16_t s_d1t[2][64][32];  // d1^T hi / lo: [unit][sample]
    __shared__ float s_dz[32], s_w3[64];
    __shared__ float s_bias[3][64][4];                                   // b2, w3, b1 partials per quarter
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int row = lane & 15, grp = lane >> 4;
    for (int k = tid; k < 4096; k += 256) s_w2t[k & 63][k >> 6] = wb[2048 + k];   // W2[u][v] -> [v][u]
    if (tid < 64) s_w3[tid] = wf[kMlpW3 + tid];
    // vector-unit ownership: unit u = tid / 4, samples 8 (tid % 4) .. +7 of each batch
    const int vu = tid >> 2, vq = tid & 3;
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
    f32x4 accW2[4], accW1[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) accW2[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 2; ++k) accW1[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t nbat = (n + 31) / 32;
    for (int64_t bt = blockIdx.x; bt < nbat; bt += gridDim.x) {
        const int64_t s0 = bt * 32;
        __syncthreads();    // the previous batch's operands are consumed
        if (tid < 32) s_dz[tid] = (s0 + tid < n) ? dz[s0 + tid] : 0.f;
        {   // x^T: feature f = tid % 32, samples 4 (tid / 32) .. +3
            const int f = tid & 31, g4 = (tid >> 5) * 4;
            uint16_t v4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v4[k] = (s0 + g4 + k < n) ? x[(s0 + g4 + k) * 32 + f] : (uint16_t)0;
            *reinterpret_cast<uint2*>(&s_xt[f][g4]) =
                make_uint2((uint32_t)v4[0] | ((uint32_t)v4[1] << 16), (uint32_t)v4[2] | ((uint32_t)v4[3] << 16));
        }
        __syncthreads();
        {   // h1^T, d2 (split), and the b2 / w3 sums: unit vu, samples 8 vq .. +7
            uint16_t hv[8], dh[8], dl[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int s = 8 * vq + k;
                const bool ok = s0 + s < n;
                hv[k] = ok ? h1[(s0 + s) * 64 + vu] : (uint16_t)0;
                const float h2v = ok ? h2[(s0 + s) * 64 + vu] : 0.f;
                const float d2 = h2v > 0.f ? s_dz[s] * s_w3[vu] : 0.f;
                gb2 += d2;
                gw3 += s_dz[s] * h2v;
                dh[k] = to_bf16(d2);
                dl[k] = to_bf16(d2 - from_bf16(dh[k]));
                s_d2[0][s][vu] = dh[k];
                s_d2[1][s][vu] = dl[k];
            }
            uint4 ph, pd, pl;
            ph = make_uint4(hv[0] | (hv[1] << 16), hv[2] | (hv[3] << 16), hv[4] | (hv[5] << 16), hv[6] | (hv[7] << 16));
            pd = make_uint4(dh[0] | (dh[1] << 16), dh[2] | (dh[3] << 16), dh[4] | (dh[5] << 16), dh[6] | (dh[7] << 16));
            pl = make_uint4(dl[0] | (dl[1] << 16), dl[2] | (dl[3] << 16), dl[4] | (dl[5] << 16), dl[6] | (dl[7] << 16));
            *reinterpret_cast<uint4*>(&s_h1t[vu][8 * vq]) = ph;
            *reinterpret_cast<uint4*>(&s_d2t[0][vu][8 * vq]) = pd;
            *reinterpret_cast<uint4*>(&s_d2t[1][vu][8 * vq]) = pl;
        }
        if (tid == 0)
            for (int s = 0; s < 32; ++s) gb3 += s_dz[s];
        __syncthreads();
        // d1 = d2 W2 masked by h1 > 0: 8 output tiles (2 sample tiles x 4 unit tiles), 2 per wave
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int tau = 2 * wid + tt, St = tau & 1, Vt = tau >> 1;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int Kt = 0; Kt < 2; ++Kt) {
                const bf16x8 b = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4*>(&s_w2t[16 * Vt + row][32 * Kt + 8 * grp]));
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bf16x8 a = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const uint4*>(&s_d2[h][16 * St + row][32 * Kt + 8 * grp]));
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
                }
            }
            const int v = 16 * Vt + row;
            uint16_t dh[4], dl[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 16 * St + 4 * grp + r;
                const float d1 = from_bf16(s_h1t[v][s]) > 0.f ? acc[r] : 0.f;
                dh[r] = to_bf16(d1);
                dl[r] = to_bf16(d1 - from_bf16(dh[r]));
            }
            *reinterpret_cast<uint2*>(&s_d1t[0][v][16 * St + 4 * grp]) =
                make_uint2((uint32_t)dh[0] | ((uint32_t)dh[1] << 16), (uint32_t)dh[2] | ((uint32_t)dh[3] << 16));
            *reinterpret_cast<uint2*>(&s_d1t[1][v][16 * St + 4 * grp]) =
                make_uint2((uint32_t)dl[0] | ((uint32_t)dl[1] << 16), (uint32_t)dl[2] | ((uint32_t)dl[3] << 16));
        }
        // gW2 tiles (unit tile wid, input tiles 0..3): K = the batch's 32 samples
        {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_d2t[0][16 * wid + row][8 * grp]));
            const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_d2t[1][16 * wid + row][8 * grp]));
#pragma unroll
            for (int Vt = 0; Vt < 4; ++Vt) {
                const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_h1t[16 * Vt + row][8 * grp]));
                accW2[Vt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b, accW2[Vt], 0, 0, 0);
                accW2[Vt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, accW2[Vt], 0, 0, 0);
            }
        }
        __syncthreads();    // d1^T complete
        {   // gW1 tiles (unit tile wid, feature tiles 0..1) and the b1 sums
            const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_d1t[0][16 * wid + row][8 * grp]));
            const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_d1t[1][16 * wid + row][8 * grp]));
#pragma unroll
            for (int Ft = 0; Ft < 2; ++Ft) {
                const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_xt[16 * Ft + row][8 * grp]));
                accW1[Ft] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b, accW1[Ft], 0, 0, 0);
                accW1[Ft] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, accW1[Ft], 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                gb1 += from_bf16(s_d1t[0][vu][8 * vq + k]) + from_bf16(s_d1t[1][vu][8 * vq + k]);
        }
    }
    float* p = part + (int64_t)blockIdx.x * kMlpCount;
#pragma unroll
    for (int Vt = 0; Vt < 4; ++Vt)
#pragma unroll
        for (int r = 0; r < 4; ++r) p[kMlpW2 + (16 * wid + 4 * grp + r) * 64 + 16 * Vt + row] = accW2[Vt][r];
#pragma unroll
    for (int Ft = 0; Ft < 2; ++Ft)
#pragma unroll
        for (int r = 0; r < 4; ++r) p[kMlpW1 + (16 * wid + 4 * grp + r) * 32 + 16 * Ft + row] = accW1[Ft][r];
    // bias and w3 sums: the four sample quarters of each unit added in a fixed order
    s_bias[0][vu][vq] = gb2;
    s_bias[1][vu][vq] = gw3;
    s_bias[2][vu][vq] = gb1;
    __syncthreads();
    if (tid < 64) {
        p[kMlpB2 + tid] = ((s_bias[0][tid][0] + s_bias[0][tid][1]) + s_bias[0][tid][2]) + s_bias[0][tid][3];
        p[kMlpW3 + tid] = ((s_bias[1][tid][0] + s_bias[1][tid][1]) + s_bias[1][tid][2]) + s_bias[1][tid][3];
        p[kMlpB1 + tid] = ((s_bias[2][tid][0] + s_bias[2][tid][1]) + s_bias[2][tid][2]) + s_bias[2][tid][3];
    }
    if (tid == 0) p[kMlpB3] = gb3;
}

__global__ __launch_bounds__(256) void k_mlp_grad_final(const float* __restrict__ part, int nblocks,
                                                        float* __restrict__ grad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpCount) return;
    float acc = 0.f;
    for (int b = 0; b < nblocks; ++b) acc += part[(int64_t)b * kMlpCount + k];
    grad[k] = acc;
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                  float b2, float eps, float bc1, float bc2,
                                                  uint16_t* __restrict__ wb) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpCount) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float wk = w[k] - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
    w[k] = wk;
    if (k < kMlpB1) wb[k] = to_bf16(wk);
    else if (k >= kMlpW2 && k < kMlpB2) wb[2048 + (k - kMlpW2)] = to_bf16(wk);
}

__global__ __launch_bounds__(256) void k_mlp_bf16_copy(const float* __restrict__ w, uint16_t* __restrict__ wb) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 2048) wb[k] = to_bf16(w[kMlpW1 + k]);
    else if (k < 2048 + 4096) wb[k] = to_bf16(w[kMlpW2 + k - 2048]);
}

__global__ __launch_bounds__(256) void k_mlp_propose(const float* __restrict__ z, const float* __restrict__ sx,
                                                     const float* __restrict__ sr, int64_t n, float thr, float vx,
                                                     float vr, uint8_t* __restrict__ prop) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    prop[i] = (z[i] > thr && sx[i] < vx && sr[i] < vr) ? 1 : 0;
}

}  // namespace

static unsigned grid_of(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

void launch_traj_push(const float* ema, int64_t n, uint16_t* ring, int slot, hipStream_t s) {
    if (n > 0) k_traj_push<<<grid_of(n, 256), 256, 0, s>>>(ema, n, ring, slot);
}

void launch_mlp_stats(const uint16_t* ring, int64_t n, int head, double* part, double* sums, hipStream_t s) {
    k_mlp_stats<<<kMlpBlocks, 256, 0, s>>>(ring, n, head, part);
    k_mlp_stats_final<<<1, 64, 0, s>>>(part, kMlpBlocks, sums);
}

void launch_mlp_features(const uint16_t* ring, int64_t n, int head, const float* mean, const float* stdv,
                         uint16_t* x, hipStream_t s) {
    if (n > 0) k_mlp_features<<<grid_of(n, 256), 256, 0, s>>>(ring, n, head, mean, stdv, x);
}

void launch_mlp_forward(const uint16_t* wb, const float* wf, const uint16_t* x, int64_t n, float* logits,
                        uint16_t* h1, float* h2, int blocks, hipStream_t s) {
    if (n <= 0) return;
    const int64_t need = (n + 63) / 64;   // 4 tiles of 16 per block
    k_mlp_forward<<<(unsigned)std::min<int64_t>(need, blocks), 256, 0, s>>>(wb, wf, x, n, logits, h1, h2);
}

void launch_mlp_bce(const float* z, const uint8_t* y, int64_t n, float* dz, double* loss, double2* part,
                    hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kL1Blocks, grid_of(n, 256));
    k_mlp_bce<<<nb, 256, 0, s>>>(z, y, n, dz, part);
    k_mlp_bce_final<<<1, 64, 0, s>>>(part, nb, n, loss);
}

void launch_mlp_backward(const uint16_t* wb, const float* wf, const uint16_t* x, const uint16_t* h1, const float* h2,
                         const float* dz, int64_t n, float* part, float* grad, hipStream_t s) {
    k_mlp_backward<<<kMlpBlocks, 256, 0, s>>>(wb, wf, x, h1, h2, dz, n, part);
    k_mlp_grad_final<<<grid_of(kMlpCount, 256), 256, 0, s>>>(part, kMlpBlocks, grad);
}

void launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, float bc1,
                     float bc2, uint16_t* wb, hipStream_t s) {
    k_mlp_adam<<<grid_of(kMlpCount, 256), 256, 0, s>>>(w, g, m, v, lr, b1, b2, eps, bc1, bc2, wb);
}

void launch_mlp_bf16_copy(const float* w, uint16_t* wb, hipStream_t s) {
    k_mlp_bf16_copy<<<grid_of(6144, 256), 256, 0, s>>>(w, wb);
}

void launch_mlp_propose(const float* z, const float* sx, const float* sr, int64_t n, float thr, float vx, float vr,
                        uint8_t* prop, hipStream_t s) {
    if (n > 0) k_mlp_propose<<<grid_of(n, 256), 256, 0, s>>>(z, sx, sr, n, thr, vx, vr, prop);
}

}  // namespace gsta
