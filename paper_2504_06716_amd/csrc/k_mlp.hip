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
//   K11f backward:  weight gradients, per-block partials summed in block
//                   order (deterministic)
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

// Weight gradients of sum_i dz_i z_i.  Each block takes batches of 16
// samples (batch b = block + k * grid) and accumulates in a fixed order:
// thread t owns W2[t/4][16 (t%4) ..], W1[t/4][8 (t%4) ..] and, for t%4 = 0,
// b1, b2, w3 of unit t/4; thread 0 owns b3.
__global__ __launch_bounds__(256) void k_mlp_backward(const uint16_t* __restrict__ wb, const float* __restrict__ wf,
                                                      const uint16_t* __restrict__ x, const uint16_t* __restrict__ h1,
                                                      const float* __restrict__ h2, const float* __restrict__ dz,
                                                      int64_t n, float* __restrict__ part) {
    __shared__ float s_x[16][32], s_h1[16][64], s_d2[16][64], s_d1[16][64], s_dz[16];
    __shared__ float s_w2[64][65];
    __shared__ float s_w3[64];
    const int tid = threadIdx.x;
    for (int k = tid; k < 4096; k += 256) s_w2[k >> 6][k & 63] = from_bf16(wb[2048 + k]);
    if (tid < 64) s_w3[tid] = wf[kMlpW3 + tid];
    const int u = tid >> 2, q = tid & 3;
    float gW2[16], gW1[8];
#pragma unroll
    for (int k = 0; k < 16; ++k) gW2[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) gW1[k] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
    const int64_t nbat = (n + 15) / 16;
    for (int64_t bt = blockIdx.x; bt < nbat; bt += gridDim.x) {
        const int64_t s0 = bt * 16;
        __syncthreads();
        // stage the batch: features, first hidden layer, dz, and d2 = dz w3 [h2 > 0]
        for (int k = tid; k < 16 * 32; k += 256) {
            const int s = k >> 5, f = k & 31;
            s_x[s][f] = (s0 + s < n) ? from_bf16(x[(s0 + s) * 32 + f]) : 0.f;
        }
        if (tid < 16) s_dz[tid] = (s0 + tid < n) ? dz[s0 + tid] : 0.f;
        __syncthreads();
        for (int k = tid; k < 16 * 64; k += 256) {
            const int s = k >> 6, v = k & 63;
            const bool ok = s0 + s < n;
            s_h1[s][v] = ok ? from_bf16(h1[(s0 + s) * 64 + v]) : 0.f;
            const float hv = ok ? h2[(s0 + s) * 64 + v] : 0.f;
            s_d2[s][v] = hv > 0.f ? s_dz[s] * s_w3[v] : 0.f;
            // reuse s_d1 to hold h2 for the w3 gradient
            s_d1[s][v] = hv;
        }
        __syncthreads();
        if (q == 0) {
            for (int s = 0; s < 16; ++s) {
                gw3 += s_dz[s] * s_d1[s][u];
                gb2 += s_d2[s][u];
            }
        }
        if (tid == 0)
            for (int s = 0; s < 16; ++s) gb3 += s_dz[s];
        __syncthreads();
        // d1[s][v] = sum_u d2[s][u] W2[u][v], masked by h1 > 0: thread -> (s = tid / 16, v = 4 (tid % 16) ..)
        {
            const int s = tid >> 4, v0 = (tid & 15) * 4;
            float acc[4] = {0.f, 0.f, 0.f, 0.f};
            for (int uu = 0; uu < 64; ++uu) {
                const float d = s_d2[s][uu];
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[k] += d * s_w2[uu][v0 + k];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) s_d1[s][v0 + k] = s_h1[s][v0 + k] > 0.f ? acc[k] : 0.f;
        }
        __syncthreads();
        for (int s = 0; s < 16; ++s) {
            const float d2 = s_d2[s][u], d1 = s_d1[s][u];
#pragma unroll
            for (int k = 0; k < 16; ++k) gW2[k] += d2 * s_h1[s][16 * q + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) gW1[k] += d1 * s_x[s][8 * q + k];
            if (q == 0) gb1 += d1;
        }
    }
    float* p = part + (int64_t)blockIdx.x * kMlpCount;
#pragma unroll
    for (int k = 0; k < 16; ++k) p[kMlpW2 + u * 64 + 16 * q + k] = gW2[k];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[kMlpW1 + u * 32 + 8 * q + k] = gW1[k];
    if (q == 0) {
        p[kMlpB1 + u] = gb1;
        p[kMlpB2 + u] = gb2;
        p[kMlpW3 + u] = gw3;
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
