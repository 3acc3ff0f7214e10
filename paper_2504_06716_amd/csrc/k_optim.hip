// Element-wise steps: L1 loss (eq. 3, lambda_SSIM = 0), masked Adam
// (Section 3.2.4: frozen Gaussians are not updated) and the freeze-map update
// (Section 3.2.1, eqs. 4 and 6).
#include "gsta_internal.h"

namespace gsta {
namespace {

// Masked Adam over the columns of one row of the [rows][n] block: 4 columns
// per thread when every stride allows 16-byte access, else one; every
// column takes the same operations whatever its position.  A frozen
// column is skipped before any of its p, g, m, v bytes are read.
template <bool VEC>
__device__ __forceinline__ void adam_columns(int row, float* __restrict__ p, int64_t pld,
                                             const float* __restrict__ g, int64_t gld, float* __restrict__ m,
                                             int64_t mld, float* __restrict__ v, int64_t vld, int64_t n,
                                             float lrr, float b1, float b2, float eps, float rbc1, float rbc2,
                                             const uint8_t* __restrict__ frozen, uint32_t* __restrict__ flags) {
    // No contraction: the compiler would otherwise fuse the four unrolled
    // column updates differently, making a column's result depend on its
    // position within its 16-byte group (and so on the column order).
#pragma clang fp contract(off)
    const float ib1 = 1.f - b1, ib2 = 1.f - b2;
    bool bad = false;
    if (VEC) {
        const int64_t i4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
        if (i4 >= n) return;
        if (i4 + 4 <= n) {
            uchar4 fz = frozen ? *reinterpret_cast<const uchar4*>(frozen + i4) : make_uchar4(0, 0, 0, 0);
            if ((fz.x & fz.y & fz.z & fz.w) != 0) return;
            float4 pp = *reinterpret_cast<const float4*>(p + row * pld + i4);
            float4 gg = *reinterpret_cast<const float4*>(g + row * gld + i4);
            float4 mm = *reinterpret_cast<const float4*>(m + row * mld + i4);
            float4 vv = *reinterpret_cast<const float4*>(v + row * vld + i4);
            float* pe = &pp.x; float* ge = &gg.x; float* me = &mm.x; float* ve = &vv.x;
            const uint8_t fe[4] = {fz.x, fz.y, fz.z, fz.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (fe[k]) continue;
                const float gk = ge[k];
                bad |= !isfinite(gk);
                me[k] = b1 * me[k] + ib1 * gk;
                ve[k] = b2 * ve[k] + ib2 * gk * gk;
                pe[k] -= lrr * (me[k] * rbc1) / (sqrtf(ve[k] * rbc2) + eps);
            }
            *reinterpret_cast<float4*>(p + row * pld + i4) = pp;
            *reinterpret_cast<float4*>(m + row * mld + i4) = mm;
            *reinterpret_cast<float4*>(v + row * vld + i4) = vv;
        } else {
            for (int64_t i = i4; i < n; ++i) {
                if (frozen && frozen[i]) continue;
                const float gk = g[row * gld + i];
                bad |= !isfinite(gk);
                float mk = b1 * m[row * mld + i] + ib1 * gk;
                float vk = b2 * v[row * vld + i] + ib2 * gk * gk;
                m[row * mld + i] = mk;
                v[row * vld + i] = vk;
                p[row * pld + i] -= lrr * (mk * rbc1) / (sqrtf(vk * rbc2) + eps);
            }
        }
    } else {
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (i >= n) return;
        if (frozen && frozen[i]) return;
        const float gk = g[row * gld + i];
        bad = !isfinite(gk);
        float mk = b1 * m[row * mld + i] + ib1 * gk;
        float vk = b2 * v[row * vld + i] + ib2 * gk * gk;
        m[row * mld + i] = mk;
        v[row * vld + i] = vk;
        p[row * pld + i] -= lrr * (mk * rbc1) / (sqrtf(vk * rbc2) + eps);
    }
    // the first lane with a bad gradient reports it (lanes that returned early had none)
    const uint64_t bb = __ballot(bad);
    if (bb != 0ull && (int)(threadIdx.x & 63) == __builtin_ctzll(bb)) atomicOr(&flags[1], 1u);
}

// Grid: x over columns, y over rows.
template <bool VEC>
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, int64_t pld,
                                              const float* __restrict__ g, int64_t gld,
                                              float* __restrict__ m, int64_t mld, float* __restrict__ v,
                                              int64_t vld, int64_t n, LrArray lr, float b1, float b2,
                                              float eps, float bc1, float bc2,
                                              const uint8_t* __restrict__ frozen,
                                              uint32_t* __restrict__ flags) {
    const int row = blockIdx.y;
    adam_columns<VEC>(row, p, pld, g, gld, m, mld, v, vld, n, lr.lr[row], b1, b2, eps, 1.f / bc1, 1.f / bc2, frozen,
                      flags);
}

// Adam whose scalars come from a device-resident schedule (graph replay);
// the same column update as k_adam.
template <bool VEC>
__global__ __launch_bounds__(256) void k_adam_sched(float* __restrict__ p, int64_t pld,
                                                    const float* __restrict__ g, int64_t gld,
                                                    float* __restrict__ m, int64_t mld, float* __restrict__ v,
                                                    int64_t vld, int64_t n, const AdamSched* __restrict__ sc,
                                                    const uint8_t* __restrict__ frozen,
                                                    uint32_t* __restrict__ flags) {
    const int row = blockIdx.y;
    const int step = sc->step;
    const float b1 = sc->beta1, b2 = sc->beta2, eps = sc->eps;
    float lrr;
    if (row < 3) {
        const float t = fminf((float)(step - 1) / (float)max(sc->decay_iters, 1), 1.0f);
        lrr = sc->pos_scale * expf((1.0f - t) * logf(sc->pos_lr_init) + t * logf(sc->pos_lr_final));
    } else {
        lrr = sc->lr[row];
    }
    const float rbc1 = 1.f / (1.f - powf(b1, (float)step)), rbc2 = 1.f / (1.f - powf(b2, (float)step));
    adam_columns<VEC>(row, p, pld, g, gld, m, mld, v, vld, n, lrr, b1, b2, eps, rbc1, rbc2, frozen, flags);
}

__global__ void k_sched_advance(AdamSched* sc) { sc->step += 1; }

__global__ __launch_bounds__(256) void k_freeze(const float* __restrict__ sx, const float* __restrict__ sr,
                                                int64_t n, float ex, float er, int mode,
                                                const uint8_t* __restrict__ proposal,
                                                uint8_t* __restrict__ frozen,
                                                unsigned long long* __restrict__ n_frozen) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool f = false;
    if (i < n) {
        bool cond = false;
        if (mode != 1) {
            cond = (sx[i] < ex) && (sr[i] < er);
            if (proposal) cond = cond || (proposal[i] != 0);
        }
        f = (mode == 0) ? ((frozen[i] != 0) || cond) : (mode == 1 ? false : cond);
        frozen[i] = f ? 1 : 0;
    }
    if (n_frozen) {   // uniform; one atomic per workgroup (same-address atomics serialise)
        __shared__ uint32_t s_w[4];
        const uint64_t bal = __ballot(f);
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t c = s_w[0] + s_w[1] + s_w[2] + s_w[3];
            if (c) atomicAdd(n_frozen, (unsigned long long)c);
        }
    }
}

__global__ void k_zero_i64(unsigned long long* p) { *p = 0ull; }

// L1 loss, pass 1: per-workgroup partial sums (double) of |C - C*| and of
// the clamped squared error, and dL/dC for every element.
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ img, const float* __restrict__ tgt,
                                            int64_t count, float* __restrict__ dL, double2* __restrict__ part) {
    __shared__ double s_a[4], s_b[4];
    const float inv = 1.0f / (float)count;
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float c = img[i], t = tgt[i];
        const float d = c - t;
        dL[i] = (d > 0.f) ? inv : ((d < 0.f) ? -inv : 0.f);
        a += (double)fabsf(d);
        const double e = (double)fminf(fmaxf(c, 0.f), 1.f) - (double)t;
        b += e * e;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        s_a[wid] = a;
        s_b[wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(s_a[0] + s_a[1] + s_a[2] + s_a[3],
                                                          s_b[0] + s_b[1] + s_b[2] + s_b[3]);
}

// Pass 2: one workgroup adds the partials in a fixed order.
__global__ __launch_bounds__(256) void k_l1_final(const double2* __restrict__ part, int nb, double* __restrict__ sums) {
    __shared__ double s_a[256], s_b[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[i].x;
        b += part[i].y;
    }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s_a[threadIdx.x] += s_a[threadIdx.x + off];
            s_b[threadIdx.x] += s_b[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[0] = s_a[0];
        sums[1] = s_b[0];
    }
}

// SH-band mask sparsity (Section 3.3): per Gaussian its three logits' sigmoid
// sum and open-gate counts, block totals in LDS, one partial per block.
__global__ __launch_bounds__(256) void k_shm_reg(const float* __restrict__ logits, int64_t n, int64_t ld,
                                                 float thr, float scale, const uint8_t* __restrict__ frozen,
                                                 float* __restrict__ grad, double* __restrict__ part, int nb) {
    __shared__ double s_v[4][256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        const bool upd = grad && !(frozen && frozen[i]);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const float x = logits[l * ld + i];
            const float sg = 1.0f / (1.0f + expf(-x));
            acc[0] += (double)sg;
            acc[1 + l] = x > thr ? 1.0 : 0.0;
            if (upd) grad[l * ld + i] += scale * (sg * (1.0f - sg));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s_v[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {   // fixed-order tree
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 4; ++q) s_v[q][threadIdx.x] += s_v[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[(int64_t)threadIdx.x * nb + blockIdx.x] = s_v[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_shm_reg_final(const double* __restrict__ part, int nb, double scale,
                                                       double* __restrict__ out) {
    __shared__ double s_v[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = (int)threadIdx.x; b < nb; b += 256)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += part[(int64_t)q * nb + b];
#pragma unroll
    for (int q = 0; q < 4; ++q) s_v[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 4; ++q) s_v[q][threadIdx.x] += s_v[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = scale * s_v[0][0];
        out[1] = s_v[1][0];
        out[2] = s_v[2][0];
        out[3] = s_v[3][0];
    }
}

}  // namespace

void launch_sh_mask_reg(const float* logits, int64_t n, int64_t ld, float thr_logit, float lambda,
                        const uint8_t* frozen, float* grad, double* part, double* out, hipStream_t s) {
    const int nb = (int)((n + 255) / 256);
    const double mean = 1.0 / (3.0 * (double)n);
    k_shm_reg<<<(unsigned)nb, 256, 0, s>>>(logits, n, ld, thr_logit, (float)((double)lambda * mean), frozen, grad,
                                           part, nb);
    k_shm_reg_final<<<1, 256, 0, s>>>(part, nb, (double)lambda * mean, out);
}

void launch_adam(float* p, int64_t pld, const float* g, int64_t gld, float* m, int64_t mld, float* v,
                 int64_t vld, int64_t n, int rows, const LrArray& lr, float b1, float b2, float eps,
                 float bc1, float bc2, const uint8_t* frozen, uint32_t* flags, hipStream_t s) {
    const bool vec = (pld % 4 == 0) && (gld % 4 == 0) && (mld % 4 == 0) && (vld % 4 == 0) &&
                     ((uintptr_t)p % 16 == 0) && ((uintptr_t)g % 16 == 0) && ((uintptr_t)m % 16 == 0) &&
                     ((uintptr_t)v % 16 == 0) && (!frozen || (uintptr_t)frozen % 4 == 0);
    if (vec) {
        const int64_t threads = (n + 3) / 4;
        k_adam<true><<<dim3((unsigned)((threads + 255) / 256), rows), 256, 0, s>>>(
            p, pld, g, gld, m, mld, v, vld, n, lr, b1, b2, eps, bc1, bc2, frozen, flags);
    } else {
        k_adam<false><<<dim3((unsigned)((n + 255) / 256), rows), 256, 0, s>>>(
            p, pld, g, gld, m, mld, v, vld, n, lr, b1, b2, eps, bc1, bc2, frozen, flags);
    }
}

void launch_adam_sched(float* p, int64_t pld, const float* g, int64_t gld, float* m, int64_t mld, float* v,
                       int64_t vld, int64_t n, int rows, AdamSched* sched, const uint8_t* frozen, uint32_t* flags,
                       hipStream_t s) {
    const bool vec = (pld % 4 == 0) && (gld % 4 == 0) && (mld % 4 == 0) && (vld % 4 == 0) &&
                     ((uintptr_t)p % 16 == 0) && ((uintptr_t)g % 16 == 0) && ((uintptr_t)m % 16 == 0) &&
                     ((uintptr_t)v % 16 == 0) && (!frozen || (uintptr_t)frozen % 4 == 0);
    if (n > 0) {
        if (vec)
            k_adam_sched<true><<<dim3((unsigned)(((n + 3) / 4 + 255) / 256), rows), 256, 0, s>>>(
                p, pld, g, gld, m, mld, v, vld, n, sched, frozen, flags);
        else
            k_adam_sched<false><<<dim3((unsigned)((n + 255) / 256), rows), 256, 0, s>>>(p, pld, g, gld, m, mld, v,
                                                                                       vld, n, sched, frozen, flags);
    }
    k_sched_advance<<<1, 1, 0, s>>>(sched);
}

void launch_freeze(const float* sx, const float* sr, int64_t n, float ex, float er, int mode,
                   const uint8_t* proposal, uint8_t* frozen, int64_t* n_frozen, hipStream_t s) {
    if (n_frozen) k_zero_i64<<<1, 1, 0, s>>>(reinterpret_cast<unsigned long long*>(n_frozen));
    if (n > 0)
        k_freeze<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            sx, sr, n, ex, er, mode, proposal, frozen, reinterpret_cast<unsigned long long*>(n_frozen));
}

void launch_l1(const float* img, const float* tgt, int64_t count, float* dL, double* sums, double2* part,
               hipStream_t s) {
    int64_t blocks = (count + 1023) / 1024;
    if (blocks > kL1Blocks) blocks = kL1Blocks;
    if (blocks < 1) blocks = 1;
    k_l1<<<(unsigned)blocks, 256, 0, s>>>(img, tgt, count, dL, part);
    k_l1_final<<<1, 256, 0, s>>>(part, (int)blocks, sums);
}

}  // namespace gsta
