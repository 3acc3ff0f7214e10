// Adaptive densification, pruning and opacity reset (Section 3.1: Gaussians
// are densified by gradient norm and pruned by opacity; Section 4.1: every
// 100 iterations, diffuse-colour gradients on a fifth of the steps, opacity
// reset every 3K).  The clone / split / prune rules are the 3DGS conventions
// the paper builds on.
//
// One densify step is a stream compaction of every per-Gaussian array:
//   K10a classify: per Gaussian a code (keep, clone, split) + per-block counts
//   K10b scan:     one workgroup turns the block counts into block offsets and
//                  the totals (kept K, clones C, split parents S)
//   K10c scatter:  survivors to [0, K), clones to [K, K+C), first children to
//                  [K+C, K+C+S), second children to [K+C+S, K+C+2S)
// All decisions are float32 comparisons of the inputs, so they are exact;
// ranks come from wave ballots, so the output order is the input order.
//
// The same ballot ranking gives the stable partition of the columns by the
// freeze map (active first) that gsta_partition_frozen applies in place.
#include <algorithm>

#include "gsta_internal.h"

namespace gsta {
namespace {

constexpr int kDB = 256;                 // Gaussians per block
constexpr uint8_t kKeep = 1, kClone = 2, kSplit = 4;

__global__ __launch_bounds__(kDB) void k_dens_classify(const float* __restrict__ P, int64_t ld, int64_t n,
                                                       const uint8_t* __restrict__ frozen,
                                                       const float* __restrict__ stats, DensCfg cfg,
                                                       uint8_t* __restrict__ code, uint32_t* __restrict__ bcount,
                                                       int64_t nb) {
    __shared__ uint32_t s_cnt[kDB / 64][3];
    const int64_t i = (int64_t)blockIdx.x * kDB + threadIdx.x;
    uint8_t c = 0;
    if (i < n) {
        const float a0 = stats[i], n0 = stats[n + i], a1 = stats[2 * n + i], n1 = stats[3 * n + i];
        const float mxy = n0 > 0.f ? a0 / n0 : 0.f;
        const float mrgb = n1 > 0.f ? a1 / n1 : 0.f;
        bool sel = mxy >= cfg.grad_threshold;
        if (cfg.use_rgb) sel = sel || (mrgb >= cfg.rgb_threshold);
        if (frozen && frozen[i]) sel = false;
        const float smax = fmaxf(fmaxf(P[3 * ld + i], P[4 * ld + i]), P[5 * ld + i]);
        const bool big = smax > cfg.split_log_scale;
        const bool live = P[10 * ld + i] >= cfg.prune_logit;
        if (live) {
            if (!(sel && big)) c |= kKeep;
            if (sel && !big) c |= kClone;
            if (sel && big) c |= kSplit;
        }
        code[i] = c;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t bk = __ballot(c & kKeep), bc = __ballot(c & kClone), bs = __ballot(c & kSplit);
    if (lane == 0) {
        s_cnt[w][0] = (uint32_t)__popcll(bk);
        s_cnt[w][1] = (uint32_t)__popcll(bc);
        s_cnt[w][2] = (uint32_t)__popcll(bs);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < kDB / 64; ++k) t += s_cnt[k][threadIdx.x];
        bcount[threadIdx.x * nb + blockIdx.x] = t;
    }
}

// Exclusive scan of the three count rows (in place) by one workgroup of
// 1024 threads; tot = (K, C, S) and counts = (n_out, K, C, S).  When n_out
// exceeds the output capacity the overflow flag is raised and the scatter
// writes nothing.
__global__ __launch_bounds__(1024) void k_dens_scan(uint32_t* __restrict__ b, int64_t nb,
                                                    uint32_t* __restrict__ tot, int64_t* __restrict__ counts,
                                                    int64_t cap, uint32_t* __restrict__ flags) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t total[3];
    for (int r = 0; r < 3; ++r) {
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        uint32_t* row = b + r * nb;
        for (int64_t base = 0; base < nb; base += 1024) {
            const int64_t j = base + threadIdx.x;
            const uint32_t x = j < nb ? row[j] : 0u;
            uint32_t incl = x;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            if (lane == 63) s_w[w] = incl;
            __syncthreads();
            uint32_t wbase = s_carry;
            for (int k = 0; k < w; ++k) wbase += s_w[k];
            if (j < nb) row[j] = wbase + incl - x;
            __syncthreads();
            if (threadIdx.x == 1023) s_carry = wbase + incl;
            __syncthreads();
        }
        total[r] = s_carry;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t n_out = (int64_t)total[0] + total[1] + 2 * (int64_t)total[2];
        tot[0] = total[0];
        tot[1] = total[1];
        tot[2] = total[2];
        tot[3] = n_out > cap ? 1u : 0u;
        counts[0] = n_out;
        counts[1] = total[0];
        counts[2] = total[1];
        counts[3] = total[2];
        if (n_out > cap) atomicOr(&flags[2], 1u);
    }
}

// Rank of this lane among the block's lanes with `pred` set, in thread order.
__device__ __forceinline__ uint32_t block_rank(bool pred, uint32_t (*s_w)[3], int r) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t m = __ballot(pred);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (lane == 0) s_w[w][r] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t base = 0;
    for (int k = 0; k < w; ++k) base += s_w[k][r];
    return base + below;
}

template <int D>
__global__ __launch_bounds__(kDB) void k_dens_scatter(
    const float* __restrict__ P, int64_t ld, const float* __restrict__ M, int64_t mld, const float* __restrict__ V,
    int64_t vld, const float* __restrict__ ema, const uint8_t* __restrict__ frozen, const float* __restrict__ noise,
    int64_t n, const uint8_t* __restrict__ code, const uint32_t* __restrict__ boff, int64_t nb,
    const uint32_t* __restrict__ tot, float child_shift, uint64_t seed, int64_t draw, float* __restrict__ Po,
    int64_t old_, float* __restrict__ Mo,
    int64_t mold, float* __restrict__ Vo, int64_t vold, float* __restrict__ ema_o, uint8_t* __restrict__ frozen_o) {
    constexpr int R = 11 + 3 * (D + 1) * (D + 1);
    __shared__ uint32_t s_w[kDB / 64][3];
    if (tot[3]) return;                          // over capacity: nothing is written
    const uint32_t K = tot[0], C = tot[1], S = tot[2];
    const int64_t n_out = (int64_t)K + C + 2 * (int64_t)S;
    const int64_t i = (int64_t)blockIdx.x * kDB + threadIdx.x;
    const uint8_t c = i < n ? code[i] : 0;
    const uint32_t rk = block_rank(c & kKeep, s_w, 0);
    const uint32_t rc = block_rank(c & kClone, s_w, 1);
    const uint32_t rs = block_rank(c & kSplit, s_w, 2);
    if (i >= n || c == 0) return;
    const float FMAX = 3.402823466e38f;
    if (c & kKeep) {
        const int64_t o = boff[blockIdx.x] + rk;
#pragma unroll 4
        for (int r = 0; r < R; ++r) {
            Po[r * old_ + o] = P[r * ld + i];
            Mo[r * mold + o] = M[r * mld + i];
            Vo[r * vold + o] = V[r * vld + i];
        }
        if (ema_o)
#pragma unroll
            for (int r = 0; r < 4; ++r) ema_o[r * n_out + o] = ema ? ema[r * n + i] : FMAX;
        if (frozen_o) frozen_o[o] = frozen ? frozen[i] : 0;
    }
    if (c & kClone) {
        const int64_t o = (int64_t)K + boff[nb + blockIdx.x] + rc;
#pragma unroll 4
        for (int r = 0; r < R; ++r) {
            Po[r * old_ + o] = P[r * ld + i];
            Mo[r * mold + o] = 0.f;
            Vo[r * vold + o] = 0.f;
        }
        if (ema_o)
#pragma unroll
            for (int r = 0; r < 4; ++r) ema_o[r * n_out + o] = FMAX;
        if (frozen_o) frozen_o[o] = 0;
    }
    if (c & kSplit) {
        const int64_t s = boff[2 * nb + blockIdx.x] + rs;
        // R(q) of the normalised quaternion (w, x, y, z)
        const float qw0 = P[6 * ld + i], qx0 = P[7 * ld + i], qy0 = P[8 * ld + i], qz0 = P[9 * ld + i];
        const float qi = 1.0f / sqrtf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
        const float w = qw0 * qi, x = qx0 * qi, y = qy0 * qi, z = qz0 * qi;
        const float Rm[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                             2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                             2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
        const float ls[3] = {P[3 * ld + i], P[4 * ld + i], P[5 * ld + i]};
        const float sc[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
        for (int ch = 0; ch < 2; ++ch) {
            const int64_t o = (int64_t)K + C + (int64_t)ch * S + s;
            float e[3];
            if (noise) {
#pragma unroll
                for (int a = 0; a < 3; ++a) e[a] = sc[a] * noise[(3 * ch + a) * n + i];
            } else {
                // child ch of Gaussian i: three standard normals by Box-Muller from the
                // four words of Philox4x64-10(counter (i, draw, ch, 0), key (seed, 1))
                uint64_t w4[4] = {(uint64_t)i, (uint64_t)draw, (uint64_t)ch, 0ull};
                philox4x64_10(w4, seed, 1ull);
                double u[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) u[a] = ((double)(w4[a] >> 11) + 0.5) * 0x1.0p-53;
                const double two_pi = 6.283185307179586476925286766559;
                const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
                const double nz[3] = {r0 * cos(two_pi * u[1]), r0 * sin(two_pi * u[1]), r1 * cos(two_pi * u[3])};
#pragma unroll
                for (int a = 0; a < 3; ++a) e[a] = sc[a] * (float)nz[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
                Po[a * old_ + o] = P[a * ld + i] + (Rm[3 * a] * e[0] + Rm[3 * a + 1] * e[1] + Rm[3 * a + 2] * e[2]);
#pragma unroll
            for (int a = 0; a < 3; ++a) Po[(3 + a) * old_ + o] = ls[a] - child_shift;
#pragma unroll 4
            for (int r = 6; r < R; ++r) Po[r * old_ + o] = P[r * ld + i];
#pragma unroll 4
            for (int r = 0; r < R; ++r) {
                Mo[r * mold + o] = 0.f;
                Vo[r * vold + o] = 0.f;
            }
            if (ema_o)
#pragma unroll
                for (int r = 0; r < 4; ++r) ema_o[r * n_out + o] = FMAX;
            if (frozen_o) frozen_o[o] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_opacity_reset(float* __restrict__ P, int64_t ld, float* __restrict__ M,
                                                       int64_t mld, float* __restrict__ V, int64_t vld, int64_t n,
                                                       const uint8_t* __restrict__ frozen, float cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (frozen && frozen[i]) return;
    P[10 * ld + i] = fminf(P[10 * ld + i], cap);
    M[10 * mld + i] = 0.f;
    V[10 * vld + i] = 0.f;
}

// Finetune switch to the absolute opacity activation: the parameter becomes
// the opacity itself (sigmoid of the logit) and the row's moments restart.
__global__ __launch_bounds__(256) void k_opacity_to_abs(float* __restrict__ P, int64_t ld, float* __restrict__ M,
                                                        int64_t mld, float* __restrict__ V, int64_t vld, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    P[10 * ld + i] = 1.0f / (1.0f + expf(-P[10 * ld + i]));
    M[10 * mld + i] = 0.f;
    V[10 * vld + i] = 0.f;
}

// ---- stable partition by the freeze map --------------------------------
// Active (frozen == 0) columns move to [0, A) and frozen ones to [A, n), each
// group in input order: with a(j) the number of active columns before j,
// active j goes to a(j) and frozen j to A + j - a(j).  src[dest] = j is the
// gather list every array is then permuted by.

__global__ __launch_bounds__(kDB) void k_part_count(const uint8_t* __restrict__ frozen, int64_t n,
                                                    uint32_t* __restrict__ bcount) {
    __shared__ uint32_t s_cnt[kDB / 64];
    const int64_t i = (int64_t)blockIdx.x * kDB + threadIdx.x;
    const bool act = i < n && frozen[i] == 0;
    const uint64_t b = __ballot(act);
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < kDB / 64; ++k) t += s_cnt[k];
        bcount[blockIdx.x] = t;
    }
}

// Exclusive scan of the nb block counts (in place) by one workgroup;
// tot[0] and n_active[0] receive the total.
__global__ __launch_bounds__(1024) void k_part_scan(uint32_t* __restrict__ b, int64_t nb,
                                                    uint32_t* __restrict__ tot, int64_t* __restrict__ n_active) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t j = base + threadIdx.x;
        const uint32_t x = j < nb ? b[j] : 0u;
        uint32_t incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint32_t wbase = s_carry;
        for (int k = 0; k < w; ++k) wbase += s_w[k];
        if (j < nb) b[j] = wbase + incl - x;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = wbase + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tot[0] = s_carry;
        if (n_active) n_active[0] = (int64_t)s_carry;
    }
}

__global__ __launch_bounds__(kDB) void k_part_src(const uint8_t* __restrict__ frozen, int64_t n,
                                                  const uint32_t* __restrict__ boff,
                                                  const uint32_t* __restrict__ tot, uint32_t* __restrict__ src) {
    __shared__ uint32_t s_w[kDB / 64];
    const int64_t i = (int64_t)blockIdx.x * kDB + threadIdx.x;
    const bool act = i < n && frozen[i] == 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t m = __ballot(act);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (lane == 0) s_w[w] = (uint32_t)__popcll(m);
    __syncthreads();
    if (i >= n) return;
    uint32_t a = boff[blockIdx.x] + below;
    for (int k = 0; k < w; ++k) a += s_w[k];
    const int64_t dest = act ? (int64_t)a : (int64_t)tot[0] + i - (int64_t)a;
    src[dest] = (uint32_t)i;
}

// out[r][i] = x[r][src[i]] (out packed with row stride n).
template <typename T>
__global__ __launch_bounds__(256) void k_part_gather(const T* __restrict__ x, int64_t ld, int64_t rows,
                                                     const uint32_t* __restrict__ src, int64_t n,
                                                     T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t j = src[i];
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) out[r * n + i] = x[r * ld + j];
}

// x[r][i] = t[r][i] (t packed with row stride n).
template <typename T>
__global__ __launch_bounds__(256) void k_part_put(const T* __restrict__ t, int64_t rows, int64_t n,
                                                  T* __restrict__ x, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) x[r * ld + i] = t[r * n + i];
}

__global__ __launch_bounds__(256) void k_part_mask(uint8_t* __restrict__ frozen, int64_t n,
                                                   const uint32_t* __restrict__ tot) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) frozen[i] = i >= (int64_t)tot[0] ? 1 : 0;
}

}  // namespace

int64_t densify_blocks(int64_t n) { return (n + kDB - 1) / kDB; }

void launch_densify(const DensIO& io, const DensCfg& cfg, uint8_t* code, uint32_t* boff, uint32_t* tot,
                    int64_t* counts, uint32_t* flags, hipStream_t s) {
    const int64_t nb = densify_blocks(io.n);
    if (nb > 0)
        k_dens_classify<<<(unsigned)nb, kDB, 0, s>>>(io.P, io.ld, io.n, io.frozen, io.stats, cfg, code, boff, nb);
    k_dens_scan<<<1, 1024, 0, s>>>(boff, nb, tot, counts, io.cap, flags);
    if (nb == 0) return;
#define GSTA_DENS_ARGS                                                                                          \
    io.P, io.ld, io.M, io.mld, io.V, io.vld, io.ema, io.frozen, io.noise, io.n, code, boff, nb, tot,            \
        cfg.child_log_scale_shift, io.seed, io.draw, io.Po, io.old_, io.Mo, io.mold, io.Vo, io.vold, io.ema_o,  \
        io.frozen_o
    switch (io.degree) {
        case 0: k_dens_scatter<0><<<(unsigned)nb, kDB, 0, s>>>(GSTA_DENS_ARGS); break;
        case 1: k_dens_scatter<1><<<(unsigned)nb, kDB, 0, s>>>(GSTA_DENS_ARGS); break;
        case 2: k_dens_scatter<2><<<(unsigned)nb, kDB, 0, s>>>(GSTA_DENS_ARGS); break;
        default: k_dens_scatter<3><<<(unsigned)nb, kDB, 0, s>>>(GSTA_DENS_ARGS); break;
    }
#undef GSTA_DENS_ARGS
}

void launch_opacity_reset(float* P, int64_t ld, float* M, int64_t mld, float* V, int64_t vld, int64_t n,
                          const uint8_t* frozen, float cap, hipStream_t s) {
    if (n <= 0) return;
    k_opacity_reset<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, ld, M, mld, V, vld, n, frozen, cap);
}

void launch_opacity_to_abs(float* P, int64_t ld, float* M, int64_t mld, float* V, int64_t vld, int64_t n,
                           hipStream_t s) {
    if (n <= 0) return;
    k_opacity_to_abs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, ld, M, mld, V, vld, n);
}

void launch_partition(int64_t n, uint8_t* frozen, const PartArray* arrays, int count, void* tmp,
                      uint32_t* src, uint32_t* boff, uint32_t* tot, int64_t* n_active, hipStream_t s) {
    const int64_t nb = densify_blocks(n);
    if (nb > 0) k_part_count<<<(unsigned)nb, kDB, 0, s>>>(frozen, n, boff);
    k_part_scan<<<1, 1024, 0, s>>>(boff, nb, tot, n_active);
    if (n == 0) return;
    k_part_src<<<(unsigned)nb, kDB, 0, s>>>(frozen, n, boff, tot, src);
    const unsigned gx = (unsigned)((n + 255) / 256);
    for (int a = 0; a < count; ++a) {
        const PartArray& p = arrays[a];
        const dim3 grid(gx, (unsigned)std::min<int64_t>(p.rows, 64));
        switch (p.elem_bytes) {
            case 1:
                k_part_gather<uint8_t><<<grid, 256, 0, s>>>((const uint8_t*)p.base, p.ld, p.rows, src, n,
                                                            (uint8_t*)tmp);
                k_part_put<uint8_t><<<grid, 256, 0, s>>>((const uint8_t*)tmp, p.rows, n, (uint8_t*)p.base, p.ld);
                break;
            case 2:
                k_part_gather<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)p.base, p.ld, p.rows, src, n,
                                                             (uint16_t*)tmp);
                k_part_put<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)tmp, p.rows, n, (uint16_t*)p.base,
                                                          p.ld);
                break;
            default:
                k_part_gather<uint32_t><<<grid, 256, 0, s>>>((const uint32_t*)p.base, p.ld, p.rows, src, n,
                                                             (uint32_t*)tmp);
                k_part_put<uint32_t><<<grid, 256, 0, s>>>((const uint32_t*)tmp, p.rows, n, (uint32_t*)p.base,
                                                          p.ld);
                break;
        }
    }
    k_part_mask<<<gx, 256, 0, s>>>(frozen, n, tot);
}

}  // namespace gsta
