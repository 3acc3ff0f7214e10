// The ablation's naive freezing rules (Section 4.3, Table 3 rows "+mingrad"
// and "+random"), applied to the freeze map in place of the thresholds of
// eqs. 4-6.
//
// mingrad: among the Gaussians whose positional gradient-norm average is
// finite (below FLT_MAX: seen at least once), the m = floor(fraction * count)
// with the smallest average, equal averages taken in ascending index order.
// An exact radix select: four passes of 8-bit digits over an order-preserving
// 32-bit key find the m-th smallest key t (one workgroup histogram per pass,
// summed into 256 global bins, and a one-workgroup pick of the digit); every
// key below t is chosen, and of the keys equal to t the first `rem` in index
// order (per-block counts of equal keys, scanned, then ranked inside each
// block by ballot).  Runs once per freeze update, so 12 small launches.
//
// random: Gaussian i is chosen iff the top 32 bits of the first word of
// Philox4x64-10(counter = (i, draw, 0, 0), key = (seed, 0)) are below
// floor(fraction * 2^32) -- an independent Bernoulli(fraction) draw per
// Gaussian and update.  Philox4x64-10 is the counter-based generator of
// Salmon et al. (SC 2011), written here from its round function.
#include "gsta_internal.h"

namespace gsta {
namespace {

constexpr float kFltMax = 3.402823466e+38f;

__global__ void k_zero_count(unsigned long long* p) { *p = 0ull; }

// freeze map update with condition `cond` (mode 0: OR, 1: reset, 2: replace)
// and the frozen count by ballot, one atomic per 256-thread workgroup (every
// thread calls this; same-address atomics serialise)
__device__ __forceinline__ void apply_and_count(bool in, int64_t i, bool cond, int mode, uint8_t* frozen,
                                                unsigned long long* n_frozen) {
    bool f = false;
    if (in) {
        f = (mode == 0) ? ((frozen[i] != 0) || cond) : (mode == 1 ? false : cond);
        frozen[i] = f ? 1 : 0;
    }
    if (n_frozen) {
        __shared__ uint32_t s_c[4];
        const uint64_t b = __ballot(f);
        if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = (uint32_t)__popcll(b);
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t c = s_c[0] + s_c[1] + s_c[2] + s_c[3];
            if (c) atomicAdd(n_frozen, (unsigned long long)c);
        }
    }
}

__global__ __launch_bounds__(256) void k_freeze_random(int64_t n, uint64_t thr, uint64_t seed, uint64_t draw,
                                                       int mode, uint8_t* __restrict__ frozen,
                                                       unsigned long long* __restrict__ n_frozen) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool cond = false;
    if (i < n) {
        uint64_t c[4] = {(uint64_t)i, draw, 0ull, 0ull};
        philox4x64_10(c, seed, 0ull);
        cond = (c[0] >> 32) < thr;
    }
    apply_and_count(i < n, i, cond, mode, frozen, n_frozen);
}

// Order-preserving key of a float (equal floats, +0 and -0 included, give
// equal keys) and whether the Gaussian takes part (average below FLT_MAX).
__device__ __forceinline__ bool sel_key(float s, uint32_t& key) {
    uint32_t b = __float_as_uint(s);
    if (b == 0x80000000u) b = 0u;
    key = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return s < kFltMax;
}

__global__ __launch_bounds__(256) void k_sel_begin(SelState* st, unsigned long long* n_frozen) {
    st->hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        st->count = 0ull;
        st->rem = 0ull;
        st->prefix = 0u;
        st->none = 0u;
        if (n_frozen) *n_frozen = 0ull;
    }
}

// Histogram of digit (key >> shift) & 255 over the candidates whose digits
// above `shift` equal the prefix found so far; the first pass also counts
// the candidates.
__global__ __launch_bounds__(256) void k_sel_hist(const float* __restrict__ score, int64_t n, SelState* st,
                                                  int shift) {
    __shared__ uint32_t h[256];
    __shared__ unsigned long long s_cnt;
    h[threadIdx.x] = 0u;
    if (threadIdx.x == 0) s_cnt = 0ull;
    __syncthreads();
    const bool first = shift == 24;
    const uint32_t hi_mask = first ? 0u : (0xFFFFFFFFu << (shift + 8));
    const uint32_t prefix = st->prefix;
    uint32_t cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t key;
        if (!sel_key(score[i], key)) continue;
        ++cnt;
        if ((key & hi_mask) == (prefix & hi_mask)) atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    if (first && cnt) atomicAdd(&s_cnt, (unsigned long long)cnt);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
    if (first && threadIdx.x == 0 && s_cnt) atomicAdd(&st->count, s_cnt);
}

// Picks the digit at `shift` of the rem-th smallest key among those with the
// current prefix, then clears the histogram for the next pass.
__global__ __launch_bounds__(256) void k_sel_pick(SelState* st, int shift, double fraction) {
    if (threadIdx.x == 0) {
        if (shift == 24) {
            const uint64_t m = (uint64_t)floor(fraction * (double)st->count);
            st->rem = m;
            st->none = m == 0ull ? 1u : 0u;
        }
        if (!st->none) {
            uint64_t cum = 0, rem = st->rem;
            for (int d = 0; d < 256; ++d) {
                const uint64_t h = st->hist[d];
                if (cum + h >= rem) {
                    st->prefix |= (uint32_t)d << shift;
                    st->rem = rem - cum;
                    break;
                }
                cum += h;
            }
        }
    }
    __syncthreads();
    st->hist[threadIdx.x] = 0u;
}

// Per block of 256 Gaussians, how many candidates have the threshold key.
__global__ __launch_bounds__(256) void k_sel_eq_count(const float* __restrict__ score, int64_t n,
                                                      const SelState* st, uint32_t* __restrict__ blk) {
    __shared__ uint32_t s_w[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t key = 0;
    const bool eq = i < n && sel_key(score[i], key) && key == st->prefix && !st->none;
    const uint64_t b = __ballot(eq);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Exclusive scan of the per-block counts in place (one workgroup).
__global__ __launch_bounds__(1024) void k_sel_scan(uint32_t* blk, int nb) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0u;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int j = base + (int)threadIdx.x;
        const uint32_t x = j < nb ? blk[j] : 0u;
        uint32_t incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint32_t wb = s_carry;
        for (int k = 0; k < w; ++k) wb += s_w[k];
        if (j < nb) blk[j] = wb + incl - x;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = wb + incl;
        __syncthreads();
    }
}

// cond = key < t, or key == t among the first rem such keys in index order.
__global__ __launch_bounds__(256) void k_sel_mark(const float* __restrict__ score, int64_t n, const SelState* st,
                                                  const uint32_t* __restrict__ blk, int mode,
                                                  uint8_t* __restrict__ frozen,
                                                  unsigned long long* __restrict__ n_frozen) {
    __shared__ uint32_t s_w[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t key = 0;
    const bool none = st->none != 0u;
    const bool cand = i < n && sel_key(score[i], key) && !none;
    const uint32_t t = st->prefix;
    const bool eq = cand && key == t;
    const uint64_t b = __ballot(eq);
    if (lane == 0) s_w[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t rank = blk[blockIdx.x] + (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
    for (int k = 0; k < w; ++k) rank += s_w[k];
    const bool cond = cand && (key < t || (eq && (uint64_t)rank < st->rem));
    apply_and_count(i < n, i, cond, mode, frozen, n_frozen);
}

}  // namespace

void launch_freeze_random(int64_t n, uint64_t thr, uint64_t seed, uint64_t draw, int mode, uint8_t* frozen,
                          int64_t* n_frozen, hipStream_t s) {
    auto* nf = reinterpret_cast<unsigned long long*>(n_frozen);
    if (nf) k_zero_count<<<1, 1, 0, s>>>(nf);
    if (n > 0) k_freeze_random<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, thr, seed, draw, mode, frozen, nf);
}

void launch_freeze_mingrad(const float* score, int64_t n, double fraction, int mode, uint8_t* frozen,
                           int64_t* n_frozen, SelState* st, uint32_t* blk, hipStream_t s) {
    auto* nf = reinterpret_cast<unsigned long long*>(n_frozen);
    k_sel_begin<<<1, 256, 0, s>>>(st, nf);
    if (n <= 0) return;
    const int nb = (int)((n + 255) / 256);
    const int hb = nb < 1024 ? nb : 1024;
    for (int shift = 24; shift >= 0; shift -= 8) {
        k_sel_hist<<<hb, 256, 0, s>>>(score, n, st, shift);
        k_sel_pick<<<1, 256, 0, s>>>(st, shift, fraction);
    }
    k_sel_eq_count<<<nb, 256, 0, s>>>(score, n, st, blk);
    k_sel_scan<<<1, 1024, 0, s>>>(blk, nb);
    k_sel_mark<<<nb, 256, 0, s>>>(score, n, st, blk, mode, frozen, nf);
}

}  // namespace gsta
