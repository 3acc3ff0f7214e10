// Depth sort, tile binning and tile ranges.
//
// The paper blends Gaussians in depth order (Section 3.1).  Here the order
// is (float32 camera depth, gid) per view, made in two stages:
//   1. a stable LSD radix sort of the N depth keys of every view (the
//      culled ones carry the largest key and sort last);
//   2. per tile, the list of the Gaussians whose 3-sigma rectangle covers
//      it, in that order: either placed directly (views of at most
//      kPlaceMaxTiles tiles, see "Direct tile placement" below), or through
//      a depth-ordered expansion of each Gaussian into one (view*T + tile,
//      gid) instance per tile of its rectangle, followed by a stable radix
//      sort of those 16-bit-or-less tile keys (stability keeps the depth
//      order inside every tile).
//
// Radix sort: 8-bit digits, chunks of 256, 1024 or 4096 keys per workgroup
// iteration (small, mid-size and large sorts).
//   hist    per-chunk digit counts -> hist[seg][digit][chunk]
//   scan    one workgroup per (digit, seg) scans its chunk counts
//   scatter per chunk: each wave ranks its contiguous quarter stably with
//           ballots and its own LDS digit counters (no block barrier per
//           item), keys are staged in LDS in digit order, then written out
//           with consecutive lanes hitting consecutive addresses.
// Counts may live on the device (the instance count is only known there):
// kernels then run a grid-stride loop over the chunks that exist.
#include "gsta_internal.h"

#include <algorithm>

namespace gsta {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_BINS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;

__device__ __forceinline__ uint32_t seg_count(const uint32_t* d_count, uint32_t h_count) {
    return d_count ? *d_count : h_count;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_tmp[wid] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
        uint32_t t = s_tmp[w];
        base += (w < wid) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + incl - x;
}

template <int RS_ITEMS>
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                           int64_t seg_stride, const uint32_t* d_count,
                                                           uint32_t h_count, int shift, uint32_t dmask,
                                                           uint32_t* __restrict__ hist,
                                                           int64_t nchunks_cap) {
    constexpr int RS_CHUNK = RS_THREADS * RS_ITEMS;
    __shared__ uint32_t s_h[RS_BINS];
    const int seg = blockIdx.y;
    const uint32_t count = seg_count(d_count, h_count);
    const int64_t nchunks = ((int64_t)count + RS_CHUNK - 1) / RS_CHUNK;
    const uint32_t* k = keys + seg * seg_stride;
    for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        s_h[threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = chunk * RS_CHUNK;
#pragma unroll 4
        for (int it = 0; it < RS_ITEMS; ++it) {
            int64_t idx = base + it * RS_THREADS + threadIdx.x;
            if (idx < count) atomicAdd(&s_h[(k[idx] >> shift) & dmask], 1u);
        }
        __syncthreads();
        hist[((int64_t)seg * RS_BINS + threadIdx.x) * nchunks_cap + chunk] = s_h[threadIdx.x];
        __syncthreads();
    }
}

// One workgroup per (digit, segment): exclusive scan over the chunks.
template <int RS_ITEMS>
__global__ __launch_bounds__(RS_THREADS) void k_radix_scan(uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ digit_tot,
                                                           const uint32_t* d_count, uint32_t h_count,
                                                           int64_t nchunks_cap) {
    constexpr int RS_CHUNK = RS_THREADS * RS_ITEMS;
    __shared__ uint32_t s_tmp[RS_WAVES];
    const int d = blockIdx.x, seg = blockIdx.y;
    const uint32_t count = seg_count(d_count, h_count);
    const int64_t nchunks = ((int64_t)count + RS_CHUNK - 1) / RS_CHUNK;
    uint32_t* row = hist + ((int64_t)seg * RS_BINS + d) * nchunks_cap;
    uint32_t carry = 0;
    for (int64_t b = 0; b < nchunks; b += RS_THREADS) {
        int64_t j = b + threadIdx.x;
        uint32_t x = (j < nchunks) ? row[j] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan_256(x, s_tmp, tot);
        if (j < nchunks) row[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) digit_tot[seg * RS_BINS + d] = carry;
}

template <int RS_ITEMS>
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t seg_stride, const uint32_t* d_count, uint32_t h_count, int shift,
    int bits, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_tot,
    int64_t nchunks_cap) {
    constexpr int RS_CHUNK = RS_THREADS * RS_ITEMS;
    constexpr int WSPAN = 64 * RS_ITEMS;           // keys of one wave in a chunk
    const uint32_t dmask = (1u << bits) - 1u;      // digits of this pass
    __shared__ uint32_t s_keys[RS_CHUNK];
    __shared__ uint32_t s_vals[RS_CHUNK];
    __shared__ uint32_t s_digit_base[RS_BINS];
    __shared__ uint32_t s_cnt[RS_WAVES][RS_BINS];
    __shared__ uint32_t s_local_start[RS_BINS];
    __shared__ uint32_t s_gbase[RS_BINS];
    __shared__ uint32_t s_tmp[RS_WAVES];

    const int seg = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint32_t count = seg_count(d_count, h_count);
    const int64_t nchunks = ((int64_t)count + RS_CHUNK - 1) / RS_CHUNK;
    const uint32_t* ki = kin + seg * seg_stride;
    const uint32_t* vi = vin + seg * seg_stride;
    uint32_t* ko = kout + seg * seg_stride;
    uint32_t* vo = vout + seg * seg_stride;
    const uint32_t* hrow = hist + (int64_t)seg * RS_BINS * nchunks_cap;

    {   // global start of each digit = exclusive scan of the digit totals
        uint32_t tot;
        uint32_t ex = block_excl_scan_256(digit_tot[seg * RS_BINS + tid], s_tmp, tot);
        s_digit_base[tid] = ex;
    }

    for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        const int64_t base = chunk * RS_CHUNK;
        const int n_valid = (int)min((int64_t)RS_CHUNK, (int64_t)count - base);
        // wave w takes the keys [w * WSPAN, (w + 1) * WSPAN) of the chunk, item by item
        uint32_t key[RS_ITEMS], val[RS_ITEMS], rank[RS_ITEMS];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const int j = wid * WSPAN + it * 64 + lane;
            const bool ok = j < n_valid;
            key[it] = ok ? ki[base + j] : 0u;
            val[it] = ok ? vi[base + j] : 0u;
        }
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) s_cnt[w][tid] = 0;
        __syncthreads();

        // Stable ranks inside the wave: lanes with the same digit found by
        // ballots; the wave's running count per digit lives in LDS (the
        // wave's own reads precede its own writes, so no barrier is needed).
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const int j = wid * WSPAN + it * 64 + lane;
            const bool ok = j < n_valid;
            const uint32_t d = (key[it] >> shift) & dmask;
            uint64_t match = __ballot(ok);
            for (int b = 0; b < bits; ++b) {
                const uint64_t bal = __ballot(ok && ((d >> b) & 1u));
                match &= ((d >> b) & 1u) ? bal : ~bal;
            }
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(match >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)match, 0u));
            const uint32_t before = ok ? s_cnt[wid][d] : 0u;
            __builtin_amdgcn_wave_barrier();
            if (ok && below == 0) s_cnt[wid][d] = before + (uint32_t)__popcll(match);
            __builtin_amdgcn_wave_barrier();
            rank[it] = before + below;
        }
        __syncthreads();
        uint32_t dtot = 0;
        {   // per digit: offsets of the waves, then the chunk-local start
#pragma unroll
            for (int w = 0; w < RS_WAVES; ++w) {
                const uint32_t c = s_cnt[w][tid];
                s_cnt[w][tid] = dtot;
                dtot += c;
            }
            uint32_t tot;
            const uint32_t ls = block_excl_scan_256(dtot, s_tmp, tot);
            s_local_start[tid] = ls;
            // global position of the chunk's first key of digit tid, minus its local start
            s_gbase[tid] = s_digit_base[tid] + hrow[(int64_t)tid * nchunks_cap + chunk] - ls;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const int j = wid * WSPAN + it * 64 + lane;
            if (j < n_valid) {
                const uint32_t d = (key[it] >> shift) & dmask;
                const uint32_t pos = s_local_start[d] + s_cnt[wid][d] + rank[it];
                if (pos < (uint32_t)RS_CHUNK) {
                    s_keys[pos] = key[it];
                    s_vals[pos] = val[it];
                }
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int it = 0; it < RS_ITEMS; ++it) {
            const int p = it * RS_THREADS + tid;
            if (p < n_valid) {
                const uint32_t k = s_keys[p];
                const uint32_t g = s_gbase[(k >> shift) & dmask] + (uint32_t)p;
                if (g < count) {
                    ko[g] = k;
                    vo[g] = s_vals[p];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Onesweep radix sort (one kernel per pass) for sorts whose key count is
// known on the host, used for the per-view depth sort.  A first kernel
// counts the digits of every pass over all keys (global histograms) and
// clears the pass state; then each pass is one kernel in which every
// workgroup takes the next chunk by ticket, ranks its keys stably (as the
// scatter above), publishes its per-digit counts, and finds how many keys of
// each digit the earlier chunks hold by decoupled look-back: the status word
// of (chunk, digit) carries the chunk's own count (flag AGG) or the count of
// every chunk up to and including it (flag INC), and a workgroup sums its
// predecessors' words backwards, eight at a time, until it meets an INC.
// Tickets make every predecessor's workgroup resident before its successor
// starts, and each publishes its AGG words before looking back, so every
// wait ends; a spin bound turns a wait that does not into a device flag.
// ---------------------------------------------------------------------------
constexpr int OS_ITEMS = 8;
constexpr int OS_CHUNK = RS_THREADS * OS_ITEMS;      // 2048 keys per workgroup
constexpr uint32_t OS_AGG = 1u << 30, OS_INC = 2u << 30, OS_CNT = (1u << 30) - 1u;
constexpr uint32_t OS_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint32_t os_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void os_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Global digit counts of every pass (tot[seg][pass][256], cleared with the
// tickets by k_os_clear), and this chunk's look-back words of every pass
// cleared: status[seg][pass][chunk][256].
__global__ __launch_bounds__(RS_THREADS) void k_os_totals(const uint32_t* __restrict__ keys, int64_t seg_stride,
                                                          uint32_t count, int passes, int per,
                                                          uint32_t* __restrict__ tot, uint32_t* __restrict__ status,
                                                          uint32_t* __restrict__ tickets, int64_t nchunks) {
    __shared__ uint32_t s_h[4][RS_BINS];
    const int seg = blockIdx.y, tid = threadIdx.x;
    const int64_t chunk = blockIdx.x;
#pragma unroll
    for (int p = 0; p < 4; ++p) s_h[p][tid] = 0u;
    // this chunk's status words of every pass, and (first chunk) the tickets and totals
    for (int p = 0; p < passes; ++p) status[(((int64_t)seg * 4 + p) * nchunks + chunk) * RS_BINS + tid] = 0u;
    __syncthreads();
    const uint32_t* k = keys + seg * seg_stride;
    const uint32_t dmask = (1u << per) - 1u;
    for (int it = 0; it < OS_ITEMS; ++it) {
        const int64_t idx = chunk * OS_CHUNK + (int64_t)it * RS_THREADS + tid;
        if (idx < count) {
            const uint32_t key = k[idx];
            for (int p = 0; p < passes; ++p) atomicAdd(&s_h[p][(key >> (p * per)) & dmask], 1u);
        }
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        if (s_h[p][tid]) atomicAdd(&tot[((int64_t)seg * 4 + p) * RS_BINS + tid], s_h[p][tid]);
}

__global__ void k_os_clear(uint32_t* __restrict__ tot, uint32_t* __restrict__ tickets, int nseg) {
    for (int i = threadIdx.x; i < nseg * 4 * RS_BINS; i += blockDim.x) tot[i] = 0u;
    for (int i = threadIdx.x; i < nseg * 4; i += blockDim.x) tickets[i] = 0u;
}

__global__ __launch_bounds__(RS_THREADS) void k_os_pass(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t seg_stride, uint32_t count, int pass, int shift, int bits,
    const uint32_t* __restrict__ tot, uint32_t* __restrict__ status, uint32_t* __restrict__ tickets,
    int64_t nchunks, uint32_t* __restrict__ flags) {
    constexpr int WSPAN = 64 * OS_ITEMS;
    const uint32_t dmask = (1u << bits) - 1u;
    __shared__ uint32_t s_keys[OS_CHUNK];
    __shared__ uint32_t s_vals[OS_CHUNK];
    __shared__ uint32_t s_cnt[RS_WAVES][RS_BINS];
    __shared__ uint32_t s_local_start[RS_BINS];
    __shared__ uint32_t s_gbase[RS_BINS];
    __shared__ uint32_t s_tmp[RS_WAVES];
    __shared__ uint32_t s_chunk;
    const int seg = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) s_chunk = atomicAdd(&tickets[seg * 4 + pass], 1u);
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) s_cnt[w][tid] = 0;
    __syncthreads();
    const int64_t chunk = s_chunk;
    uint32_t* st = status + ((int64_t)seg * 4 + pass) * nchunks * RS_BINS;
    const uint32_t* ki = kin + seg * seg_stride;
    const uint32_t* vi = vin + seg * seg_stride;
    uint32_t* ko = kout + seg * seg_stride;
    uint32_t* vo = vout + seg * seg_stride;
    const int64_t base = chunk * OS_CHUNK;
    const int n_valid = (int)min((int64_t)OS_CHUNK, (int64_t)count - base);
    uint32_t key[OS_ITEMS], val[OS_ITEMS], rank[OS_ITEMS];
#pragma unroll
    for (int it = 0; it < OS_ITEMS; ++it) {
        const int j = wid * WSPAN + it * 64 + lane;
        const bool ok = j < n_valid;
        key[it] = ok ? ki[base + j] : 0u;
        val[it] = ok ? vi[base + j] : 0u;
    }
    // stable ranks inside each wave (ballots) with the wave's digit counters in LDS
#pragma unroll
    for (int it = 0; it < OS_ITEMS; ++it) {
        const int j = wid * WSPAN + it * 64 + lane;
        const bool ok = j < n_valid;
        const uint32_t d = (key[it] >> shift) & dmask;
        uint64_t match = __ballot(ok);
        for (int b = 0; b < bits; ++b) {
            const uint64_t bal = __ballot(ok && ((d >> b) & 1u));
            match &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(match >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)match, 0u));
        const uint32_t before = ok ? s_cnt[wid][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) s_cnt[wid][d] = before + (uint32_t)__popcll(match);
        __builtin_amdgcn_wave_barrier();
        rank[it] = before + below;
    }
    __syncthreads();
    uint32_t dtot = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
        const uint32_t c = s_cnt[w][tid];
        s_cnt[w][tid] = dtot;
        dtot += c;
    }
    // publish this chunk's count of digit tid, then look back for the earlier chunks'
    if (chunk == 0) {
        os_store(&st[tid], OS_INC | dtot);
    } else {
        os_store(&st[chunk * RS_BINS + tid], OS_AGG | dtot);
    }
    uint32_t excl = 0;
    if (chunk > 0) {
        int64_t j = chunk - 1;
        uint32_t spins = 0;
        bool done = false;
        while (!done && j >= 0) {
            uint32_t v[8];
            const int m = (int)min((int64_t)8, j + 1);
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = t < m ? os_load(&st[(j - t) * RS_BINS + tid]) : 0u;
            int t = 0;
            for (; t < m; ++t) {
                const uint32_t f = v[t] & ~OS_CNT;
                if (f == 0u) break;
                excl += v[t] & OS_CNT;
                if (f == OS_INC) {
                    done = true;
                    ++t;
                    break;
                }
            }
            j -= t;
            if (t == 0 && ++spins > OS_SPIN_LIMIT) {
                atomicOr(&flags[4], 1u);
                done = true;
            }
        }
        os_store(&st[chunk * RS_BINS + tid], OS_INC | (excl + dtot));
    }
    {
        uint32_t total_all;
        const uint32_t dbase = block_excl_scan_256(tot[((int64_t)seg * 4 + pass) * RS_BINS + tid], s_tmp, total_all);
        uint32_t t2;
        const uint32_t ls = block_excl_scan_256(dtot, s_tmp, t2);
        s_local_start[tid] = ls;
        s_gbase[tid] = dbase + excl - ls;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < OS_ITEMS; ++it) {
        const int j = wid * WSPAN + it * 64 + lane;
        if (j < n_valid) {
            const uint32_t d = (key[it] >> shift) & dmask;
            const uint32_t pos = s_local_start[d] + s_cnt[wid][d] + rank[it];
            if (pos < (uint32_t)OS_CHUNK) {
                s_keys[pos] = key[it];
                s_vals[pos] = val[it];
            }
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int it = 0; it < OS_ITEMS; ++it) {
        const int p = it * RS_THREADS + tid;
        if (p < n_valid) {
            const uint32_t k = s_keys[p];
            const uint32_t g = s_gbase[(k >> shift) & dmask] + (uint32_t)p;
            if (g < count) {
                ko[g] = k;
                vo[g] = s_vals[p];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Depth-ordered expansion into tile instances.
// Element e = v*n + pos is the pos-th Gaussian of view v in depth order.
// ---------------------------------------------------------------------------
constexpr int EX_THREADS = 256;
constexpr int kExWin = 8192;    // instances per owner window of the expansion

__device__ __forceinline__ uint32_t rect_tiles(ushort4 r) {
    return (r.x < r.y && r.z < r.w) ? (uint32_t)(r.y - r.x) * (uint32_t)(r.w - r.z) : 0u;
}

__global__ __launch_bounds__(EX_THREADS) void k_tile_count(const ushort4* __restrict__ rect,
                                                           const uint32_t* __restrict__ order,
                                                           int64_t stride, int64_t n, int64_t total_el,
                                                           uint64_t* __restrict__ partials, Clears cl) {
    __shared__ uint32_t s_tmp[RS_WAVES];
    // buffers the rest of the forward expects zeroed (tile ranges, the
    // compositing's per-tile last member and checkpoint counter)
    for (int b = 0; b < Clears::kMax; ++b)
        for (int64_t j = (int64_t)blockIdx.x * EX_THREADS + threadIdx.x; j < cl.count[b];
             j += (int64_t)gridDim.x * EX_THREADS)
            cl.ptr[b][j] = 0u;
    const int64_t e = (int64_t)blockIdx.x * EX_THREADS + threadIdx.x;
    uint32_t c = 0;
    if (e < total_el) {
        const int64_t v = e / n, pos = e - v * n;
        const uint32_t gid = order[v * stride + pos];
        c = rect_tiles(rect[v * stride + gid]);
    }
    uint32_t tot;
    block_excl_scan_256(c, s_tmp, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One 1024-thread workgroup: exclusive scan of the per-block instance counts
// (uint64), the total, the clamped count and the overflow report.
__device__ __forceinline__ void scan_partials_block(uint64_t* __restrict__ partials, int64_t nb,
                                                    uint64_t* __restrict__ d_total,
                                                    uint32_t* __restrict__ d_count, uint64_t capacity,
                                                    uint32_t* flags, uint64_t* max_inst, uint64_t* s_w) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint64_t carry = 0;
    for (int64_t b = 0; b < nb; b += 1024) {
        int64_t j = b + tid;
        uint64_t x = (j < nb) ? partials[j] : 0ull;
        uint64_t incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            uint64_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[wid] = incl;
        __syncthreads();
        uint64_t base = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            uint64_t t = s_w[w];
            base += (w < wid) ? t : 0ull;
            tot += t;
        }
        __syncthreads();
        if (j < nb) partials[j] = carry + base + incl - x;
        carry += tot;
    }
    if (tid == 0) {
        *d_total = carry;
        *d_count = (uint32_t)(carry < capacity ? carry : capacity);
        if (carry > capacity) atomicOr(&flags[0], 1u);
        atomicMax((unsigned long long*)max_inst, (unsigned long long)carry);
    }
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t* __restrict__ partials, int64_t nb,
                                                        uint64_t* __restrict__ d_total,
                                                        uint32_t* __restrict__ d_count,
                                                        uint64_t capacity, uint32_t* flags,
                                                        uint64_t* max_inst) {
    __shared__ uint64_t s_w[16];
    scan_partials_block(partials, nb, d_total, d_count, capacity, flags, max_inst, s_w);
}

__global__ __launch_bounds__(EX_THREADS) void k_expand(const ushort4* __restrict__ rect,
                                                       const uint32_t* __restrict__ order, int64_t stride,
                                                       int64_t n, int64_t total_el, int ntx,
                                                       int tiles_per_view,
                                                       const uint64_t* __restrict__ partials,
                                                       uint32_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals,
                                                       uint4* __restrict__ rank_tab,
                                                       uint32_t* __restrict__ inst_off, uint64_t capacity) {
    __shared__ uint32_t s_tmp[RS_WAVES];
    __shared__ uint32_t s_off[EX_THREADS + 1];
    __shared__ uint32_t s_gid[EX_THREADS];
    __shared__ ushort4 s_rect[EX_THREADS];
    __shared__ uint32_t s_view[EX_THREADS];
    __shared__ uint8_t s_owner[kExWin];
    static_assert(EX_THREADS <= 256, "block-local Gaussian indices are stored in bytes");
    const int tid = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x * EX_THREADS + tid;
    uint32_t c = 0;
    if (e < total_el) {
        const int64_t v = e / n, pos = e - v * n;
        const uint32_t gid = order[v * stride + pos];
        const ushort4 r = rect[v * stride + gid];
        c = rect_tiles(r);
        s_gid[tid] = gid;
        s_rect[tid] = r;
        s_view[tid] = (uint32_t)v;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan_256(c, s_tmp, tot);
    s_off[tid] = ex;
    if (tid == 0) s_off[EX_THREADS] = tot;
    __syncthreads();
    const uint64_t base = partials[blockIdx.x];
    if (e < total_el) {
        const uint64_t first = base + ex;
        const uint32_t f32 = (uint32_t)(first < capacity ? first : capacity);
        const int64_t v = s_view[tid];
        inst_off[v * stride + s_gid[tid]] = f32;
        // what the ranges pass needs of this depth rank: gid, first instance, rectangle
        const ushort4 r = s_rect[tid];
        rank_tab[v * stride + (e - v * n)] =
            make_uint4(s_gid[tid], f32, (uint32_t)r.x | ((uint32_t)r.y << 16), (uint32_t)r.z | ((uint32_t)r.w << 16));
    }
    // Every instance of this block's Gaussians, one per thread in turn, in
    // windows of kExWin instances: each Gaussian first marks its instances of
    // the window with its block-local index (s_owner), then every thread
    // reads the owner of its instance instead of searching the offsets.
    for (uint32_t w0 = 0; w0 < tot; w0 += kExWin) {
        const uint32_t w1 = min(tot, w0 + (uint32_t)kExWin);
        if (c > 0) {
            const uint32_t a = max(ex, w0), b = min(ex + c, w1);
            for (uint32_t j = a; j < b; ++j) s_owner[j - w0] = (uint8_t)tid;
        }
        __syncthreads();
        for (uint32_t j = w0 + tid; j < w1; j += EX_THREADS) {
            const int lo = s_owner[j - w0];
            const ushort4 r = s_rect[lo];
            const uint32_t t = j - s_off[lo];
            const uint32_t w = (uint32_t)(r.y - r.x);
            const uint32_t tx = r.x + t % w, ty = r.z + t / w;
            const uint64_t dst = base + j;
            if (dst < capacity) {
                keys[dst] = s_view[lo] * (uint32_t)tiles_per_view + ty * (uint32_t)ntx + tx;
                // the Gaussian's depth rank in its view (the sort is stable, so ranks
                // stay increasing within each tile)
                vals[dst] = (uint32_t)((int64_t)blockIdx.x * EX_THREADS + lo - (int64_t)s_view[lo] * n);
            }
        }
        __syncthreads();
    }
}

// From the sorted (tile key, depth rank) pairs: the tile ranges, the gid at
// each list position and, in place of the rank, the instance's expansion
// index (its Gaussian's first instance + its tile's place in the rectangle).
// One 16-byte read per position from the rank table, whose entries of a
// tile's list are in increasing rank order.
__global__ void k_ranges(const uint32_t* __restrict__ keys, uint32_t* __restrict__ ids,
                         const uint4* __restrict__ rank_tab, int64_t stride, uint32_t tiles_per_view,
                         uint32_t ntx, const uint32_t* d_count, uint2* __restrict__ ranges,
                         uint32_t* __restrict__ gsort) {
    const uint32_t count = *d_count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[i];
        const uint32_t v = k / tiles_per_view, t = k - v * tiles_per_view;
        const uint4 rt = rank_tab[(int64_t)v * stride + ids[i]];
        const uint32_t ty = t / ntx, tx = t - ty * ntx;
        const uint32_t x0 = rt.z & 0xFFFFu, x1 = rt.z >> 16, y0 = rt.w & 0xFFFFu;
        gsort[i] = rt.x;
        ids[i] = rt.y + (ty - y0) * (x1 - x0) + (tx - x0);
        if (i == 0 || keys[i - 1] != k) ranges[k].x = (uint32_t)i;
        if (i + 1 == count || keys[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
    }
}

// ---------------------------------------------------------------------------
// Direct tile placement (views of at most kPlaceMaxTiles tiles): the
// tile-major, depth-ordered instance list without a key sort.
// A Gaussian covers each tile of its rectangle once, so inside a block of
// 256 consecutive Gaussians of the depth order, the place of a Gaussian's
// instance among the block's instances of tile t is the number of earlier
// Gaussians of the block covering t: a popcount over a 256-bit mask per
// tile.  Blocks follow the depth order too, so with the per-(block, tile)
// counts scanned down each tile's column, every instance has its final
// position, the one the stable tile-key sort gives it.
//   k_place_count  per block: cnt[v][b][t], the block's instance total
//                  (+ the clears of the forward)
//   k_place_scan   per 64 tiles: exclusive scan of cnt down the blocks and
//                  tile totals; one extra workgroup scans the block totals
//   k_place_write  per block: masks, ranks, ids and gsort (gid per list
//                  position); the view's first block writes the tile ranges
// ---------------------------------------------------------------------------
constexpr int PL_THREADS = 1024;                  // threads per placement workgroup
constexpr int PL_GAUSS = 256;                     // Gaussians per block (4 x 64-bit masks per tile)
constexpr int PL_PARTS = PL_THREADS / PL_GAUSS;   // threads per Gaussian in per-Gaussian loops
constexpr int PL_WAVES = PL_THREADS / 64;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a 1024-thread block.
__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(x);
    if (lane == 63) s_tmp[wid] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < PL_WAVES; ++w) {
        const uint32_t t = s_tmp[w];
        base += (w < wid) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + incl - x;
}

// k / w and k % w for k < 2^20, 1 <= w < 2^11: the float quotient is within
// one of the true one, and one correction step makes it exact.
__device__ __forceinline__ uint32_t divmod_small(uint32_t k, uint32_t w, uint32_t& r) {
    uint32_t q = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)w));
    int rr = (int)k - (int)(q * w);
    if (rr < 0) {
        --q;
        rr += (int)w;
    } else if (rr >= (int)w) {
        ++q;
        rr -= (int)w;
    }
    r = (uint32_t)rr;
    return q;
}

// The block's Gaussians (positions b*256 + i of view v's depth order, i < 256):
// gid, rectangle and the exclusive scan of their tile counts (s_off[256] = total).
__device__ __forceinline__ uint32_t place_load(const ushort4* __restrict__ rect, const uint32_t* __restrict__ order,
                                               int64_t stride, int64_t n, int v, int b, ushort4* s_rect,
                                               uint32_t* s_gid, uint32_t* s_off, uint32_t* s_tmp) {
    const int tid = threadIdx.x;
    const int64_t pos = (int64_t)b * PL_GAUSS + tid;
    uint32_t c = 0;
    if (tid < PL_GAUSS) {
        uint32_t gid = 0;
        ushort4 r = make_ushort4(0, 0, 0, 0);
        if (pos < n) {
            gid = order[(int64_t)v * stride + pos];
            r = rect[(int64_t)v * stride + gid];
            c = rect_tiles(r);
        }
        s_gid[tid] = gid;
        s_rect[tid] = r;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan_1024(c, s_tmp, tot);
    if (tid < PL_GAUSS) s_off[tid] = ex;
    if (tid == 0) s_off[PL_GAUSS] = tot;
    __syncthreads();
    return tot;
}

// Per block: cnt[v][b][t] = Gaussians of the block covering tile t, from a
// 2-D difference array over the tile grid (four updates per rectangle, then
// prefix sums along rows and columns); partials[v*nb + b] = instances.
__global__ __launch_bounds__(PL_THREADS) void k_place_count(const ushort4* __restrict__ rect,
                                                            const uint32_t* __restrict__ order, int64_t stride,
                                                            int64_t n, int nb, int ntx, int nty,
                                                            uint32_t* __restrict__ cnt,
                                                            uint64_t* __restrict__ partials, Clears cl) {
    extern __shared__ uint32_t s_d[];     // [nty + 1][ntx + 1]
    __shared__ uint32_t s_tmp[PL_WAVES];
    __shared__ uint32_t s_off[PL_GAUSS + 1];
    __shared__ uint32_t s_gid[PL_GAUSS];
    __shared__ ushort4 s_rect[PL_GAUSS];
    {   // buffers the rest of the forward expects zeroed
        const int64_t nthreads = (int64_t)gridDim.x * gridDim.y * PL_THREADS;
        const int64_t t0 = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * PL_THREADS + threadIdx.x;
        for (int k = 0; k < Clears::kMax; ++k)
            for (int64_t j = t0; j < cl.count[k]; j += nthreads) cl.ptr[k][j] = 0u;
    }
    const int b = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int pitch = ntx + 1, T = ntx * nty;
    for (int i = tid; i < (nty + 1) * pitch; i += PL_THREADS) s_d[i] = 0;
    const uint32_t tot = place_load(rect, order, stride, n, v, b, s_rect, s_gid, s_off, s_tmp);
    if (tid == 0) partials[(int64_t)v * nb + b] = tot;
    if (tid < PL_GAUSS) {
        const ushort4 r = s_rect[tid];
        if (rect_tiles(r) > 0) {
            atomicAdd(&s_d[r.z * pitch + r.x], 1u);
            atomicAdd(&s_d[r.z * pitch + r.y], 0xFFFFFFFFu);
            atomicAdd(&s_d[r.w * pitch + r.x], 0xFFFFFFFFu);
            atomicAdd(&s_d[r.w * pitch + r.y], 1u);
        }
    }
    __syncthreads();
    for (int y = wid; y < nty; y += PL_WAVES) {          // along each row
        uint32_t carry = 0;
        for (int x0 = 0; x0 < ntx; x0 += 64) {
            const int x = x0 + lane;
            const uint32_t incl = wave_incl_scan(x < ntx ? s_d[y * pitch + x] : 0u) + carry;
            if (x < ntx) s_d[y * pitch + x] = incl;
            carry = __shfl(incl, 63, 64);
        }
    }
    __syncthreads();
    for (int x = wid; x < ntx; x += PL_WAVES) {          // down each column
        uint32_t carry = 0;
        for (int y0 = 0; y0 < nty; y0 += 64) {
            const int y = y0 + lane;
            const uint32_t incl = wave_incl_scan(y < nty ? s_d[y * pitch + x] : 0u) + carry;
            if (y < nty) s_d[y * pitch + x] = incl;
            carry = __shfl(incl, 63, 64);
        }
    }
    __syncthreads();
    uint32_t* row = cnt + ((int64_t)v * nb + b) * T;
    for (int t = tid; t < T; t += PL_THREADS) {
        uint32_t x;
        const uint32_t y = divmod_small((uint32_t)t, (uint32_t)ntx, x);
        row[t] = s_d[y * pitch + x];
    }
}

// Blocks x < ceil(T/64): 64 tiles of view y, 16 waves over the blocks b.
// Block x == ceil(T/64) of view 0: the block totals.
constexpr int PL_SCAN_REG = 32;   // column entries a wave keeps in registers
__global__ __launch_bounds__(1024) void k_place_scan(uint32_t* __restrict__ cnt, int nb, int T,
                                                     uint32_t* __restrict__ tile_tot,
                                                     uint64_t* __restrict__ partials, int64_t nparts,
                                                     uint64_t* __restrict__ d_total,
                                                     uint32_t* __restrict__ d_count, uint64_t capacity,
                                                     uint32_t* flags, uint64_t* max_inst) {
    __shared__ uint32_t s_part[16][64];
    __shared__ uint64_t s_w[16];
    const int gT = (T + 63) / 64;
    if ((int)blockIdx.x == gT) {
        if (blockIdx.y == 0) scan_partials_block(partials, nparts, d_total, d_count, capacity, flags, max_inst, s_w);
        return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, v = blockIdx.y;
    const int t = blockIdx.x * 64 + lane;
    const int per = (nb + 15) / 16;
    const int b0 = min(nb, w * per), b1 = min(nb, b0 + per);
    uint32_t* col = cnt + (int64_t)v * nb * T + t;
    const bool inreg = per <= PL_SCAN_REG;
    uint32_t x[PL_SCAN_REG];
    uint32_t sum = 0;
    if (inreg) {
#pragma unroll
        for (int i = 0; i < PL_SCAN_REG; ++i) {
            x[i] = (t < T && b0 + i < b1) ? col[(int64_t)(b0 + i) * T] : 0u;
            sum += x[i];
        }
    } else if (t < T) {
#pragma unroll 8
        for (int bb = b0; bb < b1; ++bb) sum += col[(int64_t)bb * T];
    }
    s_part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t y = s_part[k][lane];
        run += (k < w) ? y : 0u;
        tot += y;
    }
    if (t < T) {
        if (inreg) {
#pragma unroll
            for (int i = 0; i < PL_SCAN_REG; ++i) {
                if (b0 + i < b1) col[(int64_t)(b0 + i) * T] = run;
                run += x[i];
            }
        } else {
#pragma unroll 8
            for (int bb = b0; bb < b1; ++bb) {
                const uint32_t y = col[(int64_t)bb * T];
                col[(int64_t)bb * T] = run;
                run += y;
            }
        }
        if (w == 0) tile_tot[(int64_t)v * T + t] = tot;
    }
}

// The index (0..255) of the k-th set bit of a tile's 256-bit mask (k < its popcount).
__device__ __forceinline__ uint32_t mask_select(const uint64_t* s_mask, int T, int t, uint32_t k) {
    uint64_t m = s_mask[t];
    uint32_t base = 0;
#pragma unroll
    for (int q = 1; q < 4; ++q) {
        const uint32_t pc = (uint32_t)__popcll(m);
        if (k >= pc) {
            k -= pc;
            m = s_mask[q * T + t];
            base += 64;
        }
    }
    uint32_t x = (uint32_t)m, pc = (uint32_t)__popc(x);
    if (k >= pc) {
        k -= pc;
        x = (uint32_t)(m >> 32);
        base += 32;
    }
#pragma unroll
    for (int h = 16; h >= 1; h >>= 1) {
        pc = (uint32_t)__popc(x & ((1u << h) - 1u));
        if (k >= pc) {
            k -= pc;
            x >>= h;
            base += (uint32_t)h;
        }
    }
    return base;
}

constexpr int64_t kPlaceStaticLds = 4352;
static_assert(65536 - kPlaceStaticLds - (40 * (int64_t)kPlaceMaxTiles + 4) >= 2 * 2048,
              "the largest placed view leaves an owner window of at least 2048 instances");

// Dynamic LDS of k_place_write: masks [4][T] (u64), block starts [T] and
// local starts [T + 1] (u32), tile owners [win] (u16).
size_t place_write_lds(int T, int win) {
    return (size_t)T * 4 * sizeof(uint64_t) + (size_t)(2 * T + 1) * sizeof(uint32_t) + (size_t)win * sizeof(uint16_t);
}

// Kept to 76 SGPRs: above about 80 a CU holds one 1024-thread block instead of two.
__global__ __launch_bounds__(PL_THREADS) __attribute__((amdgpu_num_sgpr(76))) void k_place_write(
    const ushort4* __restrict__ rect, const uint32_t* __restrict__ order, int64_t stride, int64_t n, int nb,
    int ntx, int T, int win, const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ tile_tot,
    const uint64_t* __restrict__ partials, const uint64_t* __restrict__ d_total, uint32_t* __restrict__ ids,
    uint32_t* __restrict__ gsort, uint32_t* __restrict__ inst_off, uint2* __restrict__ ranges, uint64_t capacity) {
    extern __shared__ uint64_t s_dyn[];
    uint64_t* s_mask = s_dyn;                                         // [4][T] Gaussians covering each tile
    uint32_t* s_base = reinterpret_cast<uint32_t*>(s_dyn + 4 * T);    // [T] list position of the block's first
    uint32_t* s_ls = s_base + T;                                      // [T + 1] start among the block's instances
    uint16_t* s_town = reinterpret_cast<uint16_t*>(s_ls + T + 1);    // [win] tile of each instance of a window
    __shared__ uint32_t s_tmp[PL_WAVES];
    __shared__ uint32_t s_off[PL_GAUSS + 1];
    __shared__ uint32_t s_gid[PL_GAUSS];
    __shared__ ushort4 s_rect[PL_GAUSS];
    const int b = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
    // this thread's tiles [ta, tb): their totals and the block's counts, loaded before anything waits
    constexpr int kPer = (kPlaceMaxTiles + PL_THREADS - 1) / PL_THREADS;
    const int per = (T + PL_THREADS - 1) / PL_THREADS;
    const int ta = min(T, tid * per), tb = min(T, ta + per);
    const uint32_t* tt = tile_tot + (int64_t)v * T;
    const uint32_t* crow = cnt + ((int64_t)v * nb + b) * T;
    uint32_t rt[kPer], rc[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        rt[i] = ta + i < tb ? tt[ta + i] : 0u;
        rc[i] = ta + i < tb ? crow[ta + i] : 0u;
    }
    const uint64_t base = partials[(int64_t)v * nb + b];   // expansion index of the block's first instance
    const uint64_t vbase = partials[(int64_t)v * nb];      // ... and of the view's
    const bool over = *d_total > capacity;
    const uint32_t tot = place_load(rect, order, stride, n, v, b, s_rect, s_gid, s_off, s_tmp);
    if (tid < PL_GAUSS && (int64_t)b * PL_GAUSS + tid < n)
        inst_off[(int64_t)v * stride + s_gid[tid]] = (uint32_t)min(base + s_off[tid], capacity);
    {   // tile starts: the view's first index + exclusive scan of its tile totals
        uint32_t loc = 0, all;
#pragma unroll
        for (int i = 0; i < kPer; ++i) loc += rt[i];
        uint64_t start = vbase + block_excl_scan_1024(loc, s_tmp, all);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int t = ta + i;
            if (t < tb) {
                s_base[t] = (uint32_t)(start + rc[i]);
                if (b == 0)
                    ranges[(int64_t)v * T + t] = (over || rt[i] == 0)
                                                     ? make_uint2(0u, 0u)
                                                     : make_uint2((uint32_t)start, (uint32_t)(start + rt[i]));
            }
            start += rt[i];
        }
    }
    if (over) return;   // nothing placed; the overflow is reported
    for (int i = tid; i < 4 * T; i += PL_THREADS) s_mask[i] = 0ull;
    __syncthreads();
    {   // masks: PL_PARTS threads per Gaussian walk its rectangle
        const int g = tid % PL_GAUSS, part = tid / PL_GAUSS;
        const ushort4 r = s_rect[g];
        const uint32_t c = rect_tiles(r);
        if ((uint32_t)part < c) {
            const uint32_t w = (uint32_t)(r.y - r.x);
            unsigned long long* mq = reinterpret_cast<unsigned long long*>(s_mask + (g >> 6) * T);
            const unsigned long long bit = 1ull << (g & 63);
            uint32_t x;
            uint32_t y = r.z + divmod_small((uint32_t)part, w, x);
            x += r.x;
            for (uint32_t k = (uint32_t)part; k < c; k += PL_PARTS) {
                atomicOr(&mq[y * (uint32_t)ntx + x], bit);
                x += PL_PARTS;
                while (x >= r.y) {
                    x -= w;
                    ++y;
                }
            }
        }
    }
    __syncthreads();
    {   // the block's instances per tile and where each tile's run starts
        uint32_t loc = 0, all;
        for (int t = ta; t < tb; ++t)
            loc += (uint32_t)(__popcll(s_mask[t]) + __popcll(s_mask[T + t]) + __popcll(s_mask[2 * T + t]) +
                              __popcll(s_mask[3 * T + t]));
        uint32_t st = block_excl_scan_1024(loc, s_tmp, all);
        for (int t = ta; t < tb; ++t) {
            s_ls[t] = st;
            st += (uint32_t)(__popcll(s_mask[t]) + __popcll(s_mask[T + t]) + __popcll(s_mask[2 * T + t]) +
                             __popcll(s_mask[3 * T + t]));
        }
        if (tid == 0) s_ls[T] = all;
    }
    // Tile-major walk over the block's instances in windows of `win`:
    // consecutive threads write consecutive list positions of a tile.
    for (uint32_t w0 = 0; w0 < tot; w0 += (uint32_t)win) {
        const uint32_t w1 = min(tot, w0 + (uint32_t)win);
        __syncthreads();
        for (int t = ta; t < tb; ++t) {
            const uint32_t a = max(s_ls[t], w0), e = min(s_ls[t + 1], w1);
            for (uint32_t q = a; q < e; ++q) s_town[q - w0] = (uint16_t)t;
        }
        __syncthreads();
        for (uint32_t q = w0 + tid; q < w1; q += PL_THREADS) {
            const int t = s_town[q - w0];
            const uint32_t rank = q - s_ls[t];
            const uint32_t g = mask_select(s_mask, T, t, rank);
            const ushort4 r = s_rect[g];
            uint32_t tx;
            const uint32_t ty = divmod_small((uint32_t)t, (uint32_t)ntx, tx);
            const uint64_t e = base + s_off[g] + (ty - r.z) * (uint32_t)(r.y - r.x) + (tx - r.x);
            const uint64_t p = (uint64_t)s_base[t] + rank;
            if (p < capacity && e < capacity) {
                ids[p] = (uint32_t)e;
                gsort[p] = s_gid[g];
            }
        }
    }
}

// keys[i] = tile of list position i, from the tile ranges (state export of
// the placed lists, which carry no keys).
__global__ void k_keys_from_ranges(const uint2* __restrict__ ranges, int64_t ntiles, uint32_t* __restrict__ keys) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint2 r = ranges[t];
        for (uint32_t i = r.x + threadIdx.x; i < r.y; i += blockDim.x) keys[i] = (uint32_t)t;
    }
}

// ---------------------------------------------------------------------------
// Depth sort of short segments (at most kSmallSortChunks chunks of SM_CHUNK
// keys per view): one kernel per 8-bit pass and nothing else.  A workgroup
// of 512 threads sorts one chunk of 2048 keys per pass.  Where its keys go
// needs, per digit, how many keys all chunks hold and how many the earlier
// chunks hold:
//   * the first pass reads per-chunk digit counts cnt[seg][chunk][digit],
//     which the preprocess adds up from its blocks of 256 keys (the second
//     pass clears them again for the next sort; the allocation starts them
//     at zero);
//   * every pass leaves the next one a table of prefixes: workgroup s, having
//     placed its keys, writes for e = 0 .. nchunks
//         pre[seg][s][e][d] = its keys whose new position lies in a chunk
//                             before e and whose next digit is d
//     (16-bit counts, two per word), so the next pass sums, over the source
//     chunks s, entry e = c for the keys below its chunk c and e = nchunks
//     for the totals -- plain stores and loads, no atomics and no clears.
// ---------------------------------------------------------------------------
constexpr int SM_THREADS = 512;
constexpr int SM_WAVES = SM_THREADS / 64;
constexpr int SM_ITEMS = 4;
constexpr int SM_LOG_CHUNK = 11;
constexpr int SM_CHUNK = 1 << SM_LOG_CHUNK;       // SM_THREADS * SM_ITEMS keys
constexpr int SM_MAXCH = kSmallSortChunks;        // chunks per segment
constexpr int SM_WSPAN = 64 * SM_ITEMS;           // keys of one wave in a chunk
static_assert(SM_CHUNK == SM_THREADS * SM_ITEMS, "chunk = threads x items");
static_assert(SM_CHUNK == kSmallSortChunkKeys, "chunk size shared with the preprocess");
static_assert(2 * SM_WAVES * RS_BINS <= 2 * SM_CHUNK, "table sums fit the staging area");

// Exclusive scan of one value per thread over a workgroup of NW waves.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_tmp[wid] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t t = s_tmp[w];
        base += (w < wid) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + incl - x;
}

__global__ __launch_bounds__(SM_THREADS) void k_sort_small(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t seg_stride, uint32_t count, int shift, const uint32_t* __restrict__ cnt,
    const uint32_t* __restrict__ tin, uint32_t* __restrict__ tout, uint32_t* __restrict__ tzero,
    int64_t zero_words) {
    __shared__ __align__(16) uint32_t s_stage[2 * SM_CHUNK];           // keys | values; first the table sums
    __shared__ __align__(16) uint32_t s_cnt[SM_WAVES][RS_BINS];        // per-wave digit counters
    __shared__ __align__(16) uint32_t s_next[SM_MAXCH][RS_BINS / 2];   // placed keys per (new chunk, next digit): u16 pairs
    __shared__ uint32_t s_gb[RS_BINS];                    // new position of staged key p: s_gb[d] + p
    __shared__ uint32_t s_ls[RS_BINS];                    // chunk-local start of each digit
    __shared__ uint32_t s_tmp[SM_WAVES];
    const int seg = blockIdx.y, c = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nch = (int)((count + SM_CHUNK - 1) >> SM_LOG_CHUNK);
    const uint32_t* ki = kin + seg * seg_stride;
    const uint32_t* vi = vin + seg * seg_stride;
    uint32_t* ko = kout + seg * seg_stride;
    uint32_t* vo = vout + seg * seg_stride;
    const int64_t base = (int64_t)c * SM_CHUNK;
    const int n_valid = (int)min((int64_t)SM_CHUNK, (int64_t)count - base);

    uint32_t key[SM_ITEMS], val[SM_ITEMS], rank[SM_ITEMS];
#pragma unroll
    for (int it = 0; it < SM_ITEMS; ++it) {
        const int j = wid * SM_WSPAN + it * 64 + lane;
        const bool ok = j < n_valid;
        key[it] = ok ? ki[base + j] : 0u;
        val[it] = ok ? vi[base + j] : 0u;
    }
    if (cnt) {   // first pass: wave w sums the count rows w, w + 8, ..., each lane four digits
        uint4 pre = make_uint4(0u, 0u, 0u, 0u), tot = make_uint4(0u, 0u, 0u, 0u);
        const uint4* t4 = reinterpret_cast<const uint4*>(cnt + (int64_t)seg * SM_MAXCH * RS_BINS);
        uint4 h[SM_MAXCH / SM_WAVES];
#pragma unroll
        for (int k = 0; k < SM_MAXCH / SM_WAVES; ++k)   // all loads issued at once (rows past the
            h[k] = t4[min(wid + SM_WAVES * k, nch - 1) * (RS_BINS / 4) + lane];   // last are re-reads)
#pragma unroll
        for (int k = 0; k < SM_MAXCH / SM_WAVES; ++k) {
            const int r = wid + SM_WAVES * k;
            const uint32_t in = r < nch ? ~0u : 0u, below = r < c ? ~0u : 0u;
            pre.x += h[k].x & below;
            pre.y += h[k].y & below;
            pre.z += h[k].z & below;
            pre.w += h[k].w & below;
            tot.x += h[k].x & in;
            tot.y += h[k].y & in;
            tot.z += h[k].z & in;
            tot.w += h[k].w & in;
        }
        reinterpret_cast<uint4*>(s_stage)[wid * (RS_BINS / 4) + lane] = pre;
        reinterpret_cast<uint4*>(s_stage + SM_CHUNK)[wid * (RS_BINS / 4) + lane] = tot;
    } else {     // later passes: thread (w, j) sums, over the sources s = w, w + 8, ..., the j-th
                 // 16-byte piece of rows e = c (j < 32) and e = nch (j >= 32): 8 digits each
        const int j = lane;
        const int e = j < 32 ? c : nch;
        uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        uint4 h[SM_MAXCH / SM_WAVES];
#pragma unroll
        for (int k = 0; k < SM_MAXCH / SM_WAVES; ++k) {
            const int src = min(wid + SM_WAVES * k, nch - 1);
            const int64_t row = ((int64_t)seg * SM_MAXCH + src) * (SM_MAXCH + 1) + e;
            h[k] = reinterpret_cast<const uint4*>(tin)[row * (RS_BINS / 8) + (j & 31)];
        }
#pragma unroll
        for (int k = 0; k < SM_MAXCH / SM_WAVES; ++k) {
            const uint32_t in = wid + SM_WAVES * k < nch ? ~0u : 0u;
            const uint32_t x[4] = {h[k].x & in, h[k].y & in, h[k].z & in, h[k].w & in};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[2 * q] += x[q] & 0xFFFFu;
                acc[2 * q + 1] += x[q] >> 16;
            }
        }
        // s_stage as [wave][j][8]: digit d of row c at j = d / 8, of the totals at j = 32 + d / 8
        uint4* o = reinterpret_cast<uint4*>(s_stage + (wid * 64 + j) * 8);
        o[0] = make_uint4(acc[0], acc[1], acc[2], acc[3]);
        o[1] = make_uint4(acc[4], acc[5], acc[6], acc[7]);
    }
    {   // this pass's share of clearing the table the previous pass read
        const int64_t nthr = (int64_t)gridDim.x * gridDim.y * SM_THREADS;
        const int64_t t0 = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * SM_THREADS + tid;
        uint4* z4 = reinterpret_cast<uint4*>(tzero);
        for (int64_t i = t0; i < zero_words / 4; i += nthr) z4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int i = tid; i < SM_WAVES * RS_BINS / 4; i += SM_THREADS)
        reinterpret_cast<uint4*>(&s_cnt[0][0])[i] = make_uint4(0u, 0u, 0u, 0u);
    if (tout)
        for (int i = tid; i < nch * (RS_BINS / 8); i += SM_THREADS)
            reinterpret_cast<uint4*>(&s_next[0][0])[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    {
        uint32_t pre = 0, tot = 0;
        if (tid < RS_BINS) {
#pragma unroll
            for (int w = 0; w < SM_WAVES; ++w) {
                pre += cnt ? s_stage[w * RS_BINS + tid] : s_stage[w * 512 + tid];
                tot += cnt ? s_stage[SM_CHUNK + w * RS_BINS + tid] : s_stage[w * 512 + 256 + tid];
            }
        }
        uint32_t all;
        const uint32_t start = block_excl_scan<SM_WAVES>(tot, s_tmp, all);   // first position of digit tid
        if (tid < RS_BINS) s_gb[tid] = start + pre;                          // ... of this chunk's keys of it
    }

    // Stable ranks inside each wave, as in k_radix_scatter.
    const uint32_t dmask = 0xFFu;
#pragma unroll
    for (int it = 0; it < SM_ITEMS; ++it) {
        const int j = wid * SM_WSPAN + it * 64 + lane;
        const bool ok = j < n_valid;
        const uint32_t d = (key[it] >> shift) & dmask;
        uint64_t match = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot(ok && ((d >> b) & 1u));
            match &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(match >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)match, 0u));
        const uint32_t before = ok ? s_cnt[wid][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) s_cnt[wid][d] = before + (uint32_t)__popcll(match);
        __builtin_amdgcn_wave_barrier();
        rank[it] = before + below;
    }
    __syncthreads();
    {   // per digit: offsets of the waves, then the chunk-local start
        uint32_t dtot = 0;
        if (tid < RS_BINS) {
#pragma unroll
            for (int w = 0; w < SM_WAVES; ++w) {
                const uint32_t x = s_cnt[w][tid];
                s_cnt[w][tid] = dtot;
                dtot += x;
            }
        }
        uint32_t all;
        const uint32_t ls = block_excl_scan<SM_WAVES>(dtot, s_tmp, all);
        if (tid < RS_BINS) {
            s_ls[tid] = ls;
            s_gb[tid] -= ls;
        }
    }
    __syncthreads();
    const int nshift = shift + 8;
#pragma unroll
    for (int it = 0; it < SM_ITEMS; ++it) {
        const int j = wid * SM_WSPAN + it * 64 + lane;
        if (j < n_valid) {
            const uint32_t d = (key[it] >> shift) & dmask;
            const uint32_t pos = s_ls[d] + s_cnt[wid][d] + rank[it];
            if (pos < (uint32_t)SM_CHUNK) {
                s_stage[pos] = key[it];
                s_stage[SM_CHUNK + pos] = val[it];
                if (tout) {   // at most SM_CHUNK per counter: the 16-bit halves never carry
                    const uint32_t g = s_gb[d] + pos, dn = (key[it] >> nshift) & dmask;
                    if (g < count) atomicAdd(&s_next[g >> SM_LOG_CHUNK][dn >> 1], 1u << (16 * (dn & 1u)));
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SM_ITEMS; ++it) {
        const int p = it * SM_THREADS + tid;
        if (p < n_valid) {
            const uint32_t k = s_stage[p];
            const uint32_t g = s_gb[(k >> shift) & dmask] + (uint32_t)p;
            if (g < count) {
                ko[g] = k;
                vo[g] = s_stage[SM_CHUNK + p];
            }
        }
    }
    if (!tout) return;
    // tout[seg][c][e] = prefix over e of the placed keys per next digit, e = 0 .. nch, as packed
    // 16-bit pairs (a half never exceeds SM_CHUNK, so the words add without carries): thread
    // (part, q) sums rows [4 part, 4 part + 4) of the 16-byte column q, then writes its prefixes
    // after adding the lower parts' sums (part 15 also writes e = 64).
    constexpr int Q = RS_BINS / 8;                         // 16-byte columns per row
    static_assert(SM_THREADS == Q * (SM_MAXCH / 4), "four rows per part");
    const uint4* nx = reinterpret_cast<const uint4*>(&s_next[0][0]);
    uint4* s_part = reinterpret_cast<uint4*>(&s_cnt[0][0]);   // [16][Q]; the digit counters are done
    const int q = tid & (Q - 1), part = tid / Q;
    uint4 sum = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int e = 4 * part; e < 4 * part + 4; ++e)
        if (e < nch) {
            const uint4 x = nx[e * Q + q];
            sum.x += x.x;
            sum.y += x.y;
            sum.z += x.z;
            sum.w += x.w;
        }
    s_part[part * Q + q] = sum;
    __syncthreads();
    uint4 run = make_uint4(0u, 0u, 0u, 0u);
    for (int k = 0; k < part; ++k) {
        const uint4 x = s_part[k * Q + q];
        run.x += x.x;
        run.y += x.y;
        run.z += x.z;
        run.w += x.w;
    }
    uint4* trow = reinterpret_cast<uint4*>(tout) + ((int64_t)seg * SM_MAXCH + c) * (SM_MAXCH + 1) * Q + q;
#pragma unroll
    for (int e = 4 * part; e < 4 * part + 4; ++e)
        if (e <= nch) {
            trow[(int64_t)e * Q] = run;
            if (e < nch) {
                const uint4 x = nx[e * Q + q];
                run.x += x.x;
                run.y += x.y;
                run.z += x.z;
                run.w += x.w;
            }
        }
    if (part == SM_MAXCH / 4 - 1 && nch == SM_MAXCH) trow[(int64_t)SM_MAXCH * Q] = run;
}

int grid_for(int64_t chunks) {
    int64_t g = chunks < 1 ? 1 : chunks;
    return (int)(g > 2048 ? 2048 : g);
}

template <int ITEMS>
int radix_passes(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg, const uint32_t* d_count,
                 uint32_t h_count, int bits, const RadixScratch& rs, hipStream_t s) {
    constexpr int64_t CHUNK = (int64_t)RS_THREADS * ITEMS;
    int cur = 0;
    const int64_t nchunks_cap = d_count ? rs.nchunks_cap : (h_count + CHUNK - 1) / CHUNK;
    const int grid_x = grid_for(nchunks_cap);
    // as few 8-bit-or-narrower passes as the key needs, the bits spread evenly
    // over them (11 bits: 6 + 5, so that no pass has only a few, crowded digits)
    if (bits <= 0) return cur;
    const int passes = (bits + 7) / 8;
    const int per = (bits + passes - 1) / passes;
    // first_hist_given: the producer of the keys wrote the first pass's
    // histograms (chunks of 256 keys, host count)
    const bool given = rs.first_hist_given && ITEMS == 1 && !d_count && per == 8;
    for (int shift = 0; shift < bits; shift += per) {
        const int pass_bits = (bits - shift) < per ? (bits - shift) : per;
        if (!(given && shift == 0))
            k_radix_hist<ITEMS><<<dim3(grid_x, nseg), RS_THREADS, 0, s>>>(keys[cur], seg_stride, d_count, h_count,
                                                                           shift, (1u << pass_bits) - 1u, rs.hist,
                                                                           nchunks_cap);
        k_radix_scan<ITEMS><<<dim3(RS_BINS, nseg), RS_THREADS, 0, s>>>(rs.hist, rs.digit_tot, d_count, h_count,
                                                                        nchunks_cap);
        k_radix_scatter<ITEMS><<<dim3(grid_x, nseg), RS_THREADS, 0, s>>>(
            keys[cur], vals[cur], keys[1 - cur], vals[1 - cur], seg_stride, d_count, h_count, shift, pass_bits,
            rs.hist, rs.digit_tot, nchunks_cap);
        cur = 1 - cur;
    }
    return cur;
}

}  // namespace

int64_t radix_chunks(int64_t count, int items) {
    const int64_t chunk = (int64_t)RS_THREADS * items;
    return (count + chunk - 1) / chunk;
}

int radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg,
                     const uint32_t* d_count, uint32_t h_count, int bits, const RadixScratch& rs,
                     hipStream_t s) {
    // 256, 1024, 2048 or 4096 keys per workgroup iteration: more workgroups
    // for small sorts, fewer per-chunk histograms for large ones
    if (rs.items == 1) return radix_passes<1>(keys, vals, seg_stride, nseg, d_count, h_count, bits, rs, s);
    if (rs.items == 4) return radix_passes<4>(keys, vals, seg_stride, nseg, d_count, h_count, bits, rs, s);
    if (rs.items == 8) return radix_passes<8>(keys, vals, seg_stride, nseg, d_count, h_count, bits, rs, s);
    if (rs.items == 16) return radix_passes<16>(keys, vals, seg_stride, nseg, d_count, h_count, bits, rs, s);
    return radix_passes<32>(keys, vals, seg_stride, nseg, d_count, h_count, bits, rs, s);
}

int64_t small_sort_count_words(int64_t nseg) { return nseg * SM_MAXCH * RS_BINS; }
int64_t small_sort_prefix_words(int64_t nseg) { return nseg * SM_MAXCH * (SM_MAXCH + 1) * (RS_BINS / 2); }

int radix_sort_small(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg, uint32_t count,
                     uint32_t* cnt, int64_t cnt_words, uint32_t* pre[2], hipStream_t s) {
    // 32-bit keys in 4 passes of 8 bits; the second pass clears the first pass's counts
    const int nch = (int)((count + SM_CHUNK - 1) >> SM_LOG_CHUNK);
    if (nch == 0 || nch > SM_MAXCH) return 0;
    int cur = 0;
    for (int p = 0; p < 4; ++p) {
        k_sort_small<<<dim3((unsigned)nch, (unsigned)nseg), SM_THREADS, 0, s>>>(
            keys[cur], vals[cur], keys[1 - cur], vals[1 - cur], seg_stride, count, 8 * p, p == 0 ? cnt : nullptr,
            p == 0 ? nullptr : pre[(p - 1) & 1], p < 3 ? pre[p & 1] : nullptr, p == 1 ? cnt : nullptr,
            p == 1 ? cnt_words : 0);
        cur = 1 - cur;
    }
    return cur;
}

int64_t onesweep_chunks(int64_t count) { return (count + OS_CHUNK - 1) / OS_CHUNK; }

int radix_sort_onesweep(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg, uint32_t count,
                        const OnesweepScratch& os, uint32_t* flags, hipStream_t s) {
    // 32-bit keys in 4 passes of 8 bits
    constexpr int passes = 4, per = 8;
    const int64_t nchunks = onesweep_chunks(count);
    if (nchunks == 0) return 0;
    k_os_clear<<<1, 256, 0, s>>>(os.tot, os.tickets, nseg);
    k_os_totals<<<dim3((unsigned)nchunks, nseg), RS_THREADS, 0, s>>>(keys[0], seg_stride, count, passes, per, os.tot,
                                                                    os.status, os.tickets, nchunks);
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        k_os_pass<<<dim3((unsigned)nchunks, nseg), RS_THREADS, 0, s>>>(keys[cur], vals[cur], keys[1 - cur],
                                                                      vals[1 - cur], seg_stride, count, p, p * per,
                                                                      per, os.tot, os.status, os.tickets, nchunks,
                                                                      flags);
        cur = 1 - cur;
    }
    return cur;
}

int64_t expand_blocks(int64_t elements) { return (elements + EX_THREADS - 1) / EX_THREADS; }

void launch_expand(const ushort4* rect, const uint32_t* order, int64_t stride, int64_t n, int nv,
                   int ntx, int tiles_per_view, uint64_t* partials, uint64_t* d_total,
                   uint32_t* d_count, uint32_t* keys, uint32_t* vals, uint4* rank_tab,
                   uint32_t* inst_off, uint64_t capacity, uint32_t* flags, uint64_t* max_inst, const Clears& cl,
                   hipStream_t s) {
    const int64_t total_el = n * nv;
    const int64_t nb = expand_blocks(total_el);
    k_tile_count<<<(unsigned)(nb > 0 ? nb : 1), EX_THREADS, 0, s>>>(rect, order, stride, n, total_el, partials, cl);
    k_scan_partials<<<1, 1024, 0, s>>>(partials, nb, d_total, d_count, capacity, flags, max_inst);
    if (nb > 0)
        k_expand<<<(unsigned)nb, EX_THREADS, 0, s>>>(rect, order, stride, n, total_el, ntx, tiles_per_view,
                                                    partials, keys, vals, rank_tab, inst_off, capacity);
}

int64_t place_blocks(int64_t n) { return n > 0 ? (n + PL_GAUSS - 1) / PL_GAUSS : 1; }

void launch_place(const ushort4* rect, const uint32_t* order, int64_t stride, int64_t n, int nv, int ntx, int nty,
                  uint32_t* cnt, uint32_t* tile_tot, uint64_t* partials, uint64_t* d_total, uint32_t* d_count,
                  uint32_t* ids, uint32_t* gsort, uint32_t* inst_off, uint2* ranges, uint64_t capacity,
                  uint32_t* flags, uint64_t* max_inst, const Clears& cl, hipStream_t s) {
    const int nb = (int)place_blocks(n);
    const int T = ntx * nty;
    const dim3 grid((unsigned)nb, (unsigned)nv);
    // owner window: what is left of 64 KiB of LDS after the static part
    // (< kPlaceStaticLds) and the per-tile arrays, at most 16384 instances
    const int win = std::min<int>(
        16384, (int)((65536 - kPlaceStaticLds - (int64_t)place_write_lds(T, 0)) / (int64_t)sizeof(uint16_t)) & ~255);
    k_place_count<<<grid, PL_THREADS, (size_t)(nty + 1) * (ntx + 1) * sizeof(uint32_t), s>>>(
        rect, order, stride, n, nb, ntx, nty, cnt, partials, cl);
    k_place_scan<<<dim3((unsigned)((T + 63) / 64 + 1), (unsigned)nv), 1024, 0, s>>>(
        cnt, nb, T, tile_tot, partials, (int64_t)nb * nv, d_total, d_count, capacity, flags, max_inst);
    k_place_write<<<grid, PL_THREADS, place_write_lds(T, win), s>>>(rect, order, stride, n, nb, ntx, T, win, cnt,
                                                                    tile_tot, partials, d_total, ids, gsort,
                                                                    inst_off, ranges, capacity);
}

void launch_keys_from_ranges(const uint2* ranges, int64_t ntiles, uint32_t* keys, hipStream_t s) {
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>(ntiles, 4096));
    k_keys_from_ranges<<<(unsigned)g, 256, 0, s>>>(ranges, ntiles, keys);
}

void launch_ranges(const uint32_t* keys, uint32_t* ids, const uint4* rank_tab, int64_t stride, int tiles_per_view,
                   int ntx, const uint32_t* d_count, int64_t capacity, uint2* ranges, uint32_t* gsort,
                   hipStream_t s) {
    int64_t blocks = (capacity + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_ranges<<<(unsigned)blocks, 256, 0, s>>>(keys, ids, rank_tab, stride, (uint32_t)tiles_per_view, (uint32_t)ntx,
                                              d_count, ranges, gsort);
}

// inst_gid[ids[i]] = gsort[i] for the d_count list positions (state export
// of the placed lists, which are built without inst_gid).
__global__ void k_gid_by_index(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ gsort,
                               const uint32_t* d_count, uint32_t* __restrict__ inst_gid) {
    const uint32_t count = *d_count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        inst_gid[ids[i]] = gsort[i];
}

void launch_gid_by_index(const uint32_t* ids, const uint32_t* gsort, const uint32_t* d_count, int64_t capacity,
                         uint32_t* inst_gid, hipStream_t s) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((capacity + 255) / 256, 8192));
    k_gid_by_index<<<(unsigned)blocks, 256, 0, s>>>(ids, gsort, d_count, inst_gid);
}

}  // namespace gsta
