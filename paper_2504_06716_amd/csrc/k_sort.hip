// Depth sort, tile binning and tile ranges.
//
// The paper blends Gaussians "in a sorted order" (Section 3.1).  Here the
// order is (float32 camera depth, gid) per view, made in two stages:
//   1. a stable LSD radix sort of the N depth keys of every view (the
//      culled ones carry the largest key and sort last);
//   2. a depth-ordered expansion of each Gaussian into one (view*T + tile,
//      gid) instance per tile of its 3-sigma rectangle, followed by a stable
//      radix sort of those 16-bit-or-less tile keys.  Stability keeps the
//      depth order inside every tile.
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
                                                       uint32_t* __restrict__ inst_gid,
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
        inst_off[(int64_t)s_view[tid] * stride + s_gid[tid]] = (uint32_t)(first < capacity ? first : capacity);
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
                vals[dst] = (uint32_t)dst;
                inst_gid[dst] = s_gid[lo];
            }
        }
        __syncthreads();
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* d_count,
                         uint2* __restrict__ ranges) {
    const uint32_t count = *d_count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[i];
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
//   k_place_write  per block: masks, ranks, ids and inst_gid; the view's
//                  first block writes the tile ranges
// ---------------------------------------------------------------------------
constexpr int kPlaceWin = 4096;   // instances per owner window of the placement

// The block's Gaussians (positions b*256 + tid of view v's depth order):
// gid, rectangle and the exclusive scan of their tile counts.
__device__ __forceinline__ void place_load(const ushort4* __restrict__ rect, const uint32_t* __restrict__ order,
                                           int64_t stride, int64_t n, int v, int b, ushort4* s_rect,
                                           uint32_t* s_gid, uint32_t* s_off, uint32_t* s_tmp, uint32_t& c,
                                           uint32_t& ex, uint32_t& tot) {
    const int tid = threadIdx.x;
    const int64_t pos = (int64_t)b * EX_THREADS + tid;
    c = 0;
    uint32_t gid = 0;
    ushort4 r = make_ushort4(0, 0, 0, 0);
    if (pos < n) {
        gid = order[(int64_t)v * stride + pos];
        r = rect[(int64_t)v * stride + gid];
        c = rect_tiles(r);
    }
    s_gid[tid] = gid;
    s_rect[tid] = r;
    ex = block_excl_scan_256(c, s_tmp, tot);
    s_off[tid] = ex;
    __syncthreads();
}

// f(lo, t, j) for every instance j of the block (block-local Gaussian lo,
// tile t of the view), in windows of kPlaceWin instances whose owners are
// marked in s_owner.  Every thread of the block must call it.
template <typename F>
__device__ __forceinline__ void place_for_each(uint32_t c, uint32_t ex, uint32_t tot, const ushort4* s_rect,
                                               const uint32_t* s_off, uint8_t* s_owner, int ntx, F&& f) {
    for (uint32_t w0 = 0; w0 < tot; w0 += kPlaceWin) {
        const uint32_t w1 = min(tot, w0 + (uint32_t)kPlaceWin);
        if (c > 0) {
            const uint32_t a = max(ex, w0), e = min(ex + c, w1);
            for (uint32_t j = a; j < e; ++j) s_owner[j - w0] = (uint8_t)threadIdx.x;
        }
        __syncthreads();
        for (uint32_t j = w0 + threadIdx.x; j < w1; j += EX_THREADS) {
            const int lo = s_owner[j - w0];
            const ushort4 r = s_rect[lo];
            const uint32_t k = j - s_off[lo];
            const uint32_t w = (uint32_t)(r.y - r.x);
            f(lo, (r.z + k / w) * (uint32_t)ntx + r.x + k % w, j);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(EX_THREADS) void k_place_count(const ushort4* __restrict__ rect,
                                                            const uint32_t* __restrict__ order, int64_t stride,
                                                            int64_t n, int nb, int ntx, int T,
                                                            uint32_t* __restrict__ cnt,
                                                            uint64_t* __restrict__ partials, Clears cl) {
    extern __shared__ uint32_t s_cnt[];     // [T]
    __shared__ uint32_t s_tmp[RS_WAVES];
    __shared__ uint32_t s_off[EX_THREADS];
    __shared__ uint32_t s_gid[EX_THREADS];
    __shared__ ushort4 s_rect[EX_THREADS];
    __shared__ uint8_t s_owner[kPlaceWin];
    static_assert(EX_THREADS <= 256, "block-local Gaussian indices are stored in bytes");
    {   // buffers the rest of the forward expects zeroed
        const int64_t nthreads = (int64_t)gridDim.x * gridDim.y * EX_THREADS;
        const int64_t t0 = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * EX_THREADS + threadIdx.x;
        for (int k = 0; k < Clears::kMax; ++k)
            for (int64_t j = t0; j < cl.count[k]; j += nthreads) cl.ptr[k][j] = 0u;
    }
    const int b = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
    for (int t = tid; t < T; t += EX_THREADS) s_cnt[t] = 0;
    uint32_t c, ex, tot;
    place_load(rect, order, stride, n, v, b, s_rect, s_gid, s_off, s_tmp, c, ex, tot);
    if (tid == 0) partials[(int64_t)v * nb + b] = tot;
    place_for_each(c, ex, tot, s_rect, s_off, s_owner, ntx,
                   [&](int, uint32_t t, uint32_t) { atomicAdd(&s_cnt[t], 1u); });
    uint32_t* row = cnt + ((int64_t)v * nb + b) * T;
    for (int t = tid; t < T; t += EX_THREADS) row[t] = s_cnt[t];
}

// Blocks x < ceil(T/64): 64 tiles of view y, 16 waves over the blocks b.
// Block x == ceil(T/64) of view 0: the block totals.
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
    uint32_t sum = 0;
    if (t < T) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) sum += col[(int64_t)b * T];
    }
    s_part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t x = s_part[k][lane];
        run += (k < w) ? x : 0u;
        tot += x;
    }
    if (t < T) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) {
            const uint32_t x = col[(int64_t)b * T];
            col[(int64_t)b * T] = run;
            run += x;
        }
        if (w == 0) tile_tot[(int64_t)v * T + t] = tot;
    }
}

__global__ __launch_bounds__(EX_THREADS) void k_place_write(
    const ushort4* __restrict__ rect, const uint32_t* __restrict__ order, int64_t stride, int64_t n, int nb,
    int ntx, int T, const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ tile_tot,
    const uint64_t* __restrict__ partials, const uint64_t* __restrict__ d_total, uint32_t* __restrict__ ids,
    uint32_t* __restrict__ inst_gid, uint32_t* __restrict__ inst_off, uint2* __restrict__ ranges,
    uint64_t capacity) {
    extern __shared__ uint64_t s_dyn[];
    uint64_t* s_mask = s_dyn;                                       // [4][T] covering Gaussians
    uint32_t* s_base = reinterpret_cast<uint32_t*>(s_dyn + 4 * T);  // [T] the block's first place per tile
    __shared__ uint32_t s_tmp[RS_WAVES];
    __shared__ uint32_t s_off[EX_THREADS];
    __shared__ uint32_t s_gid[EX_THREADS];
    __shared__ ushort4 s_rect[EX_THREADS];
    __shared__ uint8_t s_owner[kPlaceWin];
    const int b = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
    uint32_t c, ex, tot;
    place_load(rect, order, stride, n, v, b, s_rect, s_gid, s_off, s_tmp, c, ex, tot);
    const uint64_t base = partials[(int64_t)v * nb + b];   // expansion index of the block's first instance
    const uint64_t vbase = partials[(int64_t)v * nb];      // ... and of the view's
    const bool over = *d_total > capacity;
    if ((int64_t)b * EX_THREADS + tid < n)
        inst_off[(int64_t)v * stride + s_gid[tid]] = (uint32_t)min(base + ex, capacity);
    // tile starts: the view's first index + exclusive scan of its tile totals
    const int per = (T + EX_THREADS - 1) / EX_THREADS;
    const int ta = min(T, tid * per), tb = min(T, ta + per);
    const uint32_t* tt = tile_tot + (int64_t)v * T;
    uint32_t loc = 0;
    for (int t = ta; t < tb; ++t) loc += tt[t];
    uint32_t all;
    uint64_t start = vbase + block_excl_scan_256(loc, s_tmp, all);
    const uint32_t* crow = cnt + ((int64_t)v * nb + b) * T;
    for (int t = ta; t < tb; ++t) {
        const uint32_t rt = tt[t];
        s_base[t] = (uint32_t)(start + crow[t]);
        if (b == 0)
            ranges[(int64_t)v * T + t] = (over || rt == 0) ? make_uint2(0u, 0u)
                                                             : make_uint2((uint32_t)start, (uint32_t)(start + rt));
        start += rt;
    }
    if (over) return;   // nothing placed; the overflow is reported
    for (int i = tid; i < 4 * T; i += EX_THREADS) s_mask[i] = 0ull;
    __syncthreads();
    place_for_each(c, ex, tot, s_rect, s_off, s_owner, ntx, [&](int lo, uint32_t t, uint32_t) {
        atomicOr(reinterpret_cast<unsigned long long*>(&s_mask[(lo >> 6) * T + t]), 1ull << (lo & 63));
    });
    place_for_each(c, ex, tot, s_rect, s_off, s_owner, ntx, [&](int lo, uint32_t t, uint32_t j) {
        const int q = lo >> 6;
        uint32_t rank = (uint32_t)__popcll(s_mask[q * T + t] & ((1ull << (lo & 63)) - 1ull));
        for (int k = 0; k < q; ++k) rank += (uint32_t)__popcll(s_mask[k * T + t]);
        const uint64_t p = (uint64_t)s_base[t] + rank, e = base + j;
        if (p < capacity && e < capacity) {
            ids[p] = (uint32_t)e;
            inst_gid[e] = s_gid[lo];
        }
    });
}

// keys[i] = tile of list position i, from the tile ranges (state export of
// the placed lists, which carry no keys).
__global__ void k_keys_from_ranges(const uint2* __restrict__ ranges, int64_t ntiles, uint32_t* __restrict__ keys) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint2 r = ranges[t];
        for (uint32_t i = r.x + threadIdx.x; i < r.y; i += blockDim.x) keys[i] = (uint32_t)t;
    }
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
    for (int shift = 0; shift < bits; shift += per) {
        const int pass_bits = (bits - shift) < per ? (bits - shift) : per;
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
    return radix_passes<16>(keys, vals, seg_stride, nseg, d_count, h_count, bits, rs, s);
}

int64_t expand_blocks(int64_t elements) { return (elements + EX_THREADS - 1) / EX_THREADS; }

void launch_expand(const ushort4* rect, const uint32_t* order, int64_t stride, int64_t n, int nv,
                   int ntx, int tiles_per_view, uint64_t* partials, uint64_t* d_total,
                   uint32_t* d_count, uint32_t* keys, uint32_t* vals, uint32_t* inst_gid,
                   uint32_t* inst_off, uint64_t capacity, uint32_t* flags, uint64_t* max_inst, const Clears& cl,
                   hipStream_t s) {
    const int64_t total_el = n * nv;
    const int64_t nb = expand_blocks(total_el);
    k_tile_count<<<(unsigned)(nb > 0 ? nb : 1), EX_THREADS, 0, s>>>(rect, order, stride, n, total_el, partials, cl);
    k_scan_partials<<<1, 1024, 0, s>>>(partials, nb, d_total, d_count, capacity, flags, max_inst);
    if (nb > 0)
        k_expand<<<(unsigned)nb, EX_THREADS, 0, s>>>(rect, order, stride, n, total_el, ntx, tiles_per_view,
                                                    partials, keys, vals, inst_gid, inst_off, capacity);
}

int64_t place_blocks(int64_t n) { return n > 0 ? (n + EX_THREADS - 1) / EX_THREADS : 1; }

void launch_place(const ushort4* rect, const uint32_t* order, int64_t stride, int64_t n, int nv, int ntx, int T,
                  uint32_t* cnt, uint32_t* tile_tot, uint64_t* partials, uint64_t* d_total, uint32_t* d_count,
                  uint32_t* ids, uint32_t* inst_gid, uint32_t* inst_off, uint2* ranges, uint64_t capacity,
                  uint32_t* flags, uint64_t* max_inst, const Clears& cl, hipStream_t s) {
    const int nb = (int)place_blocks(n);
    const dim3 grid((unsigned)nb, (unsigned)nv);
    k_place_count<<<grid, EX_THREADS, (size_t)T * sizeof(uint32_t), s>>>(rect, order, stride, n, nb, ntx, T, cnt,
                                                                         partials, cl);
    k_place_scan<<<dim3((unsigned)((T + 63) / 64 + 1), (unsigned)nv), 1024, 0, s>>>(
        cnt, nb, T, tile_tot, partials, (int64_t)nb * nv, d_total, d_count, capacity, flags, max_inst);
    k_place_write<<<grid, EX_THREADS, (size_t)T * (4 * sizeof(uint64_t) + sizeof(uint32_t)), s>>>(
        rect, order, stride, n, nb, ntx, T, cnt, tile_tot, partials, d_total, ids, inst_gid, inst_off, ranges,
        capacity);
}

void launch_keys_from_ranges(const uint2* ranges, int64_t ntiles, uint32_t* keys, hipStream_t s) {
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>(ntiles, 4096));
    k_keys_from_ranges<<<(unsigned)g, 256, 0, s>>>(ranges, ntiles, keys);
}

void launch_ranges(const uint32_t* keys, const uint32_t* d_count, int64_t capacity, uint2* ranges,
                   hipStream_t s) {
    int64_t blocks = (capacity + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_ranges<<<(unsigned)blocks, 256, 0, s>>>(keys, d_count, ranges);
}

}  // namespace gsta
