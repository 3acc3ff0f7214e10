// Internal declarations of libgsta: device-side camera record, helpers
// shared by several kernels, and the host launchers the C ABI calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsta {

constexpr int kTile = 16;                 // tile edge in pixels
constexpr int kTilePix = kTile * kTile;   // one thread per pixel of a tile
constexpr int kMaxViews = 8;              // views per render call (kernel-argument camera array)

// Rasterizer conventions (3D Gaussian splatting; the paper builds on it).
constexpr float kDilate = 0.3f;           // added to the diagonal of the 2-D covariance
constexpr float kTanClamp = 1.3f;         // tangent ratio clamp inside the EWA Jacobian
constexpr float kPowerFloor = -4.5f;      // 3-sigma ellipse
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
// The splat records hold the conic pre-scaled so that one pixel's exponent
// comes out in base 2: A = -log2(e)/2 a, B = -log2(e) b, C = -log2(e)/2 c,
// power2 = A dx^2 + B dx dy + C dy^2 = log2(e) (-(a dx^2 + c dy^2)/2 - b dx dy).
constexpr float kConicScaleAC = -0.5f * kLog2e;
constexpr float kConicScaleB = -kLog2e;
constexpr float kPower2Floor = kPowerFloor * kLog2e;   // the 3-sigma floor in base-2 units

struct DevCam {
    int width, height;
    float fx, fy, cx, cy;
    float R[9];          // world -> camera rotation, row-major
    float t[3];
    float pos[3];        // camera centre (world)
    float near_z;
    float limx, limy;    // tangent clamp limits
    int ntx, nty;        // tiles per row / column
};

struct CamArray {
    DevCam c[kMaxViews];
};

struct LrArray {
    float lr[64];
};

inline __host__ __device__ int n_rows(int degree) { return 11 + 3 * (degree + 1) * (degree + 1); }

// -------------------------------------------------------------------------
// Splat evaluation shared by the forward and backward compositing kernels.
// Both kernels must take bit-identical membership/termination decisions and
// transmittance values, so the arithmetic lives in one place, written with
// explicit fused multiply-adds and floating-point contraction disabled.
// -------------------------------------------------------------------------
struct SplatEval {
    float dx, dy, power2, G, oG, alpha;   // power2: the exponent in base 2 (power * log2 e)
};

// Split in two so that a wave can skip the exponential when none of its
// pixels lies inside the splat's 3-sigma ellipse.  A, B, C: the scaled conic
// of the record (kConicScaleAC, kConicScaleB).
__device__ __forceinline__ void eval_power(float u, float v, float A, float B, float C, float px, float py,
                                           SplatEval& e) {
#pragma clang fp contract(off)
    e.dx = u - px;
    e.dy = v - py;
    float t = (A * e.dx) * e.dx;
    t = fmaf(C * e.dy, e.dy, t);
    e.power2 = fmaf(B * e.dx, e.dy, t);
}

__device__ __forceinline__ void eval_alpha(float o, SplatEval& e) {
#pragma clang fp contract(off)
    e.G = __builtin_amdgcn_exp2f(e.power2);
    e.oG = o * e.G;
    e.alpha = fminf(kAlphaMax, e.oG);
}

__device__ __forceinline__ void eval_splat(float u, float v, float A, float B, float C, float o,
                                           float px, float py, SplatEval& e) {
    eval_power(u, v, A, B, C, px, py, e);
    eval_alpha(o, e);
}

__device__ __forceinline__ float next_T(float T, float alpha) {
#pragma clang fp contract(off)
    return T * (1.0f - alpha);
}

// Wave-wide (64 lanes) float sum, result valid in every lane.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// -------------------------------------------------------------------------
// Host launchers (all asynchronous on `s`).
// -------------------------------------------------------------------------

// hist0 (optional): the depth sort's first-pass digit counts, of every block
// of 256 keys as [nv][256][ceil(n/256)] for radix_sort_pairs with
// first_hist_given, or with hist_chunks added to the per-chunk counts
// [nv][kSmallSortChunks][256] of radix_sort_small (which must be zero).
// SH-band masks of the finetune stage (Section 3.3): logits [3][ld] (same
// ld as the parameters) or null, the gate threshold as a logit, and the
// backward's output dL/dlogit ([3][gld], or null).
struct ShMask {
    const float* logit = nullptr;
    float thr_logit = 0.f;
    float* grad = nullptr;
};

// The sparsity term of the SH-band masks (Section 3.3): out[0] = lambda *
// mean sigmoid(logit) over the 3 n logits, out[1..3] = open gates of bands
// 1..3 (logit > thr_logit); grad (if not null) += lambda sigmoid'(logit) /
// (3 n) for every non-frozen column.  part: [4][ceil(n / 256)] scratch.
void launch_sh_mask_reg(const float* logits, int64_t n, int64_t ld, float thr_logit, float lambda,
                        const uint8_t* frozen, float* grad, double* part, double* out, hipStream_t s);

void launch_preprocess_fwd(const float* P, int64_t ld, int64_t n, int degree, const CamArray& cams,
                           int nv, float4* geo, float4* col, float4* rgb, ushort4* rect,
                           uint32_t* dkey, uint32_t* dval, int64_t stride, uint32_t* hist0, bool hist_chunks,
                           int opact, const ShMask& sm, hipStream_t s);

// Sums each active Gaussian's per-tile 2-D gradients (partials at its
// expansion offsets inst_off[v][gid], in tile order, taking a slot only if
// its stamp is the current generation), chains them to every parameter, sums
// over views, and updates the gradient-norm EMAs.
// grad2d_out ([nv][9][n], optional) receives the per-view 2-D gradients;
// dstats ([4][n], optional) accumulates the densification statistics.
void launch_preprocess_bwd(const float* P, int64_t ld, int64_t n, int degree, const CamArray& cams,
                           int nv, const ushort4* rect, const uint32_t* inst_off, int64_t stride,
                           const float* partials, const uint32_t* stamps, uint32_t* gen,
                           const uint32_t* d_count, const uint8_t* frozen, float* d2sum, float* G,
                           int64_t gld, float* ema, float beta, float* grad2d_out, float* dstats, int opact,
                           const ShMask& sm, hipStream_t s);

// LSD radix sort of (key, value) pairs, `nseg` independent segments of
// seg_stride elements; element count per segment from d_count (device, if
// not null) or h_count.  Sorts `bits` low-order key bits.  Returns which
// buffer (0 or 1) holds the result.
// first_hist_given (items 1, host count, 8-bit digits): the producer of the
// keys has written the first pass's chunk histograms into `hist` (chunk =
// 256 keys, row pitch ceil(h_count/256)), so that pass needs no histogram
// kernel.
struct RadixScratch {
    uint32_t* hist;          // [nseg][256][nchunks_cap]
    uint32_t* digit_tot;     // [nseg][256]
    int64_t nchunks_cap;     // chunks reserved per segment (device-count sorts)
    int items;               // keys per thread per chunk: 1, 4, 8 or 16
    bool first_hist_given = false;
};
int radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg,
                     const uint32_t* d_count, uint32_t h_count, int bits, const RadixScratch& rs,
                     hipStream_t s);
int64_t radix_chunks(int64_t count, int items);
// Onesweep variant for host-known counts (the per-view depth sort): a
// global-histogram kernel and one decoupled-look-back kernel per 8-bit pass.
struct OnesweepScratch {
    uint32_t* tot;           // [nseg][4][256] digit totals of each pass
    uint32_t* status;        // [nseg][4][chunks][256] look-back words
    uint32_t* tickets;       // [nseg][4] chunk tickets
};
int64_t onesweep_chunks(int64_t count);
int radix_sort_onesweep(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg, uint32_t count,
                        const OnesweepScratch& os, uint32_t* flags, hipStream_t s);

// Depth sort of views of at most kSmallSortKeys keys: one kernel per 8-bit
// pass (kSmallSortChunkKeys keys per workgroup).  cnt: the first pass's
// per-chunk digit counts, [nseg][kSmallSortChunks][256], which the
// preprocess adds to a zeroed table; the sort clears its cnt_words words
// again.  pre: two prefix tables of small_sort_prefix_words(nseg) words that
// carry each pass's counts to the next.  Returns the buffer holding the
// result (0); does nothing for count 0 or above the limit.
constexpr int kSmallSortChunks = 64;
constexpr int kSmallSortChunkKeys = 2048;
constexpr int64_t kSmallSortKeys = (int64_t)kSmallSortChunks * kSmallSortChunkKeys;
int64_t small_sort_count_words(int64_t nseg);
int64_t small_sort_prefix_words(int64_t nseg);
int radix_sort_small(uint32_t* keys[2], uint32_t* vals[2], int64_t seg_stride, int nseg, uint32_t count,
                     uint32_t* cnt, int64_t cnt_words, uint32_t* pre[2], hipStream_t s);

// Depth-ordered tile-instance expansion: counts per Gaussian in depth
// order, exclusive scan, a key per touched tile.  Writes keys[j] =
// view*T + tile and vals[j] = the Gaussian's depth rank in its view for
// every instance j of the expansion, inst_off[v][gid] = the first j of each
// Gaussian (its instances are contiguous, in row-major tile order), and
// rank_tab[v][rank] = (gid, first j, rectangle x0 | x1 << 16, y0 | y1 << 16).
// Its first kernel also zeroes the buffers named in `cl`.
struct Clears {
    static constexpr int kMax = 3;
    uint32_t* ptr[kMax] = {nullptr, nullptr, nullptr};
    int64_t count[kMax] = {0, 0, 0};
};
void launch_expand(const ushort4* rect, const uint32_t* order, int64_t stride, int64_t n, int nv,
                   int ntx, int tiles_per_view, uint64_t* partials, uint64_t* d_total,
                   uint32_t* d_count, uint32_t* keys, uint32_t* vals, uint4* rank_tab,
                   uint32_t* inst_off, uint64_t capacity, uint32_t* flags, uint64_t* max_inst, const Clears& cl,
                   hipStream_t s);
int64_t expand_blocks(int64_t elements);

// Direct tile placement, the alternative to expansion + tile-key sort +
// ranges for views of at most kPlaceMaxTiles tiles: writes ids (the
// tile-major, depth-ordered list of expansion indices, as the stable sort
// orders them), gsort (the gid at each list position), inst_off and the
// ranges of all nv*T tiles (empty ones as {0, 0}), and zeroes the buffers
// named in `cl`.  inst_gid is not written.  Scratch: cnt
// [nv][place_blocks(n)][T], tile_tot [nv][T], partials [nv*place_blocks(n)].
// On overflow (instances > capacity) nothing is placed and every range is
// empty; the overflow is reported as by launch_expand.
constexpr int kPlaceMaxTiles = 1408;
int64_t place_blocks(int64_t n);
void launch_place(const ushort4* rect, const uint32_t* order, int64_t stride, int64_t n, int nv, int ntx, int nty,
                  uint32_t* cnt, uint32_t* tile_tot, uint64_t* partials, uint64_t* d_total, uint32_t* d_count,
                  uint32_t* ids, uint32_t* gsort, uint32_t* inst_off, uint2* ranges, uint64_t capacity,
                  uint32_t* flags, uint64_t* max_inst, const Clears& cl, hipStream_t s);
// inst_gid[ids[i]] = gsort[i] for the d_count list positions (the state
// export of the gid of each expansion index, for either way of building
// the lists).
void launch_gid_by_index(const uint32_t* ids, const uint32_t* gsort, const uint32_t* d_count, int64_t capacity,
                         uint32_t* inst_gid, hipStream_t s);
// keys[i] = tile index of list position i, from the ranges of ntiles tiles.
void launch_keys_from_ranges(const uint2* ranges, int64_t ntiles, uint32_t* keys, hipStream_t s);

// Tile ranges of the sorted keys (`ranges` must hold zeros beforehand),
// gsort[i] = the gid at each list position, and ids[i] turned from the
// depth rank the sort carried into the instance's expansion index, both
// from rank_tab [views][stride] (gid, first instance, rectangle of each
// depth rank, written by launch_expand).
void launch_ranges(const uint32_t* keys, uint32_t* ids, const uint4* rank_tab, int64_t stride, int tiles_per_view,
                   int ntx, const uint32_t* d_count, int64_t capacity, uint2* ranges, uint32_t* gsort,
                   hipStream_t s);

// Splat-segment checkpoints of the forward compositing, read by the
// backward.  Every tile's depth-ordered list is cut into segments of K
// splats (K a power of two).  When a forward wave reaches a segment boundary
// with pixels still active, it takes a slot of the pool and stores, per
// pixel of each 64-pixel group (tile-linear pixel index / 64), the state
// before that splat: transmittance and the double-precision colour prefix.
// idx[(global list position / K) * 4 + group] names the slot (unique: two
// boundaries of different tiles are more than K positions apart).  The
// backward runs one work item per (tile, segment) up to the tile's last
// member, starting from the checkpoint, so a heavy tile is spread over many
// workgroups instead of one.
constexpr int kCkptGroups = kTilePix / 64;    // 64-pixel groups per tile
constexpr int kMinSegShift = 6;               // shortest segment: 64 splats
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
// Checkpoint pool slots one forward batch (at most 256 list positions) can
// need: one per 64-pixel group and segment boundary, at the shortest segment.
constexpr uint32_t kBatchSlotsMax = 4u * (256u >> 6);
struct SegCkpt {
    uint32_t shift;          // log2 K; 31 disables segments (one item per tile, no checkpoints)
    uint32_t* idx;           // [(capacity >> min shift) + 2][4] slot per (boundary bucket, group)
    double* pool;            // [pool_cap][4][64]: T, colour r, g, b
    uint32_t pool_cap;
    uint32_t* ctr;           // [1] slots taken by the forward beyond the first batches
    uint32_t first_slots;    // pool slots [0, first_slots): the first batch of tile v*T + t owns
                             // [(v*T + t) * kBatchSlotsMax, + kBatchSlotsMax)
    uint32_t* tile_last;     // [V * T] largest `last` of each tile (zeroed before the forward)
    uint32_t* item_off;      // [V * T + 1] exclusive scan of the items per tile
    uint32_t* item_tile;     // [item_cap] tile (view * T + tile) of each work item
    uint32_t item_cap;       // entries of item_tile
    uint32_t* stamps;        // [capacity] generation of each backward partial slot
    const uint32_t* gen;     // [1] current backward generation
    uint32_t* flags;         // flags[3]: the pool ran out
};
// Compositing with `waves` (1, 2 or 4) waves per 16x16 tile.  gsort holds
// the Gaussian at each position of the tile lists, `ids` (backward only) its
// index in the depth-ordered expansion.  The backward writes each (tile, splat)
// 2-D gradient into partials[expansion index][9] without atomics; it is a
// persistent kernel of `blocks` workgroups over the (tile, segment) items.
// It writes each non-zero per-tile total together with the call's
// generation stamp (stamps[slot] = *gen); the preprocess backward takes a
// slot only when its stamp is the current generation, so no slot is ever
// cleared.  The preprocess backward's last kernel advances the device-side
// generation once every reader of it has finished (stream-ordered, so a
// captured graph replays it too).
// The L1 loss of the rendered image fused into the forward compositing
// (target null: none).  Per pixel and channel, d = image - target gives
// dL[i] = sign(d) * inv (0 at d = 0), and each workgroup adds |d| and
// (clamp(image, 0, 1) - target)^2 (double) into part[workgroup]; the
// work-item scan after the forward adds the parts in a fixed order into
// sums[0], sums[1] (as gsta_l1_loss).  part: one double2 per forward workgroup.
struct FusedL1 {
    const float* target = nullptr;
    float* dL = nullptr;
    double2* part = nullptr;
    double* sums = nullptr;
    float inv = 0.f;          // 1 / (elements of the image)
};
void launch_composite_fwd(int waves, const uint2* ranges, const uint32_t* gsort, const float4* geo, const float4* col, const float4* rgb, int64_t stride,
                          const CamArray& cams, int nv, float bg0, float bg1, float bg2, float* image,
                          float* T_final, uint32_t* last, double* cfg, const SegCkpt& sc, unsigned long long* pairs,
                          const FusedL1& l1, hipStream_t s);
void launch_composite_bwd(int waves, int blocks, const uint2* ranges, const uint32_t* ids, const uint32_t* gsort,
                          const float4* geo, const float4* col, const float4* rgb, int64_t stride,
                          const uint8_t* frozen, const CamArray& cams, int nv, float bg0, float bg1, float bg2,
                          const float* T_final, const uint32_t* last, const double* cfg, const float* dL_dimage,
                          float* partials, const uint32_t* d_count, const SegCkpt& sc, unsigned long long* pairs,
                          hipStream_t s);
// Workgroups of the backward compositing that fit on one compute unit.
int composite_bwd_blocks_per_cu(int waves);
// The per-splat backward variant over the same work items (one 64-lane
// workgroup per item, one splat per lane, pixel state passed lane to lane);
// same outputs as launch_composite_bwd, equal to rounding.
void launch_composite_bwd_splat(int blocks, const uint2* ranges, const uint32_t* ids, const uint32_t* gsort,
                                const float4* geo, const float4* col, const float4* rgb, int64_t stride,
                                const uint8_t* frozen, const CamArray& cams, int nv, float bg0, float bg1, float bg2,
                                const float* T_final, const uint32_t* last, const double* cfg,
                                const float* dL_dimage, float* partials, const SegCkpt& sc, hipStream_t s);
int composite_bwd_splat_blocks_per_cu();
void launch_adam(float* p, int64_t pld, const float* g, int64_t gld, float* m, int64_t mld, float* v,
                 int64_t vld, int64_t n, int rows, const LrArray& lr, float b1, float b2, float eps,
                 float bc1, float bc2, const uint8_t* frozen, uint32_t* flags, hipStream_t s);

// Device mirror of gsta_adam_sched (same layout).
struct AdamSched {
    int32_t step;
    int32_t decay_iters;
    float beta1, beta2, eps;
    float pos_lr_init, pos_lr_final, pos_scale;
    float lr[64];
};
void launch_adam_sched(float* p, int64_t pld, const float* g, int64_t gld, float* m, int64_t mld, float* v,
                       int64_t vld, int64_t n, int rows, AdamSched* sched, const uint8_t* frozen, uint32_t* flags,
                       hipStream_t s);

// The 11 taps of the SSIM window (Gaussian, sigma 1.5, normalised).
struct SsimTaps {
    double w[11];
};
int64_t ssim_blocks(int nv, int H, int W);
void launch_dssim(const float* img, const float* tgt, int nv, int H, int W, float lambda, float* dL, double* ssim_sum,
                  float* gmap, double* part, hipStream_t s);

// Philox4x64-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2,
// 3", SC 2011): counter c (4 words) -> 4 random words, key (k0, k1).  Ten
// rounds, each multiplying words 0 and 2 by two constants into 128-bit
// products and mixing their high halves with words 1 and 3 and the key; the
// key advances by two Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// State of the exact radix select of the "mingrad" freezing rule.
struct SelState {
    uint32_t hist[256];          // digit histogram of the current pass
    unsigned long long count;    // Gaussians taking part (finite average)
    unsigned long long rem;      // how many of the keys with the current prefix are still to choose
    uint32_t prefix;             // digits of the threshold key found so far
    uint32_t none;               // nothing to choose (m = 0)
};
void launch_freeze_random(int64_t n, uint64_t thr, uint64_t seed, uint64_t draw, int mode, uint8_t* frozen,
                          int64_t* n_frozen, hipStream_t s);
void launch_freeze_mingrad(const float* score, int64_t n, double fraction, int mode, uint8_t* frozen,
                           int64_t* n_frozen, SelState* st, uint32_t* blk, hipStream_t s);
void launch_freeze(const float* sx, const float* sr, int64_t n, float ex, float er, int mode,
                   const uint8_t* proposal, uint8_t* frozen, int64_t* n_frozen, hipStream_t s);

// Densify-and-prune (stream compaction of every per-Gaussian array).
struct DensCfg {
    float grad_threshold, rgb_threshold;
    int use_rgb;
    float split_log_scale, prune_logit, child_log_scale_shift;
};
struct DensIO {
    const float *P, *M, *V;          // [R][ld], [R][mld], [R][vld]
    int64_t ld, mld, vld, n;
    int degree;
    const float* ema;                // [4][n] or null
    const uint8_t* frozen;           // [n] or null
    const float* stats;              // [4][n]
    const float* noise;              // [6][n], or null: drawn in the kernel from Philox (seed, draw)
    uint64_t seed;
    int64_t draw;
    float *Po, *Mo, *Vo;             // [R][old_] ...
    int64_t old_, mold, vold, cap;   // cap: output columns available
    float* ema_o;                    // [4][n_out] or null
    uint8_t* frozen_o;               // [n_out] or null
};
int64_t densify_blocks(int64_t n);
void launch_densify(const DensIO& io, const DensCfg& cfg, uint8_t* code, uint32_t* boff, uint32_t* tot,
                    int64_t* counts, uint32_t* flags, hipStream_t s);
void launch_opacity_to_abs(float* P, int64_t ld, float* M, int64_t mld, float* V, int64_t vld, int64_t n,
                           hipStream_t s);
void launch_opacity_reset(float* P, int64_t ld, float* M, int64_t mld, float* V, int64_t vld, int64_t n,
                          const uint8_t* frozen, float cap, hipStream_t s);
// Stable partition of the columns by the freeze map (active first), applied
// in place to each array through tmp; src [n] and boff [blocks] are scratch.
struct PartArray {
    void* base;
    int64_t rows, ld;
    int elem_bytes;
};
void launch_partition(int64_t n, uint8_t* frozen, const PartArray* arrays, int count, void* tmp,
                      uint32_t* src, uint32_t* boff, uint32_t* tot, int64_t* n_active, hipStream_t s);
// Learned freeze proposer: flat float32 parameters W1 [64][32], b1 [64],
// W2 [64][64], b2 [64], w3 [64], b3; bf16 copies of W1 then W2.
constexpr int kMlpW1 = 0, kMlpB1 = 2048, kMlpW2 = 2112, kMlpB2 = 6208, kMlpW3 = 6272, kMlpB3 = 6336;
constexpr int kMlpCount = 6337;
constexpr int kMlpBf16 = 2048 + 4096;
constexpr int kMlpBlocks = 256;   // fixed grid of the reductions (deterministic partial sums)
void launch_traj_push(const float* ema, int64_t n, uint16_t* ring, int slot, hipStream_t s);
void launch_mlp_stats(const uint16_t* ring, int64_t n, int head, double* part, double* sums, hipStream_t s);
void launch_mlp_features(const uint16_t* ring, int64_t n, int head, const float* mean, const float* stdv,
                         uint16_t* x, hipStream_t s);
void launch_mlp_forward(const uint16_t* wb, const float* wf, const uint16_t* x, int64_t n, float* logits,
                        uint16_t* h1, float* h2, int blocks, hipStream_t s);
void launch_mlp_backward(const uint16_t* wb, const float* wf, const uint16_t* x, const uint16_t* h1, const float* h2,
                         const float* dz, int64_t n, float* part, float* grad, hipStream_t s);
void launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, float bc1,
                     float bc2, uint16_t* wb, hipStream_t s);
void launch_mlp_bf16_copy(const float* w, uint16_t* wb, hipStream_t s);
void launch_mlp_propose(const float* z, const float* sx, const float* sr, int64_t n, float thr, float vx, float vr,
                        uint8_t* prop, hipStream_t s);
constexpr int kL1Blocks = 1024;   // partial sums of the loss (fixed-order second pass)
// Message for gsta_last_error(NULL): the last failure of a call that takes no
// context, on this thread.
void set_noctx_error(const char* fmt, ...);
void launch_l1(const float* img, const float* tgt, int64_t count, float* dL, double* sums, double2* part,
               hipStream_t s);
void launch_mlp_bce(const float* z, const uint8_t* y, int64_t n, float* dz, double* loss, double2* part,
                    hipStream_t s);

}  // namespace gsta
