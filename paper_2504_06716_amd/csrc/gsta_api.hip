// C ABI of libgsta: context and scratch management, argument validation and
// the order of kernel launches for each entry point (see include/gsta.h).
#include "../../include/gsta.h"
#include "gsta_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace gsta;

namespace {

constexpr int kCounters = 6;   // profiling counters, see gsta_read_profile
constexpr int64_t kPlaceBytes = (int64_t)1 << 29;   // placement count scratch limit
const uint32_t kGen0 = 1u;      // first backward generation (stamps start at 0)
const int64_t kPoolBudgetSlots = (int64_t)1 << 22;   // checkpoint slots sized for full walks: 8 GiB

struct Slot {
    float4* geo = nullptr;
    float4* col = nullptr;
    float4* rgb = nullptr;
    ushort4* rect = nullptr;
    uint32_t* dkey[2] = {nullptr, nullptr};
    uint32_t* dval[2] = {nullptr, nullptr};
    uint32_t* ikey[2] = {nullptr, nullptr};
    uint32_t* ival[2] = {nullptr, nullptr};
    uint32_t* inst_gid = nullptr;   // [cap] gid of each expansion index (written for the state export)
    uint4* rank_tab = nullptr;      // [V][S] gid, first instance, rectangle of each depth rank (sorted path)
    uint32_t* gsort = nullptr;      // [cap] gid at each tile-list position
    uint32_t* inst_off = nullptr;   // [V][S] first expansion index of each Gaussian
    uint2* ranges = nullptr;
    float* T_final = nullptr;
    uint32_t* last = nullptr;
    double* cfg = nullptr;
    uint64_t* n_total = nullptr;
    uint32_t* n_count = nullptr;
    // segment checkpoints of the forward compositing (see SegCkpt)
    uint32_t* ck_idx = nullptr;
    double* ck_pool = nullptr;
    uint32_t* ck_ctr = nullptr;
    uint32_t* tile_last = nullptr;
    uint32_t* item_off = nullptr;
    uint32_t* item_tile = nullptr;
    uint32_t shift = 31;             // segment length of the last forward (31: none)
    // what the last forward in this slot rendered
    int depth_buf = 0, inst_buf = 0;
    bool placed = false;             // lists built by direct placement (no sorted keys)
    bool valid = false;
    int64_t n = 0, ld = 0;
    int degree = 0;
    const float* block = nullptr;
    const float* sh_mask = nullptr;
    float sh_mask_threshold = 0.f;
    int nv = 0;
    gsta_camera cams[kMaxViews];
    float bg[3] = {0.f, 0.f, 0.f};
};

}  // namespace

struct gsta_ctx {
    gsta_limits lim{};
    int64_t stride = 0;       // per-view row stride of per-Gaussian scratch
    int64_t tiles_max = 0;    // tiles per view at the reserved size
    std::vector<Slot> slots;
    std::vector<void*> allocs;
    uint32_t* hist = nullptr;
    uint32_t* digit_tot = nullptr;
    int64_t chunks_depth = 0, chunks_inst = 0;
    int items_depth = 16, items_inst = 16;
    uint64_t* partials = nullptr;
    double2* fwd_lpart = nullptr;    // [V][tiles_max][4] fused-loss sums per forward workgroup
    uint32_t* place_cnt = nullptr;   // [place_views][ceil(stride/256)][tiles_max] placement counts
    uint32_t* tile_tot = nullptr;    // [place_views][tiles_max] instances per tile
    int place_views = 0;             // views the placement scratch holds (0: always sort)
    int binning = 0;                 // GSTA_OPT_BINNING
    int depth_sort = 0;              // GSTA_OPT_DEPTH_SORT
    uint32_t* os_tot = nullptr;      // onesweep depth sort: [V][4][256] digit totals
    uint32_t* os_status = nullptr;   // [V][4][chunks][256] look-back words
    uint32_t* os_tickets = nullptr;  // [V][4] chunk tickets
    uint32_t* sort_cnt = nullptr;    // depth sort of short views: first-pass counts [V][64][256]
    uint32_t* sort_pre[2] = {};      // ... and the prefix tables between passes
    float* tile_grads = nullptr;   // [cap][9] per (tile, splat) 2-D gradient of the backward
    uint32_t* stamps = nullptr;    // [cap] backward generation that wrote each slot
    uint32_t* gen = nullptr;       // [1] backward generation (starts at 1; stamps start at 0)
    float* d2sum = nullptr;        // [V][9][stride] per-view 2-D gradient of each Gaussian
    double2* loss_part = nullptr;  // [kL1Blocks] loss partial sums
    int fwd_waves = 0, bwd_waves = 2;   // forward: one workgroup per 8x8 quarter
    uint32_t seg_shift = 6;        // backward segments of 64 splats (31: off)
    uint32_t pool_cap = 0;         // checkpoint slots per state slot
    uint32_t first_slots = 0;      // of which the tiles' first batches own the first ones
    uint32_t item_cap = 0;         // backward work items per state slot
    int cus = 1, bwd_blocks = 1;   // persistent backward grid
    int bwd_variant = 0;           // 0 per pixel (lanes = pixels), 1 per splat (lanes = splats)
    int bwd_splat_blocks = 1;      // persistent grid of the per-splat variant
    uint32_t* flags = nullptr;     // [0] instance overflow, [1] non-finite gradient, [2] densify overflow
    uint8_t* dens_code = nullptr;  // [max_gaussians] densify decisions
    uint32_t* dens_boff = nullptr; // [3][blocks] densify block counts / offsets
    uint32_t* dens_tot = nullptr;  // [4] kept, clones, splits, overflow
    uint32_t* part_src = nullptr;  // [max_gaussians] freeze partition gather list
    uint32_t* part_tot = nullptr;  // [1] active count of the partition
    float* ssim_g = nullptr;       // [3][max_views * 3 * H * W] D-SSIM partial-derivative maps
    double* ssim_part = nullptr;   // [ssim_blocks] per-workgroup SSIM sums
    double* shm_part = nullptr;    // [4][ceil(max_gaussians / 256)] SH-mask term partials
    SelState* sel = nullptr;       // [1] radix-select state of the mingrad freezing rule
    uint32_t* sel_blk = nullptr;   // [ceil(max_gaussians / 256)] equal-key counts per block
    float* mlp_part = nullptr;     // [kMlpBlocks][kMlpCount] proposer gradient partials
    double* mlp_stats = nullptr;   // [kMlpBlocks][64] feature-statistics partials
    uint64_t* max_inst = nullptr;
    std::string err;
    // profiling
    uint32_t profiling = 0;                   // phase mask
    bool capturing = false;                   // between gsta_graph_begin and gsta_graph_end
    // profiling counters: [0] fwd pairs, [1] bwd pairs, [2] fwd wave iterations,
    // [3] bwd wave iterations, [4] bwd wave reductions
    unsigned long long* pairs = nullptr;
    struct Pending {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double ms[GSTA_N_PHASES] = {};
    int64_t launches[GSTA_N_PHASES] = {};
};

namespace {

thread_local std::string g_noctx_err;   // last failure of a context-free call on this thread

gsta_status fail(gsta_ctx* ctx, gsta_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

gsta_status hip_check(gsta_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return GSTA_OK;
    return fail(ctx, GSTA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void free_all(gsta_ctx* ctx) {
    for (void* p : ctx->allocs) (void)hipFree(p);
    ctx->allocs.clear();
    ctx->slots.clear();
}

template <typename T>
bool alloc(gsta_ctx* ctx, T** p, int64_t count) {
    void* q = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) return false;
    ctx->allocs.push_back(q);
    *p = reinterpret_cast<T*>(q);
    return true;
}

int64_t tiles_of(int w, int h) { return (int64_t)((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile); }

gsta_status check_limits(gsta_ctx* ctx, const gsta_limits* l) {
    if (!l) return fail(ctx, GSTA_ERR_INVALID, "limits is NULL");
    if (l->max_gaussians < 1 || l->max_gaussians > (int64_t)0x7FFFFFFF)
        return fail(ctx, GSTA_ERR_INVALID, "max_gaussians out of range: %lld", (long long)l->max_gaussians);
    if (l->max_views < 1 || l->max_views > kMaxViews)
        return fail(ctx, GSTA_ERR_INVALID, "max_views must be in [1, %d]", kMaxViews);
    if (l->max_width < 1 || l->max_height < 1 || l->max_width > 16384 || l->max_height > 16384)
        return fail(ctx, GSTA_ERR_INVALID, "max image size out of range");
    if (l->tile_w != kTile || l->tile_h != kTile) return fail(ctx, GSTA_ERR_INVALID, "tiles must be 16x16");
    if (l->instance_capacity < 1 || l->instance_capacity > (int64_t)0xFFFFFFFFll)
        return fail(ctx, GSTA_ERR_INVALID, "instance_capacity must be in [1, 2^32-1]");
    if (l->n_slots < 1 || l->n_slots > 64) return fail(ctx, GSTA_ERR_INVALID, "n_slots must be in [1, 64]");
    if (tiles_of(l->max_width, l->max_height) * l->max_views > 65536)
        return fail(ctx, GSTA_ERR_INVALID, "views x tiles must fit 16-bit tile keys (<= 65536)");
    return GSTA_OK;
}

gsta_status allocate(gsta_ctx* ctx, const gsta_limits* l) {
    ctx->lim = *l;
    const int64_t V = l->max_views;
    ctx->stride = (l->max_gaussians + 63) / 64 * 64;
    ctx->tiles_max = tiles_of(l->max_width, l->max_height);
    const int64_t S = ctx->stride, cap = l->instance_capacity;
    const int64_t HW = (int64_t)l->max_width * l->max_height;
    ctx->slots.assign((size_t)l->n_slots, Slot());
    // checkpoint slots: the forward reserves, per tile and walked batch of up
    // to 256 list positions, one slot per 64-pixel group and boundary (up to
    // 4 boundaries at the shortest segment, 64), and one batch ahead.  The
    // tiles' first batches own their slots; the counter hands out the rest:
    // at most one per group and 64 walked positions -- (cap >> 6) per group
    // when every list is walked to its end (transmittance never reaching its
    // floor) -- plus each tile's one batch reserved ahead.  The pool holds
    // that many (2 KiB per slot: 128 bytes per instance of capacity) where
    // they fit kPoolBudgetSlots, so no walk can run out; past it, the larger
    // of the budget and one slot per 256 instances, and running out is
    // reported.
    static_assert(kBatchSlotsMax == (uint32_t)kCkptGroups * (256u >> kMinSegShift), "batch slot bound");
    const int64_t per_batch = kBatchSlotsMax;
    ctx->first_slots = (uint32_t)(V * ctx->tiles_max * per_batch);
    const int64_t ahead = 2 * V * ctx->tiles_max * per_batch;
    const int64_t full = kCkptGroups * ((cap >> kMinSegShift) + 1) + ahead;
    const int64_t pool_cap = std::min<int64_t>(
        std::max<int64_t>(4096, std::min<int64_t>(full, std::max<int64_t>(cap / 256 + ahead, kPoolBudgetSlots))),
        (int64_t)1 << 30);
    ctx->pool_cap = (uint32_t)pool_cap;
    // work items of the backward: ceil(tile_last / K) per tile, K >= 2^kMinSegShift,
    // and the tiles' walks add up to at most the instance capacity
    const int64_t item_cap = (cap >> kMinSegShift) + V * ctx->tiles_max + 1;
    ctx->item_cap = (uint32_t)std::min<int64_t>(item_cap, 0xFFFFFFFFll);
    bool ok = true;
    for (Slot& s : ctx->slots) {
        ok = ok && alloc(ctx, &s.geo, V * S) && alloc(ctx, &s.col, V * S) && alloc(ctx, &s.rgb, V * S) &&
             alloc(ctx, &s.rect, V * S) && alloc(ctx, &s.dkey[0], V * S) && alloc(ctx, &s.dkey[1], V * S) &&
             alloc(ctx, &s.dval[0], V * S) && alloc(ctx, &s.dval[1], V * S) && alloc(ctx, &s.ikey[0], cap) &&
             alloc(ctx, &s.ikey[1], cap) && alloc(ctx, &s.ival[0], cap) && alloc(ctx, &s.ival[1], cap) &&
             alloc(ctx, &s.inst_gid, cap) && alloc(ctx, &s.gsort, cap) && alloc(ctx, &s.inst_off, V * S) &&
             alloc(ctx, &s.rank_tab, V * S) &&
             alloc(ctx, &s.ranges, V * ctx->tiles_max) && alloc(ctx, &s.T_final, V * HW) &&
             alloc(ctx, &s.last, V * HW) && alloc(ctx, &s.cfg, 3 * V * HW) && alloc(ctx, &s.n_total, 1) &&
             alloc(ctx, &s.n_count, 1) && alloc(ctx, &s.ck_idx, ((cap >> kMinSegShift) + 2) * kCkptGroups) &&
             alloc(ctx, &s.ck_pool, (int64_t)pool_cap * 256) && alloc(ctx, &s.ck_ctr, 1) &&
             alloc(ctx, &s.tile_last, V * ctx->tiles_max) && alloc(ctx, &s.item_off, V * ctx->tiles_max + 1) &&
             alloc(ctx, &s.item_tile, item_cap);
    }
    ctx->items_depth = S <= (1 << 20) ? 1 : 16;
    // tile-key sort: 1024, 2048 or 4096 keys per chunk; the larger chunks of
    // large sorts give each digit longer runs of consecutive writes
    ctx->items_inst = cap <= (1 << 20) ? 4 : (cap <= (1 << 24) ? 8 : 32);
    ctx->chunks_depth = radix_chunks(S, ctx->items_depth);
    ctx->chunks_inst = radix_chunks(cap, ctx->items_inst);
    const int64_t hist_words = std::max(V * 256 * ctx->chunks_depth, 256 * ctx->chunks_inst);
    // direct placement: counts of every (256-Gaussian block, tile) for as many
    // views as fit kPlaceBytes (none where the tiles exceed kPlaceMaxTiles)
    const int64_t place_view_words = place_blocks(S) * ctx->tiles_max;
    ctx->place_views = ctx->tiles_max > kPlaceMaxTiles ? 0
                       : (int)std::min<int64_t>(V, kPlaceBytes / (4 * place_view_words));
    const int64_t pv = std::max(ctx->place_views, 1);
    ok = ok && alloc(ctx, &ctx->hist, hist_words) && alloc(ctx, &ctx->digit_tot, V * 256) &&
         alloc(ctx, &ctx->partials, std::max(expand_blocks(V * S), V * place_blocks(S)) + 1) &&
         alloc(ctx, &ctx->place_cnt, ctx->place_views > 0 ? pv * place_view_words : 1) &&
         alloc(ctx, &ctx->tile_tot, pv * ctx->tiles_max) && alloc(ctx, &ctx->fwd_lpart, V * ctx->tiles_max * 4) && alloc(ctx, &ctx->tile_grads, 9 * cap + 4) &&
         alloc(ctx, &ctx->stamps, cap) && alloc(ctx, &ctx->gen, 1) && alloc(ctx, &ctx->d2sum, 9 * V * S) &&
         alloc(ctx, &ctx->loss_part, kL1Blocks) && alloc(ctx, &ctx->dens_code, l->max_gaussians) &&
         alloc(ctx, &ctx->dens_boff, 3 * densify_blocks(l->max_gaussians)) && alloc(ctx, &ctx->dens_tot, 4) &&
         alloc(ctx, &ctx->part_src, l->max_gaussians) && alloc(ctx, &ctx->part_tot, 1) &&
         alloc(ctx, &ctx->sel, 1) && alloc(ctx, &ctx->sel_blk, (l->max_gaussians + 255) / 256) &&
         alloc(ctx, &ctx->ssim_g, 3 * V * 3 * HW) &&
         alloc(ctx, &ctx->ssim_part, ssim_blocks((int)V, l->max_height, l->max_width)) &&
         alloc(ctx, &ctx->shm_part, 4 * ((l->max_gaussians + 255) / 256) + 4) &&
         alloc(ctx, &ctx->mlp_part, (int64_t)kMlpBlocks * kMlpCount) &&
         alloc(ctx, &ctx->mlp_stats, (int64_t)kMlpBlocks * 64) &&
         alloc(ctx, &ctx->os_tot, V * 4 * 256) && alloc(ctx, &ctx->os_tickets, V * 4) &&
         alloc(ctx, &ctx->os_status, V * 4 * onesweep_chunks(S) * 256) &&
         alloc(ctx, &ctx->sort_cnt, small_sort_count_words(V)) &&
         alloc(ctx, &ctx->sort_pre[0], small_sort_prefix_words(V)) &&
         alloc(ctx, &ctx->sort_pre[1], small_sort_prefix_words(V)) &&
         alloc(ctx, &ctx->flags, 8) && alloc(ctx, &ctx->max_inst, 1) && alloc(ctx, &ctx->pairs, kCounters);
    if (!ok) {
        free_all(ctx);
        return fail(ctx, GSTA_ERR_OOM, "device allocation failed");
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ctx->cus = 1;
    ctx->bwd_blocks = ctx->cus * composite_bwd_blocks_per_cu(ctx->bwd_waves);
    ctx->bwd_splat_blocks = ctx->cus * composite_bwd_splat_blocks_per_cu();
    if (hipMemset(ctx->flags, 0, 8 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(ctx->stamps, 0, (size_t)std::max<int64_t>(cap, 1) * sizeof(uint32_t)) != hipSuccess ||
        hipMemcpy(ctx->gen, &kGen0, sizeof(kGen0), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(ctx->max_inst, 0, sizeof(uint64_t)) != hipSuccess ||
        hipMemset(ctx->sort_cnt, 0, small_sort_count_words(V) * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(ctx->pairs, 0, kCounters * sizeof(unsigned long long)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_all(ctx);
        return fail(ctx, GSTA_ERR_HIP, "initialising flags failed");
    }
    return GSTA_OK;
}

bool cam_ok(const gsta_camera& c) {
    return c.width > 0 && c.height > 0 && std::isfinite(c.fx) && std::isfinite(c.fy) && c.fx > 0.f &&
           c.fy > 0.f && std::isfinite(c.cx) && std::isfinite(c.cy) && std::isfinite(c.near_z) &&
           c.near_z > 0.f;
}

DevCam to_dev(const gsta_camera& c) {
    DevCam d;
    d.width = c.width;
    d.height = c.height;
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) d.R[3 * r + k] = c.world_to_cam[4 * r + k];
        d.t[r] = c.world_to_cam[4 * r + 3];
        d.pos[r] = c.cam_pos[r];
    }
    d.near_z = c.near_z;
    d.limx = kTanClamp * (0.5f * (float)c.width) / c.fx;
    d.limy = kTanClamp * (0.5f * (float)c.height) / c.fy;
    d.ntx = (c.width + kTile - 1) / kTile;
    d.nty = (c.height + kTile - 1) / kTile;
    return d;
}

SegCkpt seg_ckpt(gsta_ctx* ctx, Slot& s) {
    SegCkpt c;
    c.shift = s.shift;
    c.idx = s.ck_idx;
    c.pool = s.ck_pool;
    c.pool_cap = ctx->pool_cap;
    c.ctr = s.ck_ctr;
    c.first_slots = ctx->first_slots;
    c.tile_last = s.tile_last;
    c.item_off = s.item_off;
    c.item_tile = s.item_tile;
    c.item_cap = ctx->item_cap;
    c.stamps = ctx->stamps;
    c.gen = ctx->gen;
    c.flags = ctx->flags;
    return c;
}

gsta_status check_params(gsta_ctx* ctx, const gsta_params* g, const char* name) {
    if (!g) return fail(ctx, GSTA_ERR_INVALID, "%s is NULL", name);
    if (!g->block && g->n > 0) return fail(ctx, GSTA_ERR_INVALID, "%s.block is NULL", name);
    if (g->n < 0 || g->n > ctx->lim.max_gaussians)
        return fail(ctx, GSTA_ERR_INVALID, "%s.n = %lld outside [0, max_gaussians = %lld]", name,
                    (long long)g->n, (long long)ctx->lim.max_gaussians);
    if (g->ld < g->n || g->ld < 1) return fail(ctx, GSTA_ERR_INVALID, "%s.ld < n", name);
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(ctx, GSTA_ERR_INVALID, "%s.sh_degree not in 0..3", name);
    if (g->opacity_act != 0 && g->opacity_act != 1)
        return fail(ctx, GSTA_ERR_INVALID, "%s.opacity_act must be 0 (sigmoid) or 1 (absolute)", name);
    return GSTA_OK;
}

// The SH-band masks of the parameters of a render call.
gsta_status check_sh_mask(gsta_ctx* ctx, const gsta_params* g) {
    if (g->sh_mask && !(g->sh_mask_threshold > 0.f && g->sh_mask_threshold < 1.f))
        return fail(ctx, GSTA_ERR_INVALID, "g.sh_mask_threshold must be in (0, 1)");
    return GSTA_OK;
}

// The band gates of g: sigmoid(logit) > t taken as logit > ln(t / (1 - t)),
// the threshold's logit rounded once to float32.
ShMask sh_mask_of(const gsta_params* g, float* grad_out) {
    ShMask m;
    if (g->sh_mask) {
        const double t = (double)g->sh_mask_threshold;
        m.logit = g->sh_mask;
        m.thr_logit = (float)std::log(t / (1.0 - t));
        m.grad = grad_out;
    }
    return m;
}

gsta_status check_views(gsta_ctx* ctx, const gsta_camera* cams, int32_t nv, CamArray& ca) {
    if (!cams) return fail(ctx, GSTA_ERR_INVALID, "cams is NULL");
    if (nv < 1 || nv > ctx->lim.max_views)
        return fail(ctx, GSTA_ERR_INVALID, "n_views = %d outside [1, %d]", nv, ctx->lim.max_views);
    for (int v = 0; v < nv; ++v) {
        if (!cam_ok(cams[v])) return fail(ctx, GSTA_ERR_INVALID, "camera %d is invalid", v);
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
            return fail(ctx, GSTA_ERR_INVALID, "all views of a call must share width and height");
        if (cams[v].width > ctx->lim.max_width || cams[v].height > ctx->lim.max_height)
            return fail(ctx, GSTA_ERR_INVALID, "image %dx%d exceeds the reserved %dx%d", cams[v].width,
                        cams[v].height, ctx->lim.max_width, ctx->lim.max_height);
        ca.c[v] = to_dev(cams[v]);
    }
    for (int v = nv; v < kMaxViews; ++v) ca.c[v] = ca.c[0];
    return GSTA_OK;
}

int key_bits(int64_t keys) {
    int b = 1;
    while (((int64_t)1 << b) < keys) ++b;
    return b;
}

hipEvent_t take_event(gsta_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records a pair of events around the launches of one phase when profiling.
struct PhaseTimer {
    gsta_ctx* ctx;
    int phase;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    PhaseTimer(gsta_ctx* c, int ph, hipStream_t st) : ctx(c), phase(ph), s(st) {
        if (!(ctx->profiling & (1u << ph))) return;
        a = take_event(ctx);
        b = take_event(ctx);
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~PhaseTimer() {
        if (!a || !b) return;
        (void)hipEventRecord(b, s);
        ctx->pending.push_back({phase, a, b});
    }
};

// Base of the profiling counters for a compositing phase (each kernel writes
// its own fixed entries), or NULL when the phase is not profiled.
unsigned long long* pair_counter(gsta_ctx* ctx, int which) {
    const int phase = which == 0 ? GSTA_PHASE_COMPOSITE : GSTA_PHASE_COMPOSITE_BWD;
    return ((ctx->profiling & (1u << phase)) && (ctx->profiling & GSTA_PROFILE_COUNTERS)) ? ctx->pairs : nullptr;
}

}  // namespace

void gsta::set_noctx_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_noctx_err = buf;
}

extern "C" {

gsta_status gsta_create(const gsta_limits* lim, gsta_ctx** out) {
    if (!out) return GSTA_ERR_INVALID;
    *out = nullptr;
    gsta_ctx* ctx = new gsta_ctx();
    gsta_status st = check_limits(ctx, lim);
    if (st == GSTA_OK) st = allocate(ctx, lim);
    if (st != GSTA_OK) {
        // keep the context so the caller can read the message
        *out = ctx;
        return st;
    }
    *out = ctx;
    return GSTA_OK;
}

gsta_status gsta_reserve(gsta_ctx* ctx, const gsta_limits* lim) {
    if (ctx && ctx->capturing) return fail(ctx, GSTA_ERR_INVALID, "gsta_reserve synchronises: not while a graph is captured");
    if (!ctx) return GSTA_ERR_INVALID;
    gsta_status st = check_limits(ctx, lim);
    if (st != GSTA_OK) return st;
    gsta_limits nl = ctx->lim;
    nl.max_gaussians = std::max(nl.max_gaussians, lim->max_gaussians);
    nl.max_views = std::max(nl.max_views, lim->max_views);
    nl.max_height = std::max(nl.max_height, lim->max_height);
    nl.max_width = std::max(nl.max_width, lim->max_width);
    nl.instance_capacity = std::max(nl.instance_capacity, lim->instance_capacity);
    nl.n_slots = std::max(nl.n_slots, lim->n_slots);
    if (memcmp(&nl, &ctx->lim, sizeof(nl)) == 0 && !ctx->allocs.empty()) return GSTA_OK;
    st = check_limits(ctx, &nl);
    if (st != GSTA_OK) return st;
    if ((st = hip_check(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize")) != GSTA_OK) return st;
    free_all(ctx);
    return allocate(ctx, &nl);
}

void gsta_destroy(gsta_ctx* ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (auto& p : ctx->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    free_all(ctx);
    delete ctx;
}

gsta_status gsta_set_option(gsta_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    switch (option) {
        case GSTA_OPT_FWD_WAVES:
            if (value != 0 && value != 1 && value != 2 && value != 4)
                return fail(ctx, GSTA_ERR_INVALID, "forward waves per tile must be 0, 1, 2 or 4");
            ctx->fwd_waves = (int)value;
            return GSTA_OK;
        case GSTA_OPT_BWD_WAVES:
            if (value != 1 && value != 2 && value != 4)
                return fail(ctx, GSTA_ERR_INVALID, "backward waves per tile must be 1, 2 or 4");
            ctx->bwd_waves = (int)value;
            ctx->bwd_blocks = ctx->cus * composite_bwd_blocks_per_cu(ctx->bwd_waves);
            return GSTA_OK;
        case GSTA_OPT_BWD_SEGMENT: {
            if (value == 0) {
                ctx->seg_shift = 31;
                return GSTA_OK;
            }
            int sh = 0;
            while (sh < 30 && ((int64_t)1 << sh) < value) ++sh;
            if (((int64_t)1 << sh) != value || sh < kMinSegShift || sh > 16)
                return fail(ctx, GSTA_ERR_INVALID, "backward segment length must be 0 or a power of two in [64, 65536]");
            ctx->seg_shift = (uint32_t)sh;
            return GSTA_OK;
        }
        case GSTA_OPT_BINNING:
            if (value != 0 && value != 1) return fail(ctx, GSTA_ERR_INVALID, "binning must be 0 or 1");
            ctx->binning = (int)value;
            return GSTA_OK;
        case GSTA_OPT_DEPTH_SORT:
            if (value < 0 || value > 2) return fail(ctx, GSTA_ERR_INVALID, "depth sort must be 0, 1 or 2");
            ctx->depth_sort = (int)value;
            return GSTA_OK;
        case GSTA_OPT_BWD_VARIANT:
            if (value != 0 && value != 1) return fail(ctx, GSTA_ERR_INVALID, "backward variant must be 0 or 1");
            ctx->bwd_variant = (int)value;
            return GSTA_OK;
        default:
            return fail(ctx, GSTA_ERR_INVALID, "unknown option %d", option);
    }
}

gsta_status gsta_set_profiling(gsta_ctx* ctx, int32_t phase_mask) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (ctx->capturing && phase_mask) return fail(ctx, GSTA_ERR_INVALID, "no profiling while a graph is captured");
    ctx->profiling = (uint32_t)phase_mask & (((1u << GSTA_N_PHASES) - 1u) | GSTA_PROFILE_COUNTERS);
    return GSTA_OK;
}

gsta_status gsta_read_profile(gsta_ctx* ctx, double* ms, int64_t* launches, int64_t* pairs) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = hip_check(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize")) != GSTA_OK) return st;
    for (auto& p : ctx->pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            ctx->ms[p.phase] += t;
            ctx->launches[p.phase] += 1;
        }
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
    unsigned long long pr[kCounters] = {};
    if ((st = hip_check(ctx, hipMemcpy(pr, ctx->pairs, sizeof(pr), hipMemcpyDeviceToHost), "read pairs")) != GSTA_OK)
        return st;
    const unsigned long long z[kCounters] = {};
    if ((st = hip_check(ctx, hipMemcpy(ctx->pairs, z, sizeof(z), hipMemcpyHostToDevice), "clear pairs")) != GSTA_OK)
        return st;
    for (int i = 0; i < GSTA_N_PHASES; ++i) {
        if (ms) ms[i] = ctx->ms[i];
        if (launches) launches[i] = ctx->launches[i];
        ctx->ms[i] = 0.0;
        ctx->launches[i] = 0;
    }
    if (pairs)
        for (int i = 0; i < kCounters; ++i) pairs[i] = (int64_t)pr[i];
    return GSTA_OK;
}

const char* gsta_last_error(const gsta_ctx* ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

gsta_status gsta_check(gsta_ctx* ctx, hipStream_t stream, int64_t* max_instances) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (ctx->capturing) return fail(ctx, GSTA_ERR_INVALID, "gsta_check synchronises: not while a graph is captured");
    gsta_status st;
    if ((st = hip_check(ctx, hipStreamSynchronize(stream), "hipStreamSynchronize")) != GSTA_OK) return st;
    uint32_t flags[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t mi = 0;
    if ((st = hip_check(ctx, hipMemcpy(flags, ctx->flags, sizeof(flags), hipMemcpyDeviceToHost), "read flags")) != GSTA_OK)
        return st;
    if ((st = hip_check(ctx, hipMemcpy(&mi, ctx->max_inst, sizeof(mi), hipMemcpyDeviceToHost), "read counts")) != GSTA_OK)
        return st;
    const uint32_t zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint64_t z64 = 0;
    if ((st = hip_check(ctx, hipMemcpy(ctx->flags, zeros, sizeof(zeros), hipMemcpyHostToDevice), "clear flags")) != GSTA_OK)
        return st;
    if ((st = hip_check(ctx, hipMemcpy(ctx->max_inst, &z64, sizeof(z64), hipMemcpyHostToDevice), "clear counts")) != GSTA_OK)
        return st;
    if (max_instances) *max_instances = (int64_t)mi;
    if (flags[0]) return fail(ctx, GSTA_ERR_CAPACITY, "tile instances (%llu) exceeded the capacity (%lld)",
                              (unsigned long long)mi, (long long)ctx->lim.instance_capacity);
    if (flags[2]) return fail(ctx, GSTA_ERR_CAPACITY, "densified set exceeded the output capacity");
    if (flags[3]) return fail(ctx, GSTA_ERR_CAPACITY, "compositing checkpoints exceeded their pool (%u slots)",
                              ctx->pool_cap);
    if (flags[4]) return fail(ctx, GSTA_ERR_HIP, "the depth sort's look-back did not complete (spin bound reached)");
    if (flags[1]) return fail(ctx, GSTA_ERR_NONFINITE, "non-finite gradient met by the optimizer");
    return GSTA_OK;
}

gsta_status gsta_get_state(gsta_ctx* ctx, int32_t slot, int32_t field, void* dst, int64_t bytes,
                           hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (slot < 0 || slot >= (int)ctx->slots.size()) return fail(ctx, GSTA_ERR_INVALID, "bad slot %d", slot);
    Slot& s = ctx->slots[slot];
    if (!s.valid) return fail(ctx, GSTA_ERR_INVALID, "slot %d holds no forward state", slot);
    if (!dst) return fail(ctx, GSTA_ERR_INVALID, "dst is NULL");
    const int64_t n = s.n, V = s.nv, S = ctx->stride;
    const int64_t HW = (int64_t)s.cams[0].width * s.cams[0].height;
    const int64_t T = tiles_of(s.cams[0].width, s.cams[0].height);
    const void* src = nullptr;
    int64_t elem = 0, rows = 1, row_elems = 0, src_pitch = 0;
    switch (field) {
        case GSTA_STATE_REC_GEO: src = s.geo; elem = 16; rows = V; row_elems = n; src_pitch = S; break;
        case GSTA_STATE_REC_COL: src = s.col; elem = 16; rows = V; row_elems = n; src_pitch = S; break;
        case GSTA_STATE_REC_RGB: src = s.rgb; elem = 16; rows = V; row_elems = n; src_pitch = S; break;
        case GSTA_STATE_RECT: src = s.rect; elem = 8; rows = V; row_elems = n; src_pitch = S; break;
        case GSTA_STATE_DEPTH_ORDER: src = s.dval[s.depth_buf]; elem = 4; rows = V; row_elems = n; src_pitch = S; break;
        case GSTA_STATE_INST_KEYS: src = s.ikey[s.inst_buf]; elem = 4; row_elems = ctx->lim.instance_capacity; src_pitch = row_elems; break;
        case GSTA_STATE_INST_IDS: src = s.ival[s.inst_buf]; elem = 4; row_elems = ctx->lim.instance_capacity; src_pitch = row_elems; break;
        case GSTA_STATE_RANGES: src = s.ranges; elem = 8; row_elems = V * T; src_pitch = row_elems; break;
        case GSTA_STATE_T_FINAL: src = s.T_final; elem = 4; row_elems = V * HW; src_pitch = row_elems; break;
        case GSTA_STATE_LAST: src = s.last; elem = 4; row_elems = V * HW; src_pitch = row_elems; break;
        case GSTA_STATE_N_INSTANCES: src = s.n_total; elem = 8; row_elems = 1; src_pitch = 1; break;
        case GSTA_STATE_INST_GID: src = s.inst_gid; elem = 4; row_elems = ctx->lim.instance_capacity; src_pitch = row_elems; break;
        default: return fail(ctx, GSTA_ERR_INVALID, "unknown state field %d", field);
    }
    const int64_t full = rows * row_elems * elem;
    if (bytes < 0 || bytes > full) return fail(ctx, GSTA_ERR_INVALID, "bytes %lld > field size %lld", (long long)bytes, (long long)full);
    if (field == GSTA_STATE_INST_KEYS && s.placed) {
        // placed lists carry no keys: write them from the tile ranges
        launch_keys_from_ranges(s.ranges, V * T, s.ikey[0], stream);
        gsta_status st = hip_check(ctx, hipGetLastError(), "keys from ranges");
        if (st != GSTA_OK) return st;
        src = s.ikey[0];
    }
    if (field == GSTA_STATE_INST_GID) {
        // the lists are built without the per-expansion-index gids
        launch_gid_by_index(s.ival[s.inst_buf], s.gsort, s.n_count, ctx->lim.instance_capacity, s.inst_gid,
                            stream);
        gsta_status st = hip_check(ctx, hipGetLastError(), "gids by index");
        if (st != GSTA_OK) return st;
    }
    if (rows == 1 || src_pitch == row_elems) {
        return hip_check(ctx, hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, stream), "copy state");
    }
    if (bytes != full) return fail(ctx, GSTA_ERR_INVALID, "per-view fields are copied whole (%lld bytes)", (long long)full);
    return hip_check(ctx, hipMemcpy2DAsync(dst, (size_t)(row_elems * elem), src, (size_t)(src_pitch * elem),
                                           (size_t)(row_elems * elem), (size_t)rows, hipMemcpyDeviceToDevice, stream),
                     "copy state");
}

}  // extern "C"

namespace {

gsta_status render_forward(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams, int32_t n_views,
                           const float* bg, float* image, int32_t state_slot, FusedL1 l1, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = check_params(ctx, g, "g")) != GSTA_OK) return st;
    if ((st = check_sh_mask(ctx, g)) != GSTA_OK) return st;
    CamArray ca;
    if ((st = check_views(ctx, cams, n_views, ca)) != GSTA_OK) return st;
    if (!bg) return fail(ctx, GSTA_ERR_INVALID, "bg is NULL");
    if (!image) return fail(ctx, GSTA_ERR_INVALID, "image is NULL");
    if (state_slot < 0 || state_slot >= (int)ctx->slots.size())
        return fail(ctx, GSTA_ERR_INVALID, "state_slot %d outside [0, %d)", state_slot, (int)ctx->slots.size());
    Slot& s = ctx->slots[state_slot];
    const int64_t n = g->n, S = ctx->stride;
    const int nv = n_views;
    const int ntx = ca.c[0].ntx;
    const int64_t T = (int64_t)ca.c[0].ntx * ca.c[0].nty;

    // depth sort: one kernel per pass for short views (default), onesweep, or
    // the hist / scan / scatter passes; the preprocess provides the first
    // pass's digit counts for the first (added to its zeroed count table) and
    // (with chunks of 256 keys) the last
    const bool small = ctx->depth_sort == 0 && n <= kSmallSortKeys;
    const bool onesweep = ctx->depth_sort == 1 && n < ((int64_t)1 << 30);
    const bool hist_given = small || (!onesweep && ctx->items_depth == 1);
    uint32_t* hist0 = !hist_given ? nullptr : small ? ctx->sort_cnt : ctx->hist;
    if (n > 0) {
        PhaseTimer pt(ctx, GSTA_PHASE_PREPROCESS, stream);
        launch_preprocess_fwd(g->block, g->ld, n, g->sh_degree, ca, nv, s.geo, s.col, s.rgb, s.rect,
                              s.dkey[0], s.dval[0], S, hist0, small, g->opacity_act,
                              sh_mask_of(g, nullptr), stream);
    }
    {
        PhaseTimer pt(ctx, GSTA_PHASE_DEPTH_SORT, stream);
        if (n == 0) {
            s.depth_buf = 0;
        } else if (small) {
            s.depth_buf = radix_sort_small(s.dkey, s.dval, S, nv, (uint32_t)n, ctx->sort_cnt,
                                           small_sort_count_words(ctx->lim.max_views), ctx->sort_pre, stream);
        } else if (onesweep) {
            OnesweepScratch os{ctx->os_tot, ctx->os_status, ctx->os_tickets};
            s.depth_buf = radix_sort_onesweep(s.dkey, s.dval, S, nv, (uint32_t)n, os, ctx->flags, stream);
        } else {
            RadixScratch rd{ctx->hist, ctx->digit_tot, ctx->chunks_depth, ctx->items_depth, hist_given};
            s.depth_buf = radix_sort_pairs(s.dkey, s.dval, S, nv, nullptr, (uint32_t)n, 32, rd, stream);
        }
    }
    s.placed = ctx->binning == 0 && nv <= ctx->place_views && T <= kPlaceMaxTiles;
    if (s.placed) {
        // one pass from the depth order to the tile lists (no tile-key sort)
        PhaseTimer pt(ctx, GSTA_PHASE_BINNING, stream);
        Clears cl;
        cl.ptr[0] = s.tile_last;
        cl.count[0] = T * nv;
        cl.ptr[1] = s.ck_ctr;
        cl.count[1] = 1;
        launch_place(s.rect, s.dval[s.depth_buf], S, n, nv, ntx, ca.c[0].nty, ctx->place_cnt, ctx->tile_tot,
                     ctx->partials, s.n_total, s.n_count, s.ival[0], s.gsort, s.inst_off, s.ranges,
                     (uint64_t)ctx->lim.instance_capacity, ctx->flags, ctx->max_inst, cl, stream);
        s.inst_buf = 0;
    } else {
        {
            PhaseTimer pt(ctx, GSTA_PHASE_BINNING, stream);
            Clears cl;
            cl.ptr[0] = reinterpret_cast<uint32_t*>(s.ranges);
            cl.count[0] = 2 * T * nv;
            cl.ptr[1] = s.tile_last;
            cl.count[1] = T * nv;
            cl.ptr[2] = s.ck_ctr;
            cl.count[2] = 1;
            launch_expand(s.rect, s.dval[s.depth_buf], S, n, nv, ntx, (int)T, ctx->partials, s.n_total,
                          s.n_count, s.ikey[0], s.ival[0], s.rank_tab, s.inst_off,
                          (uint64_t)ctx->lim.instance_capacity, ctx->flags, ctx->max_inst, cl, stream);
        }
        PhaseTimer pt(ctx, GSTA_PHASE_TILE_SORT, stream);
        RadixScratch ri{ctx->hist, ctx->digit_tot, ctx->chunks_inst, ctx->items_inst};
        s.inst_buf = radix_sort_pairs(s.ikey, s.ival, 0, 1, s.n_count, 0u, key_bits(T * nv), ri, stream);
        launch_ranges(s.ikey[s.inst_buf], s.ival[s.inst_buf], s.rank_tab, S, (int)T, ntx, s.n_count,
                      ctx->lim.instance_capacity, s.ranges, s.gsort, stream);
    }
    {
        PhaseTimer pt(ctx, GSTA_PHASE_COMPOSITE, stream);
        s.shift = ctx->seg_shift;
        if (l1.target) {
            l1.part = ctx->fwd_lpart;
            l1.inv = 1.0f / (float)(nv * 3 * (int64_t)ca.c[0].width * ca.c[0].height);
        }
        launch_composite_fwd(ctx->fwd_waves, s.ranges, s.gsort, s.geo, s.col, s.rgb, S, ca,
                             nv, bg[0], bg[1], bg[2], image, s.T_final, s.last, s.cfg, seg_ckpt(ctx, s),
                             pair_counter(ctx, 0), l1, stream);
    }
    if ((st = hip_check(ctx, hipGetLastError(), "render_forward launch")) != GSTA_OK) {
        s.valid = false;
        return st;
    }
    s.valid = true;
    s.n = n;
    s.ld = g->ld;
    s.degree = g->sh_degree;
    s.block = g->block;
    s.sh_mask = g->sh_mask;
    s.sh_mask_threshold = g->sh_mask_threshold;
    s.nv = nv;
    for (int v = 0; v < nv; ++v) s.cams[v] = cams[v];
    for (int c = 0; c < 3; ++c) s.bg[c] = bg[c];
    return GSTA_OK;
}

}  // namespace

extern "C" {

gsta_status gsta_render_forward(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams,
                                int32_t n_views, const float* bg, float* image, int32_t state_slot,
                                hipStream_t stream) {
    return render_forward(ctx, g, cams, n_views, bg, image, state_slot, FusedL1{}, stream);
}

gsta_status gsta_render_forward_l1(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams,
                                   int32_t n_views, const float* bg, const float* target, float* image,
                                   float* dL_dimage, double* sums, int32_t state_slot, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (!target || !dL_dimage || !sums) return fail(ctx, GSTA_ERR_INVALID, "NULL target, dL_dimage or sums");
    FusedL1 l1;
    l1.target = target;
    l1.dL = dL_dimage;
    l1.sums = sums;
    return render_forward(ctx, g, cams, n_views, bg, image, state_slot, l1, stream);
}

gsta_status gsta_render_backward(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams,
                                 int32_t n_views, const float* bg, int32_t state_slot,
                                 const float* dL_dimage, const uint8_t* frozen, gsta_params* grad,
                                 float* grad2d, float* ema, float ema_beta, float* dstats,
                                 hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = check_params(ctx, g, "g")) != GSTA_OK) return st;
    if ((st = check_sh_mask(ctx, g)) != GSTA_OK) return st;
    if ((st = check_params(ctx, grad, "grad")) != GSTA_OK) return st;
    CamArray ca;
    if ((st = check_views(ctx, cams, n_views, ca)) != GSTA_OK) return st;
    if (!bg || !dL_dimage) return fail(ctx, GSTA_ERR_INVALID, "bg or dL_dimage is NULL");
    if (grad->n != g->n || grad->sh_degree != g->sh_degree)
        return fail(ctx, GSTA_ERR_INVALID, "grad must match g in n and sh_degree");
    if (!(ema_beta >= 0.f && ema_beta < 1.f)) return fail(ctx, GSTA_ERR_INVALID, "ema_beta must be in [0, 1)");
    if (state_slot < 0 || state_slot >= (int)ctx->slots.size())
        return fail(ctx, GSTA_ERR_INVALID, "state_slot %d outside [0, %d)", state_slot, (int)ctx->slots.size());
    Slot& s = ctx->slots[state_slot];
    if (!s.valid) return fail(ctx, GSTA_ERR_INVALID, "state_slot %d holds no forward state", state_slot);
    bool same = s.n == g->n && s.ld == g->ld && s.degree == g->sh_degree && s.block == g->block && s.nv == n_views &&
                memcmp(s.cams, cams, sizeof(gsta_camera) * n_views) == 0 && s.bg[0] == bg[0] && s.bg[1] == bg[1] &&
                s.bg[2] == bg[2] && s.sh_mask == g->sh_mask &&
                (!g->sh_mask || s.sh_mask_threshold == g->sh_mask_threshold);
    if (!same) return fail(ctx, GSTA_ERR_INVALID, "backward arguments differ from the forward in slot %d", state_slot);
    const int64_t n = g->n, S = ctx->stride;
    const int nv = n_views;
    {
        PhaseTimer pt(ctx, GSTA_PHASE_COMPOSITE_BWD, stream);
        unsigned long long* pairs = pair_counter(ctx, 1);
        if (ctx->bwd_variant == 1 && !pairs)   // (the pair counts come from the per-pixel variant)
            launch_composite_bwd_splat(ctx->bwd_splat_blocks, s.ranges, s.ival[s.inst_buf], s.gsort, s.geo, s.col,
                                       s.rgb, S, frozen, ca, nv, bg[0], bg[1], bg[2], s.T_final, s.last, s.cfg,
                                       dL_dimage, ctx->tile_grads, seg_ckpt(ctx, s), stream);
        else
            launch_composite_bwd(ctx->bwd_waves, ctx->bwd_blocks, s.ranges, s.ival[s.inst_buf], s.gsort, s.geo,
                                 s.col, s.rgb, S, frozen, ca, nv, bg[0], bg[1], bg[2], s.T_final, s.last, s.cfg,
                                 dL_dimage, ctx->tile_grads, s.n_count, seg_ckpt(ctx, s), pairs, stream);
    }
    if (n > 0) {
        PhaseTimer pt(ctx, GSTA_PHASE_PREPROCESS_BWD, stream);
        launch_preprocess_bwd(g->block, g->ld, n, g->sh_degree, ca, nv, s.rect, s.inst_off, S, ctx->tile_grads,
                              ctx->stamps, ctx->gen, s.n_count, frozen, ctx->d2sum, grad->block,
                              grad->ld, ema, ema_beta, grad2d, dstats, g->opacity_act,
                              sh_mask_of(g, grad->sh_mask), stream);
    }
    return hip_check(ctx, hipGetLastError(), "render_backward launch");
}

gsta_status gsta_adam_masked(gsta_ctx* ctx, gsta_params* p, const gsta_params* grad, gsta_params* m,
                             gsta_params* v, const float* lr_per_row, float beta1, float beta2, float eps,
                             int32_t step, const uint8_t* frozen, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = check_params(ctx, p, "p")) != GSTA_OK) return st;
    if ((st = check_params(ctx, grad, "grad")) != GSTA_OK) return st;
    if ((st = check_params(ctx, m, "m")) != GSTA_OK) return st;
    if ((st = check_params(ctx, v, "v")) != GSTA_OK) return st;
    if (grad->n != p->n || m->n != p->n || v->n != p->n || grad->sh_degree != p->sh_degree ||
        m->sh_degree != p->sh_degree || v->sh_degree != p->sh_degree)
        return fail(ctx, GSTA_ERR_INVALID, "p, grad, m, v must share n and sh_degree");
    if (!lr_per_row) return fail(ctx, GSTA_ERR_INVALID, "lr_per_row is NULL");
    if (step < 1) return fail(ctx, GSTA_ERR_INVALID, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return fail(ctx, GSTA_ERR_INVALID, "betas must be in [0, 1) and eps >= 0");
    const int rows = n_rows(p->sh_degree);
    LrArray lr;
    for (int r = 0; r < 64; ++r) lr.lr[r] = r < rows ? lr_per_row[r] : 0.f;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    PhaseTimer pt(ctx, GSTA_PHASE_ADAM, stream);
    if (p->n > 0)
        launch_adam(p->block, p->ld, grad->block, grad->ld, m->block, m->ld, v->block, v->ld, p->n, rows, lr, beta1,
                    beta2, eps, bc1, bc2, frozen, ctx->flags, stream);
    return hip_check(ctx, hipGetLastError(), "adam launch");
}

static_assert(sizeof(gsta_adam_sched) == sizeof(AdamSched), "gsta_adam_sched layout");

gsta_status gsta_adam_masked_sched(gsta_ctx* ctx, gsta_params* p, const gsta_params* grad, gsta_params* m,
                                   gsta_params* v, gsta_adam_sched* sched, const uint8_t* frozen,
                                   hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = check_params(ctx, p, "p")) != GSTA_OK) return st;
    if ((st = check_params(ctx, grad, "grad")) != GSTA_OK) return st;
    if ((st = check_params(ctx, m, "m")) != GSTA_OK) return st;
    if ((st = check_params(ctx, v, "v")) != GSTA_OK) return st;
    if (grad->n != p->n || m->n != p->n || v->n != p->n || grad->sh_degree != p->sh_degree ||
        m->sh_degree != p->sh_degree || v->sh_degree != p->sh_degree)
        return fail(ctx, GSTA_ERR_INVALID, "p, grad, m, v must share n and sh_degree");
    if (!sched) return fail(ctx, GSTA_ERR_INVALID, "sched is NULL");
    PhaseTimer pt(ctx, GSTA_PHASE_ADAM, stream);
    launch_adam_sched(p->block, p->ld, grad->block, grad->ld, m->block, m->ld, v->block, v->ld, p->n,
                      n_rows(p->sh_degree), reinterpret_cast<AdamSched*>(sched), frozen, ctx->flags, stream);
    return hip_check(ctx, hipGetLastError(), "adam launch");
}

gsta_status gsta_update_freeze_mask(gsta_ctx* ctx, const float* score_xyz, const float* score_rgb, int64_t n,
                                    float eps_xyz, float eps_rgb, int32_t mode, const uint8_t* proposal,
                                    uint8_t* frozen, int64_t* n_frozen, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (mode < 0 || mode > 2) return fail(ctx, GSTA_ERR_INVALID, "mode must be 0, 1 or 2");
    if (n < 0) return fail(ctx, GSTA_ERR_INVALID, "n < 0");
    if (!frozen && n > 0) return fail(ctx, GSTA_ERR_INVALID, "frozen is NULL");
    if (mode != 1 && n > 0 && (!score_xyz || !score_rgb))
        return fail(ctx, GSTA_ERR_INVALID, "scores are NULL");
    PhaseTimer pt(ctx, GSTA_PHASE_FREEZE, stream);
    launch_freeze(score_xyz, score_rgb, n, eps_xyz, eps_rgb, mode, proposal, frozen, n_frozen, stream);
    return hip_check(ctx, hipGetLastError(), "freeze launch");
}

gsta_status gsta_dssim_loss(gsta_ctx* ctx, const float* image, const float* target, int32_t n_views,
                            int32_t height, int32_t width, float lambda, float* dL_dimage, double* ssim_sum,
                            hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (n_views < 1 || n_views > ctx->lim.max_views || height < 1 || height > ctx->lim.max_height || width < 1 ||
        width > ctx->lim.max_width)
        return fail(ctx, GSTA_ERR_INVALID, "views x height x width = %d x %d x %d beyond the reserved %d x %d x %d",
                    n_views, height, width, ctx->lim.max_views, ctx->lim.max_height, ctx->lim.max_width);
    if (!(lambda >= 0.f && lambda <= 1.f)) return fail(ctx, GSTA_ERR_INVALID, "lambda must be in [0, 1]");
    if (!image || !target || !dL_dimage || !ssim_sum) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    PhaseTimer pt(ctx, GSTA_PHASE_LOSS, stream);
    launch_dssim(image, target, n_views, height, width, lambda, dL_dimage, ssim_sum, ctx->ssim_g, ctx->ssim_part,
                 stream);
    return hip_check(ctx, hipGetLastError(), "dssim launch");
}

gsta_status gsta_adam_rows(gsta_ctx* ctx, float* p, const float* grad, float* m, float* v, int64_t n,
                           int64_t ld, int32_t rows, const float* lr_per_row, float beta1, float beta2, float eps,
                           int32_t step, const uint8_t* frozen, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (n < 0 || n > ctx->lim.max_gaussians)
        return fail(ctx, GSTA_ERR_INVALID, "n = %lld outside [0, max_gaussians = %lld]", (long long)n,
                    (long long)ctx->lim.max_gaussians);
    if (ld < n || ld < 1) return fail(ctx, GSTA_ERR_INVALID, "ld < n");
    if (rows < 1 || rows > 64) return fail(ctx, GSTA_ERR_INVALID, "rows must be in [1, 64]");
    if (n > 0 && (!p || !grad || !m || !v)) return fail(ctx, GSTA_ERR_INVALID, "NULL p, grad, m or v");
    if (!lr_per_row) return fail(ctx, GSTA_ERR_INVALID, "lr_per_row is NULL");
    if (step < 1) return fail(ctx, GSTA_ERR_INVALID, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return fail(ctx, GSTA_ERR_INVALID, "betas must be in [0, 1) and eps >= 0");
    LrArray lr;
    for (int r = 0; r < 64; ++r) lr.lr[r] = r < rows ? lr_per_row[r] : 0.f;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    PhaseTimer pt(ctx, GSTA_PHASE_ADAM, stream);
    if (n > 0) launch_adam(p, ld, grad, ld, m, ld, v, ld, n, rows, lr, beta1, beta2, eps, bc1, bc2, frozen, ctx->flags, stream);
    return hip_check(ctx, hipGetLastError(), "adam_rows launch");
}

gsta_status gsta_sh_mask_reg(gsta_ctx* ctx, const float* logits, int64_t n, int64_t ld, float threshold,
                             float lambda, const uint8_t* frozen, float* grad, double* out, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (n < 1 || n > ctx->lim.max_gaussians)
        return fail(ctx, GSTA_ERR_INVALID, "n = %lld outside [1, max_gaussians = %lld]", (long long)n,
                    (long long)ctx->lim.max_gaussians);
    if (ld < n) return fail(ctx, GSTA_ERR_INVALID, "ld < n");
    if (!(threshold > 0.f && threshold < 1.f)) return fail(ctx, GSTA_ERR_INVALID, "threshold must be in (0, 1)");
    if (!(lambda >= 0.f)) return fail(ctx, GSTA_ERR_INVALID, "lambda must be >= 0");
    if (!logits || !out) return fail(ctx, GSTA_ERR_INVALID, "NULL logits or out");
    const double t = (double)threshold;
    PhaseTimer pt(ctx, GSTA_PHASE_LOSS, stream);
    launch_sh_mask_reg(logits, n, ld, (float)std::log(t / (1.0 - t)), lambda, frozen, grad, ctx->shm_part, out,
                       stream);
    return hip_check(ctx, hipGetLastError(), "sh_mask_reg launch");
}

gsta_status gsta_update_freeze_mask_rule(gsta_ctx* ctx, int32_t rule, const float* score, int64_t n,
                                         double fraction, uint64_t seed, uint64_t draw, int32_t mode,
                                         uint8_t* frozen, int64_t* n_frozen, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (rule != GSTA_FREEZE_RULE_MINGRAD && rule != GSTA_FREEZE_RULE_RANDOM)
        return fail(ctx, GSTA_ERR_INVALID, "rule must be GSTA_FREEZE_RULE_MINGRAD or GSTA_FREEZE_RULE_RANDOM");
    if (mode < 0 || mode > 2) return fail(ctx, GSTA_ERR_INVALID, "mode must be 0, 1 or 2");
    if (!(fraction >= 0.0 && fraction <= 1.0)) return fail(ctx, GSTA_ERR_INVALID, "fraction must be in [0, 1]");
    if (n < 0 || n > ctx->lim.max_gaussians)
        return fail(ctx, GSTA_ERR_INVALID, "n = %lld outside [0, max_gaussians = %lld]", (long long)n,
                    (long long)ctx->lim.max_gaussians);
    if (!frozen && n > 0) return fail(ctx, GSTA_ERR_INVALID, "frozen is NULL");
    if (rule == GSTA_FREEZE_RULE_MINGRAD && !score && n > 0) return fail(ctx, GSTA_ERR_INVALID, "score is NULL");
    PhaseTimer pt(ctx, GSTA_PHASE_FREEZE, stream);
    if (rule == GSTA_FREEZE_RULE_RANDOM) {
        const double t = std::floor(fraction * 4294967296.0);
        const uint64_t thr = t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t;
        launch_freeze_random(n, thr, seed, draw, mode, frozen, n_frozen, stream);
    } else {
        launch_freeze_mingrad(score, n, fraction, mode, frozen, n_frozen, ctx->sel, ctx->sel_blk, stream);
    }
    return hip_check(ctx, hipGetLastError(), "freeze rule launch");
}

gsta_status gsta_partition_frozen(gsta_ctx* ctx, int64_t n, uint8_t* frozen, const gsta_columns* arrays,
                                  int32_t count, void* tmp, int64_t tmp_bytes, int64_t* n_active,
                                  hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (n < 0 || n > ctx->lim.max_gaussians)
        return fail(ctx, GSTA_ERR_INVALID, "n = %lld outside [0, max_gaussians = %lld]", (long long)n,
                    (long long)ctx->lim.max_gaussians);
    if (count < 0 || count > 64) return fail(ctx, GSTA_ERR_INVALID, "count = %d outside [0, 64]", count);
    if (count > 0 && !arrays) return fail(ctx, GSTA_ERR_INVALID, "arrays is NULL");
    if (n > 0 && !frozen) return fail(ctx, GSTA_ERR_INVALID, "frozen is NULL");
    // byte ranges [lo, hi) of every array, the mask and tmp; none may overlap
    std::vector<PartArray> pa((size_t)count);
    std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
    int64_t need = 0;
    for (int a = 0; a < count; ++a) {
        const gsta_columns& c = arrays[a];
        if (c.elem_bytes != 1 && c.elem_bytes != 2 && c.elem_bytes != 4)
            return fail(ctx, GSTA_ERR_INVALID, "arrays[%d].elem_bytes must be 1, 2 or 4", a);
        if (c.rows < 1 || c.ld < n) return fail(ctx, GSTA_ERR_INVALID, "arrays[%d]: rows < 1 or ld < n", a);
        if (n > 0 && !c.base) return fail(ctx, GSTA_ERR_INVALID, "arrays[%d].base is NULL", a);
        if (n > 0 && (uintptr_t)c.base % c.elem_bytes != 0)
            return fail(ctx, GSTA_ERR_INVALID, "arrays[%d].base is not aligned to its elements", a);
        pa[a] = PartArray{c.base, c.rows, c.ld, c.elem_bytes};
        need = std::max(need, c.rows * n * c.elem_bytes);
        if (n > 0) {
            const uintptr_t lo = (uintptr_t)c.base;
            ranges.push_back({lo, lo + (uintptr_t)(((c.rows - 1) * c.ld + n) * c.elem_bytes)});
        }
    }
    if (n > 0 && count > 0) {
        if (!tmp || tmp_bytes < need)
            return fail(ctx, GSTA_ERR_INVALID, "tmp holds %lld bytes, %lld needed", (long long)tmp_bytes,
                        (long long)need);
        if ((uintptr_t)tmp % 4 != 0) return fail(ctx, GSTA_ERR_INVALID, "tmp is not 4-byte aligned");
        ranges.push_back({(uintptr_t)tmp, (uintptr_t)tmp + (uintptr_t)need});
    }
    if (n > 0) ranges.push_back({(uintptr_t)frozen, (uintptr_t)frozen + (uintptr_t)n});
    for (size_t x = 0; x < ranges.size(); ++x)
        for (size_t y = x + 1; y < ranges.size(); ++y)
            if (ranges[x].first < ranges[y].second && ranges[y].first < ranges[x].second)
                return fail(ctx, GSTA_ERR_INVALID, "arrays, frozen and tmp must not overlap");
    PhaseTimer pt(ctx, GSTA_PHASE_FREEZE, stream);
    launch_partition(n, frozen, pa.data(), count, tmp, ctx->part_src, ctx->dens_boff, ctx->part_tot, n_active,
                     stream);
    return hip_check(ctx, hipGetLastError(), "partition launch");
}

gsta_status gsta_densify_prune(gsta_ctx* ctx, const gsta_params* g, const gsta_params* m,
                               const gsta_params* v, const float* ema, const uint8_t* frozen,
                               const float* dstats, const float* noise, const gsta_densify_cfg* cfg,
                               gsta_params* g_out, gsta_params* m_out, gsta_params* v_out,
                               float* ema_out, uint8_t* frozen_out, int64_t* counts, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    const gsta_params* in[3] = {g, m, v};
    gsta_params* out[3] = {g_out, m_out, v_out};
    const char* names[6] = {"g", "m", "v", "g_out", "m_out", "v_out"};
    for (int k = 0; k < 3; ++k) {
        if ((st = check_params(ctx, in[k], names[k])) != GSTA_OK) return st;
        if ((st = check_params(ctx, out[k], names[3 + k])) != GSTA_OK) return st;
    }
    const int64_t n = g->n, cap = g_out->n;
    const int D = g->sh_degree;
    if (g->opacity_act != 0)
        return fail(ctx, GSTA_ERR_INVALID, "densification prunes by the opacity logit: g.opacity_act must be 0");
    if (g->sh_mask)
        return fail(ctx, GSTA_ERR_INVALID, "densification does not carry SH-band masks (a finetune-stage parameter)");
    for (int k = 0; k < 3; ++k) {
        if (in[k]->n != n || in[k]->sh_degree != D || out[k]->sh_degree != D || out[k]->n != cap)
            return fail(ctx, GSTA_ERR_INVALID, "g, m, v must share n; outputs share the capacity; one sh_degree");
        if (n > 0 && !out[k]->block) return fail(ctx, GSTA_ERR_INVALID, "%s.block is NULL", names[3 + k]);
    }
    if (!cfg || !counts) return fail(ctx, GSTA_ERR_INVALID, "cfg or counts is NULL");
    if (n > 0 && !dstats) return fail(ctx, GSTA_ERR_INVALID, "dstats is NULL");
    if (!std::isfinite(cfg->split_log_scale) || !std::isfinite(cfg->prune_logit) ||
        !std::isfinite(cfg->child_log_scale_shift) || std::isnan(cfg->grad_threshold) ||
        std::isnan(cfg->rgb_threshold))
        return fail(ctx, GSTA_ERR_INVALID, "densify thresholds must be finite");
    // outputs must not overlap the inputs (the scatter reads while it writes)
    const int R = n_rows(D);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (n == 0) break;
            const char* ia = (const char*)in[a]->block;
            const char* ob = (const char*)out[b]->block;
            const size_t la = (size_t)((R - 1) * in[a]->ld + n) * sizeof(float);
            const size_t lb = (size_t)((R - 1) * out[b]->ld + cap) * sizeof(float);
            if (ia < ob + lb && ob < ia + la)
                return fail(ctx, GSTA_ERR_INVALID, "%s overlaps %s", names[3 + b], names[a]);
        }
    DensIO io;
    io.P = g->block; io.M = m->block; io.V = v->block;
    io.ld = g->ld; io.mld = m->ld; io.vld = v->ld; io.n = n; io.degree = D;
    io.ema = ema; io.frozen = frozen; io.stats = dstats; io.noise = noise;
    io.seed = cfg->noise_seed; io.draw = cfg->noise_draw;
    io.Po = g_out->block; io.Mo = m_out->block; io.Vo = v_out->block;
    io.old_ = g_out->ld; io.mold = m_out->ld; io.vold = v_out->ld; io.cap = cap;
    io.ema_o = ema_out; io.frozen_o = frozen_out;
    DensCfg dc;
    dc.grad_threshold = cfg->grad_threshold;
    dc.rgb_threshold = cfg->rgb_threshold;
    dc.use_rgb = cfg->use_rgb != 0;
    dc.split_log_scale = cfg->split_log_scale;
    dc.prune_logit = cfg->prune_logit;
    dc.child_log_scale_shift = cfg->child_log_scale_shift;
    PhaseTimer pt(ctx, GSTA_PHASE_DENSIFY, stream);
    launch_densify(io, dc, ctx->dens_code, ctx->dens_boff, ctx->dens_tot, counts, ctx->flags, stream);
    return hip_check(ctx, hipGetLastError(), "densify launch");
}

gsta_status gsta_opacity_reset(gsta_ctx* ctx, gsta_params* g, gsta_params* m, gsta_params* v,
                               const uint8_t* frozen, float logit_cap, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = check_params(ctx, g, "g")) != GSTA_OK) return st;
    if ((st = check_params(ctx, m, "m")) != GSTA_OK) return st;
    if ((st = check_params(ctx, v, "v")) != GSTA_OK) return st;
    if (m->n != g->n || v->n != g->n) return fail(ctx, GSTA_ERR_INVALID, "g, m, v must share n");
    if (!std::isfinite(logit_cap)) return fail(ctx, GSTA_ERR_INVALID, "logit_cap must be finite");
    if (g->opacity_act != 0) return fail(ctx, GSTA_ERR_INVALID, "the opacity reset caps the logit: g.opacity_act must be 0");
    PhaseTimer pt(ctx, GSTA_PHASE_DENSIFY, stream);
    launch_opacity_reset(g->block, g->ld, m->block, m->ld, v->block, v->ld, g->n, frozen, logit_cap, stream);
    return hip_check(ctx, hipGetLastError(), "opacity reset launch");
}

gsta_status gsta_opacity_to_absolute(gsta_ctx* ctx, gsta_params* g, gsta_params* m, gsta_params* v,
                                     hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    gsta_status st;
    if ((st = check_params(ctx, g, "g")) != GSTA_OK) return st;
    if ((st = check_params(ctx, m, "m")) != GSTA_OK) return st;
    if ((st = check_params(ctx, v, "v")) != GSTA_OK) return st;
    if (m->n != g->n || v->n != g->n) return fail(ctx, GSTA_ERR_INVALID, "g, m, v must share n");
    if (g->opacity_act != 0) return fail(ctx, GSTA_ERR_INVALID, "g already uses the absolute activation");
    PhaseTimer pt(ctx, GSTA_PHASE_DENSIFY, stream);
    launch_opacity_to_abs(g->block, g->ld, m->block, m->ld, v->block, v->ld, g->n, stream);
    return hip_check(ctx, hipGetLastError(), "opacity activation switch launch");
}

// ---- learned freeze proposer ----------------------------------------------

#define GSTA_CTX_OK()                                                 \
    do {                                                              \
        if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;     \
    } while (0)

gsta_status gsta_traj_push(gsta_ctx* ctx, const float* ema, int64_t n, uint16_t* ring, int32_t slot,
                           hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 0 || slot < 0 || slot > 7) return fail(ctx, GSTA_ERR_INVALID, "n < 0 or slot outside [0, 8)");
    if (n > 0 && (!ema || !ring)) return fail(ctx, GSTA_ERR_INVALID, "ema or ring is NULL");
    launch_traj_push(ema, n, ring, slot, stream);
    return hip_check(ctx, hipGetLastError(), "trajectory push launch");
}

gsta_status gsta_mlp_feature_stats(gsta_ctx* ctx, const uint16_t* ring, int64_t n, int32_t head, double* sums,
                                   hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 0 || head < 0 || head > 7) return fail(ctx, GSTA_ERR_INVALID, "n < 0 or head outside [0, 8)");
    if (!sums || (n > 0 && !ring)) return fail(ctx, GSTA_ERR_INVALID, "ring or sums is NULL");
    launch_mlp_stats(ring, n, head, ctx->mlp_stats, sums, stream);
    return hip_check(ctx, hipGetLastError(), "feature statistics launch");
}

gsta_status gsta_mlp_features(gsta_ctx* ctx, const uint16_t* ring, int64_t n, int32_t head, const float* mean,
                              const float* std_dev, uint16_t* x, hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 0 || head < 0 || head > 7) return fail(ctx, GSTA_ERR_INVALID, "n < 0 or head outside [0, 8)");
    if (n > 0 && (!ring || !mean || !std_dev || !x)) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    if (((uintptr_t)x & 15u) != 0) return fail(ctx, GSTA_ERR_INVALID, "x must be 16-byte aligned");
    launch_mlp_features(ring, n, head, mean, std_dev, x, stream);
    return hip_check(ctx, hipGetLastError(), "features launch");
}

gsta_status gsta_mlp_forward(gsta_ctx* ctx, const uint16_t* w_bf16, const float* w, const uint16_t* x, int64_t n,
                             float* logits, uint16_t* h1, float* h2, hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 0) return fail(ctx, GSTA_ERR_INVALID, "n < 0");
    if (n > 0 && (!w_bf16 || !w || !x || !logits)) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    if ((((uintptr_t)x | (uintptr_t)w_bf16 | (uintptr_t)h1) & 15u) != 0)
        return fail(ctx, GSTA_ERR_INVALID, "x, w_bf16 and h1 must be 16-byte aligned");
    PhaseTimer pt(ctx, GSTA_PHASE_FREEZE, stream);
    launch_mlp_forward(w_bf16, w, x, n, logits, h1, h2, ctx->cus * 4, stream);
    return hip_check(ctx, hipGetLastError(), "mlp forward launch");
}

gsta_status gsta_mlp_bce(gsta_ctx* ctx, const float* logits, const uint8_t* labels, int64_t n, float* dz,
                         double* loss, hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 1) return fail(ctx, GSTA_ERR_INVALID, "n must be >= 1");
    if (!logits || !labels || !dz || !loss) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    launch_mlp_bce(logits, labels, n, dz, loss, ctx->loss_part, stream);
    return hip_check(ctx, hipGetLastError(), "bce launch");
}

gsta_status gsta_mlp_backward(gsta_ctx* ctx, const uint16_t* w_bf16, const float* w, const uint16_t* x,
                              const uint16_t* h1, const float* h2, const float* dz, int64_t n, float* grad,
                              hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 0) return fail(ctx, GSTA_ERR_INVALID, "n < 0");
    if (!w_bf16 || !w || !grad || (n > 0 && (!x || !h1 || !h2 || !dz)))
        return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    launch_mlp_backward(w_bf16, w, x, h1, h2, dz, n, ctx->mlp_part, grad, stream);
    return hip_check(ctx, hipGetLastError(), "mlp backward launch");
}

gsta_status gsta_mlp_adam(gsta_ctx* ctx, float* w, const float* grad, float* m, float* v, float lr, float beta1,
                          float beta2, float eps, int32_t step, uint16_t* w_bf16, hipStream_t stream) {
    GSTA_CTX_OK();
    if (!w || !grad || !m || !v || !w_bf16) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    if (step < 1) return fail(ctx, GSTA_ERR_INVALID, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return fail(ctx, GSTA_ERR_INVALID, "betas must be in [0, 1) and eps >= 0");
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    launch_mlp_adam(w, grad, m, v, lr, beta1, beta2, eps, bc1, bc2, w_bf16, stream);
    return hip_check(ctx, hipGetLastError(), "mlp adam launch");
}

gsta_status gsta_mlp_sync_bf16(gsta_ctx* ctx, const float* w, uint16_t* w_bf16, hipStream_t stream) {
    GSTA_CTX_OK();
    if (!w || !w_bf16) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    launch_mlp_bf16_copy(w, w_bf16, stream);
    return hip_check(ctx, hipGetLastError(), "bf16 copy launch");
}

gsta_status gsta_mlp_propose(gsta_ctx* ctx, const float* logits, const float* score_xyz, const float* score_rgb,
                             int64_t n, float logit_threshold, float veto_xyz, float veto_rgb, uint8_t* proposal,
                             hipStream_t stream) {
    GSTA_CTX_OK();
    if (n < 0) return fail(ctx, GSTA_ERR_INVALID, "n < 0");
    if (n > 0 && (!logits || !score_xyz || !score_rgb || !proposal))
        return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    PhaseTimer pt(ctx, GSTA_PHASE_FREEZE, stream);
    launch_mlp_propose(logits, score_xyz, score_rgb, n, logit_threshold, veto_xyz, veto_rgb, proposal, stream);
    return hip_check(ctx, hipGetLastError(), "propose launch");
}

gsta_status gsta_l1_loss(gsta_ctx* ctx, const float* image, const float* target, int64_t count,
                         float* dL_dimage, double* sums, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (count < 1) return fail(ctx, GSTA_ERR_INVALID, "count must be >= 1");
    if (!image || !target || !dL_dimage || !sums) return fail(ctx, GSTA_ERR_INVALID, "NULL pointer argument");
    PhaseTimer pt(ctx, GSTA_PHASE_LOSS, stream);
    launch_l1(image, target, count, dL_dimage, sums, ctx->loss_part, stream);
    return hip_check(ctx, hipGetLastError(), "l1 launch");
}

// ---- captured iterations and the autotuner ---------------------------------

struct gsta_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

gsta_status gsta_graph_begin(gsta_ctx* ctx, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (!stream) return fail(ctx, GSTA_ERR_INVALID, "the null stream cannot be captured; use a created stream");
    if (ctx->capturing) return fail(ctx, GSTA_ERR_INVALID, "a capture is already open on this context");
    if (ctx->profiling) return fail(ctx, GSTA_ERR_INVALID, "switch profiling off before capturing");
    gsta_status st = hip_check(ctx, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal),
                               "hipStreamBeginCapture");
    if (st == GSTA_OK) ctx->capturing = true;
    return st;
}

gsta_status gsta_graph_end(gsta_ctx* ctx, hipStream_t stream, gsta_graph** out) {
    if (!ctx || ctx->allocs.empty() || !out) return GSTA_ERR_INVALID;
    *out = nullptr;
    if (!ctx->capturing) return fail(ctx, GSTA_ERR_INVALID, "no capture is open on this context");
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    gsta_status st = hip_check(ctx, hipStreamEndCapture(stream, &g), "hipStreamEndCapture");
    if (st != GSTA_OK) return st;
    hipGraphExec_t e = nullptr;
    st = hip_check(ctx, hipGraphInstantiate(&e, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (st != GSTA_OK) {
        (void)hipGraphDestroy(g);
        return st;
    }
    gsta_graph* gr = new gsta_graph();
    gr->graph = g;
    gr->exec = e;
    *out = gr;
    return GSTA_OK;
}

gsta_status gsta_graph_launch(gsta_graph* graph, hipStream_t stream) {
    if (!graph || !graph->exec) return GSTA_ERR_INVALID;
    return hipGraphLaunch(graph->exec, stream) == hipSuccess ? GSTA_OK : GSTA_ERR_HIP;
}

void gsta_graph_destroy(gsta_graph* graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

gsta_status gsta_autotune(gsta_ctx* ctx, const gsta_params* g, const gsta_camera* cams, int32_t n_views,
                          const float* bg, float* image, float* dL_dimage, gsta_params* grad, const uint8_t* frozen,
                          int32_t repeats, gsta_tuning* out, hipStream_t stream) {
    if (!ctx || ctx->allocs.empty()) return GSTA_ERR_INVALID;
    if (ctx->capturing) return fail(ctx, GSTA_ERR_INVALID, "the autotuner synchronises: not while a graph is captured");
    if (repeats < 1 || repeats > 1000) return fail(ctx, GSTA_ERR_INVALID, "repeats must be in [1, 1000]");
    if (!image || !dL_dimage || !grad) return fail(ctx, GSTA_ERR_INVALID, "NULL scratch argument");
    const int fwd0 = ctx->fwd_waves, bwd0 = ctx->bwd_waves, var0 = ctx->bwd_variant;
    const uint32_t seg0 = ctx->seg_shift;
    const uint32_t prof0 = ctx->profiling;
    ctx->profiling = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    gsta_status st = hip_check(ctx, hipEventCreate(&e0), "hipEventCreate");
    if (st == GSTA_OK) st = hip_check(ctx, hipEventCreate(&e1), "hipEventCreate");
    auto restore = [&](gsta_status s) {
        ctx->fwd_waves = fwd0;
        ctx->bwd_waves = bwd0;
        ctx->bwd_blocks = ctx->cus * composite_bwd_blocks_per_cu(bwd0);
        ctx->bwd_variant = var0;
        ctx->seg_shift = seg0;
        ctx->profiling = prof0;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return s;
    };
    if (st != GSTA_OK) return restore(st);
    // ms per call of `fn` over `repeats` calls after one untimed call
    auto timed = [&](auto fn, float* ms) -> gsta_status {
        gsta_status s = fn();
        if (s != GSTA_OK) return s;
        if ((s = hip_check(ctx, hipEventRecord(e0, stream), "hipEventRecord")) != GSTA_OK) return s;
        for (int r = 0; r < repeats; ++r)
            if ((s = fn()) != GSTA_OK) return s;
        if ((s = hip_check(ctx, hipEventRecord(e1, stream), "hipEventRecord")) != GSTA_OK) return s;
        if ((s = hip_check(ctx, hipEventSynchronize(e1), "hipEventSynchronize")) != GSTA_OK) return s;
        float t = 0.f;
        if ((s = hip_check(ctx, hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime")) != GSTA_OK) return s;
        *ms = t / (float)repeats;
        return GSTA_OK;
    };
    auto forward = [&]() { return gsta_render_forward(ctx, g, cams, n_views, bg, image, 0, stream); };
    auto step = [&]() {
        gsta_status s = gsta_render_forward(ctx, g, cams, n_views, bg, image, 0, stream);
        if (s == GSTA_OK)
            s = gsta_render_backward(ctx, g, cams, n_views, bg, 0, dL_dimage, frozen, grad, nullptr, nullptr, 0.9f,
                                     nullptr, stream);
        return s;
    };
    gsta_tuning best{};
    int cands = 0;
    // forward launch shape first (it does not depend on the backward's)
    float best_f = 3.0e38f;
    const int fwd_c[4] = {0, 1, 2, 4};
    for (int f : fwd_c) {
        ctx->fwd_waves = f;
        float ms = 0.f;
        if ((st = timed(forward, &ms)) != GSTA_OK) return restore(st);
        ++cands;
        if (ms < best_f) {
            best_f = ms;
            best.fwd_waves = f;
            best.fwd_ms = ms;
        }
    }
    ctx->fwd_waves = best.fwd_waves;
    // then the backward: the per-pixel variant's waves x segment length and
    // the per-splat variant x segment length, timed as forward + backward
    // (the segment length also sets the forward's checkpoints)
    float best_s = 3.0e38f;
    const int bwd_c[4] = {1, 2, 4, 0};   // 0: the per-splat variant
    const uint32_t seg_c[4] = {6, 7, 8, 31};
    for (int b : bwd_c)
        for (uint32_t sh : seg_c) {
            ctx->bwd_variant = b == 0 ? 1 : 0;
            ctx->bwd_waves = b == 0 ? bwd0 : b;
            ctx->bwd_blocks = ctx->cus * composite_bwd_blocks_per_cu(ctx->bwd_waves);
            ctx->seg_shift = sh;
            float ms = 0.f;
            if ((st = timed(step, &ms)) != GSTA_OK) return restore(st);
            ++cands;
            if (ms < best_s) {
                best_s = ms;
                best.bwd_variant = ctx->bwd_variant;
                best.bwd_waves = ctx->bwd_waves;
                best.bwd_segment = sh >= 31 ? 0 : (1 << sh);
                best.step_ms = ms;
            }
        }
    best.candidates = cands;
    restore(GSTA_OK);
    ctx->fwd_waves = best.fwd_waves;
    ctx->bwd_waves = best.bwd_waves;
    ctx->bwd_variant = best.bwd_variant;
    ctx->bwd_blocks = ctx->cus * composite_bwd_blocks_per_cu(best.bwd_waves);
    ctx->seg_shift = best.bwd_segment == 0 ? 31u : (uint32_t)__builtin_ctz((unsigned)best.bwd_segment);
    if (out) *out = best;
    return GSTA_OK;
}

}  // extern "C"
