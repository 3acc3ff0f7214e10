// Tile compositing, forward and backward.
//
// Forward (Section 3.1, eq. 2): by default one 64-thread workgroup per 8x8
// quarter of a 16x16 tile (one pixel per lane); optionally one workgroup of
// W waves per tile, each thread owning 4/W pixels.  The tile's depth-ordered
// splats are staged in LDS in batches of one record per thread (a gather by
// gid) -- in quarter mode only those whose member extent reaches the
// quarter -- then every pixel walks the batch front to back.  The workgroup
// stops fetching batches once all its pixels have terminated
// (__syncthreads_count), and at every K-th list position it checkpoints its
// still-active pixels' state for the backward.  Colour is accumulated in
// double precision and kept per pixel for the backward.
//
// Backward (Section 3.2.4): W waves (default 2) per work item, one item per
// (tile, segment of K splats), starting from the state the forward
// checkpointed at the segment boundary.  Each pixel re-walks the
// segment up to its last member and recomputes the transmittance with the
// same instructions as the forward (shared eval_splat / next_T), so every
// membership and termination decision is identical.  The colour behind a
// member enters dL/dalpha only through its dot product with dL/dC, which
// each pixel carries as one double: the forward colour's (at a segment start
// minus the checkpointed prefix's), less w (dL/dC . c) per walked splat.
// Frozen splats still attenuate the pixels behind them but get no gradient
// work.  Per splat, a thread sums its pixels' 9 terms (dL/d opacity, colour,
// and the moments of dalpha alpha over dx, dy), each row of 16 lanes sums
// them with DPP operations, the rows' totals (4 per wave) are added through
// LDS in a fixed order every kChunk splats, the splat's conic turns the
// moments into its 2-D gradient, and the tile's total is written to the splat's own
// slot (its position in the depth-ordered expansion) -- no atomics, so the
// backward is deterministic.  The per-Gaussian sum over tiles happens in the
// preprocess backward, in a fixed order too.
#include "gsta_internal.h"

namespace gsta {
namespace {

// The row totals of nine values at once, transposing as it sums: at each of
// the four exchanges (lane ^ 1, lane ^ 2 within quads, then the row rotated
// by 4 and by 8, whose partners share the lower lane bits) a lane keeps the
// half of its values that its bit of the lane index selects and adds its
// partner's copy of them, so the pairs of values halve each time: 13 + 7 + 4
// + 2 adds and selects instead of 36 adds.  Lane l of a row ends with the
// row total of value l & 7 (out) and of value 8 (out8).
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ float keep_add(float a, float b, bool hi) {
    const float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp_row<CTRL>(send);
}
__device__ __forceinline__ void row_sum9(const float (&g)[9], int lane, float& out, float& out8) {
    const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0, b2 = (lane & 4) != 0;
    const float p0 = keep_add<0xB1>(g[0], g[1], b0), p1 = keep_add<0xB1>(g[2], g[3], b0);
    const float p2 = keep_add<0xB1>(g[4], g[5], b0), p3 = keep_add<0xB1>(g[6], g[7], b0);
    float v8 = g[8] + dpp_row<0xB1>(g[8]);
    const float r0 = keep_add<0x4E>(p0, p1, b1), r1 = keep_add<0x4E>(p2, p3, b1);
    v8 += dpp_row<0x4E>(v8);
    float s0 = keep_add<0x124>(r0, r1, b2);   // row_ror:4
    v8 += dpp_row<0x124>(v8);
    s0 += dpp_row<0x128>(s0);                 // row_ror:8
    v8 += dpp_row<0x128>(v8);
    out = s0;
    out8 = v8;
}

// One splat record as staged in LDS: mean + scaled conic (A, B), scaled
// conic C + opacity, colour.
struct Rec {
    float4 g;    // u, v, A, B (conic scaled by kConicScaleAC, kConicScaleB)
    float4 co;   // C, opacity, half-extent x, half-extent y
    float4 c;    // r, g, b
};

__device__ __forceinline__ Rec fetch_rec(const float4* __restrict__ geo, const float4* __restrict__ col,
                                         const float4* __restrict__ rgbv, int64_t vs, uint32_t gid) {
    Rec r;
    r.g = geo[vs + gid];
    r.co = col[vs + gid];
    r.c = rgbv[vs + gid];
    return r;
}

// Pixel p of thread tid.  Every 64-pixel group (the unit of the checkpoints)
// is an 8x8 quarter of the tile, lane l at (l % 8, l / 8) in it.  Tile mode:
// 4/W pixels per thread, group wave + p W.  Quadrant mode (one wave per
// quarter, blockIdx.x = 4 * tile + quarter): one pixel per lane.
template <int W, bool QUAD>
__device__ __forceinline__ void pixel_of(int tid, int p, int quarter, int tx0, int ty0, int& px, int& py) {
    const int lane = tid & 63;
    const int g = QUAD ? quarter : (tid >> 6) + p * W;
    px = tx0 + (g & 1) * 8 + (lane & 7);
    py = ty0 + (g >> 1) * 8 + (lane >> 3);
}

// Pool slots a tile-mode workgroup reserves per batch of B list positions for
// its segment boundaries: one per boundary and 64-pixel group.
template <int B>
__device__ __forceinline__ uint32_t batch_slots(uint32_t shift) {
    return (uint32_t)kCkptGroups * ((uint32_t)(B - 1) / (1u << shift) + 1u);
}

// Quadrant mode (batches of 64): a quarter reserves its slots per block of
// S = max(256, K) list positions, S / K of them, one batch ahead.
__device__ __forceinline__ uint32_t quad_block(uint32_t shift) { return max(256u, 1u << shift); }

// Whether the batch at list offset b0 (a multiple of B) of a list of len
// positions holds a segment boundary (a positive multiple of K).
template <int B>
__device__ __forceinline__ bool batch_has_boundary(uint32_t b0, uint32_t len, uint32_t shift) {
    const uint32_t K = 1u << shift;
    const uint32_t first = b0 == 0u ? K : (b0 + K - 1u) / K * K;
    return first < min(b0 + (uint32_t)B, len);
}

// Forward state at a segment boundary (global list position gpos, at offset k
// of its batch), for the pixel groups of this thread that still have active
// pixels.  Called with the lanes that are still walking; done lanes are
// inactive.  The group's pool slot is fixed by the batch's block of slots
// (ckbase, reserved by the workgroup a batch ahead): no counter on the walk.
// sub: the boundary's index within the reserved block (tile mode: within
// the batch; quadrant mode: within the S-position block).
template <int W, int P, int B, bool QUAD>
__device__ __forceinline__ void fwd_checkpoint(const SegCkpt& sc, uint32_t gpos, uint32_t sub, uint32_t ckbase,
                                               int tid, int quarter, const bool* done, const float* T,
                                               const double (*C)[3]) {
    const int lane = tid & 63, wid = tid >> 6;
    const size_t bucket = (size_t)(gpos >> sc.shift);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t m = __ballot(!done[p]);
        if (m == 0ull) continue;
        const int first = __builtin_ctzll(m);
        const int g = QUAD ? quarter : wid + p * W;   // 64-pixel group of pixel p
        const uint64_t slot64 = QUAD ? (uint64_t)ckbase + sub
                                     : (uint64_t)ckbase + (uint64_t)kCkptGroups * sub + (uint64_t)g;
        const bool ok = ckbase != kNoSlot && slot64 < (uint64_t)sc.pool_cap;
        const uint32_t slot = (uint32_t)slot64;
        if (lane == first) {
            sc.idx[bucket * kCkptGroups + g] = ok ? slot : kNoSlot;
            if (!ok) atomicOr(sc.flags + 3, 1u);
        }
        if (ok && !done[p]) {
            double* d = sc.pool + (size_t)slot * 256;
            d[lane] = (double)T[p];
            d[64 + lane] = C[p][0];
            d[128 + lane] = C[p][1];
            d[192 + lane] = C[p][2];
        }
    }
}

// Records per step of the forward walk (a multiple of which every chunk
// length is).
constexpr int kStep = 4;

// Whether a splat can be a member of a pixel of the box [x0, x1] x [y0, y1]
// (pixel coordinates).  A member has power2 >= max(kPower2Floor,
// -log2(255 o)) (the 3-sigma floor and alpha >= 1/255), i.e. the positive
// form Q(d) = -power2(d) at most minus that bound; Q's minimum over the box is
// 0 if the centre is inside, else on an edge, where it is the clamped
// stationary point of a parabola.  The margin (0.1 in log2 units, plus a
// relative 1e-4 of the form's size over the box) covers the float rounding of
// this test and of the walk's own evaluation, so a false answer is certain.
__device__ __forceinline__ bool splat_reaches_box(float u, float v, float A, float B, float C, float o, float x0,
                                                  float x1, float y0, float y1) {
    const float a = -A, b = -B, c = -C;   // Q = a dx^2 + b dx dy + c dy^2, d = (u, v) - pixel
    const float dx0 = u - x1, dx1 = u - x0, dy0 = v - y1, dy1 = v - y0;
    float qmin = 0.f;
    if (!(dx0 <= 0.f && dx1 >= 0.f && dy0 <= 0.f && dy1 >= 0.f)) {
        const float ry = 0.5f * b / c, rx = 0.5f * b / a;
        const float ya = fminf(fmaxf(-ry * dx0, dy0), dy1), yb = fminf(fmaxf(-ry * dx1, dy0), dy1);
        const float xa = fminf(fmaxf(-rx * dy0, dx0), dx1), xb = fminf(fmaxf(-rx * dy1, dx0), dx1);
        const float qa = (a * dx0 + b * ya) * dx0 + c * ya * ya, qb = (a * dx1 + b * yb) * dx1 + c * yb * yb;
        const float qc = (c * dy0 + b * xa) * dy0 + a * xa * xa, qd = (c * dy1 + b * xb) * dy1 + a * xb * xb;
        qmin = fminf(fminf(qa, qb), fminf(qc, qd));
    }
    const float thr = fmaxf(kPower2Floor, -log2f(255.0f * o));
    const float dxm = fmaxf(fabsf(dx0), fabsf(dx1)), dym = fmaxf(fabsf(dy0), fabsf(dy1));
    const float size = a * dxm * dxm + c * dym * dym + fabsf(b) * dxm * dym;
    return qmin <= -thr + 0.1f + 1e-4f * size;
}

template <int W, bool QUAD, bool CNT>
__global__ __launch_bounds__(64 * W, QUAD ? 5 : 1) void k_composite_fwd(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ gsort,
    const float4* __restrict__ geo, const float4* __restrict__ col, const float4* __restrict__ rgbv,
    int64_t stride, CamArray cams, float bg0, float bg1, float bg2, float* __restrict__ image,
    float* __restrict__ T_final, uint32_t* __restrict__ last_out, double* __restrict__ cfg, SegCkpt sc,
    unsigned long long* __restrict__ pairs, FusedL1 l1) {
    constexpr int NT = 64 * W, P = QUAD ? 1 : 4 / W, B = NT;
    // kStep - 1 slots past the batch hold zero-opacity records, which a
    // step reaching past the last staged record evaluates as non-members
    __shared__ float4 s_geo[B + kStep - 1];
    __shared__ float4 s_co[B + kStep - 1];
    __shared__ double s_rgb[3][B + kStep - 1];   // colours, converted once when staged
    __shared__ unsigned int s_pairs;
    __shared__ uint32_t s_last;
    __shared__ uint32_t s_ckbase;      // pool slots of the current batch's segment boundaries
    __shared__ uint32_t s_pos[QUAD ? B + kStep - 1 : 1];  // quadrant mode: list position + 1 of each kept record
    const int v = blockIdx.y;
    const DevCam& cm = cams.c[v];
    const int tiles = cm.ntx * cm.nty;
    const int tile = QUAD ? (int)(blockIdx.x >> 2) : (int)blockIdx.x;
    const int quarter = (int)(blockIdx.x & 3);
    const int tid = threadIdx.x;
    const int tx0 = (tile % cm.ntx) * kTile, ty0 = (tile / cm.ntx) * kTile;
    const uint2 rg = ranges[(int64_t)v * tiles + tile];
    const int64_t vs = (int64_t)v * stride;

    float fpx[P], fpy[P], T[P];
    double C[P][3];
    uint32_t last[P];
    bool done[P], inside[P];
    bool alldone = true;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        int px, py;
        pixel_of<W, QUAD>(tid, p, quarter, tx0, ty0, px, py);
        inside[p] = px < cm.width && py < cm.height;
        fpx[p] = (float)px;
        fpy[p] = (float)py;
        T[p] = 1.0f;
        C[p][0] = C[p][1] = C[p][2] = 0.0;
        last[p] = 0;
        done[p] = !inside[p];
        alldone = alldone && done[p];
    }
    uint32_t evals = 0, witer = 0;
    if (tid == 0) {
        s_pairs = 0;
        s_last = 0;
    }
    if (tid < kStep - 1) {
        s_geo[B + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
        s_co[B + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
        s_rgb[0][B + tid] = s_rgb[1][B + tid] = s_rgb[2][B + tid] = 0.0;
    }
    // checkpoints at list positions that are multiples of K (none in quadrant mode)
    const uint32_t kmask = sc.shift >= 31u ? 0xFFFFFFFFu : ((1u << sc.shift) - 1u);
    const bool ckpt = kmask != 0xFFFFFFFFu;
    const uint32_t len = rg.y - rg.x;
    // The first batch's boundary slots are the tile's own; thread 0 reserves
    // each later batch's block from the counter one batch ahead, so the
    // counter's latency stays off the walk (a walk that ends early leaves one
    // reserved block unused).
    uint32_t ck_next = kNoSlot, ck_cur = kNoSlot;
    if (ckpt && tid == 0) {
        if (QUAD)   // the first S positions: the quarter's part of the tile's own block
            ck_next = (uint32_t)(v * tiles + tile) * kBatchSlotsMax +
                      (uint32_t)quarter * (quad_block(sc.shift) >> sc.shift);
        else if (batch_has_boundary<B>(0u, len, sc.shift))
            ck_next = (uint32_t)(v * tiles + tile) * kBatchSlotsMax;
    }

    // Two-stage software pipeline: while a batch is composited, the records
    // of the next batch and the ids of the one after are in flight.  The
    // loads are unconditional, from positions inside the list (a lane past
    // its end reads the last entry, which the staging ignores): loads under
    // a lane mask would make the compiler wait for them before the walk.
    Rec cur;
    uint32_t gid_nxt = 0;
    if (rg.y > rg.x) {   // uniform
        const uint32_t j = rg.x + tid, jl = rg.y - 1u;
        cur = fetch_rec(geo, col, rgbv, vs, gsort[min(j, jl)]);
        gid_nxt = gsort[min(j + B, jl)];
    }
    // quadrant mode: the quarter's pixel box
    const float qx0 = (float)(tx0 + (quarter & 1) * 8), qy0 = (float)(ty0 + (quarter >> 1) * 8);
    for (uint32_t base = rg.x; base < rg.y; base += B) {
        if (__syncthreads_count(!alldone) == 0) break;
        int cnt;
        if (QUAD) {
            // Keep only the splats whose member extent (col.z, col.w: half-widths
            // beyond which no pixel can be a member) and member ellipse reach
            // the quarter: the others are non-members of every pixel here and
            // would leave T and the colour as they are.  The kept records stay
            // in list order.
            const bool hit = base + tid < rg.y && cur.g.x + cur.co.z >= qx0 && cur.g.x - cur.co.z <= qx0 + 7.0f &&
                             cur.g.y + cur.co.w >= qy0 && cur.g.y - cur.co.w <= qy0 + 7.0f &&
                             splat_reaches_box(cur.g.x, cur.g.y, cur.g.z, cur.g.w, cur.co.x, cur.co.y, qx0,
                                               qx0 + 7.0f, qy0, qy0 + 7.0f);
            const uint64_t hm = __ballot(hit);
            const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(hm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
            cnt = __popcll(hm);
            if (hit) {
                s_geo[r] = cur.g;
                s_co[r] = cur.co;
                s_rgb[0][r] = (double)cur.c.x;
                s_rgb[1][r] = (double)cur.c.y;
                s_rgb[2][r] = (double)cur.c.z;
                s_pos[r] = base - rg.x + (uint32_t)tid + 1u;
            }
            if (tid >= cnt && tid < cnt + kStep - 1) {   // zero-opacity records after the kept ones
                s_geo[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                s_co[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                s_rgb[0][tid] = s_rgb[1][tid] = s_rgb[2][tid] = 0.0;
            }
        } else {
            cnt = (int)min((uint32_t)B, rg.y - base);
            if (base + tid < rg.y) {
                s_geo[tid] = cur.g;
                s_co[tid] = cur.co;
                s_rgb[0][tid] = (double)cur.c.x;
                s_rgb[1][tid] = (double)cur.c.y;
                s_rgb[2][tid] = (double)cur.c.z;
            } else if (base + tid < rg.y + (uint32_t)(kStep - 1)) {
                // zero-opacity records after the list's last splat: a step that
                // reaches past the end evaluates them and they are never members
                s_geo[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                s_co[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
                s_rgb[0][tid] = s_rgb[1][tid] = s_rgb[2][tid] = 0.0;
            }
        }
        if (ckpt && tid == 0) {
            const uint32_t b1 = base - rg.x + (uint32_t)B;
            if (QUAD) {
                const uint32_t S = quad_block(sc.shift);
                if ((base - rg.x) % S == 0u) ck_cur = ck_next;          // a new block of S positions
                if (b1 % S == 0u)                                      // its last batch: reserve the next
                    ck_next = b1 < len ? sc.first_slots + atomicAdd(sc.ctr, S >> sc.shift) : kNoSlot;
                s_ckbase = ck_cur;
            } else {
                s_ckbase = ck_next;
                ck_next = batch_has_boundary<B>(b1, len, sc.shift)
                              ? sc.first_slots + atomicAdd(sc.ctr, batch_slots<B>(sc.shift)) : kNoSlot;
            }
        }
        __syncthreads();
        {
            const uint32_t jn = base + B + tid;
            cur = fetch_rec(geo, col, rgbv, vs, gid_nxt);
            gid_nxt = gsort[min(jn + B, rg.y - 1u)];
        }
        // Each lane leaves the walk as soon as its pixels are done.  kStep
        // records per step, all evaluated unconditionally so that their
        // exponentials and LDS reads overlap; the transmittance then advances
        // through them in list order with selects (the same operations on the
        // same values as one splat at a time), and the colour takes them in
        // the same order.
        // Checkpoints fall on chunk starts: chunks of K splats (of the batch
        // when K is longer), so the steps inside a chunk test nothing.
        // (Quadrant mode: one chunk per batch, the batch start checkpointed
        // even when no record of the batch was kept.)
        const int L = ckpt ? min(B, 1 << sc.shift) : B;
        for (int kc = 0; (QUAD ? kc == 0 : kc < cnt) && !alldone; kc += L) {
            {
                const uint32_t pos0 = base - rg.x + (uint32_t)kc;
                if (ckpt && pos0 != 0u && (pos0 & kmask) == 0u)
                    fwd_checkpoint<W, P, B, QUAD>(sc, base + (uint32_t)kc,
                                                  QUAD ? (pos0 % quad_block(sc.shift)) >> sc.shift
                                                       : (uint32_t)kc >> sc.shift,
                                                  s_ckbase, tid, quarter, done, T, C);
            }
            const int kend = min(cnt, kc + L);
            for (int k = kc; k < kend && !alldone; k += kStep) {
                // offsets k .. k + kStep - 1 (past cnt: the zero-opacity records)
                float4 g[kStep];
                double rgb[kStep][3];
                float2 o[kStep];
                uint32_t pos1[kStep];    // list positions + 1 (the `last` a contributing record sets)
#pragma unroll
                for (int i = 0; i < kStep; ++i) {
                    g[i] = s_geo[k + i];
                    const float4 t = s_co[k + i];
                    o[i] = make_float2(t.x, t.y);
                    rgb[i][0] = s_rgb[0][k + i];
                    rgb[i][1] = s_rgb[1][k + i];
                    rgb[i][2] = s_rgb[2][k + i];
                    pos1[i] = QUAD ? s_pos[k + i] : base - rg.x + (uint32_t)(k + i) + 1u;
                }
                const int nreal = min(kStep, cnt - k);   // (counted by the counting variant only)
                bool all = true;
                if (CNT) witer += (uint32_t)nreal;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (!done[p]) {
                        SplatEval e[kStep];
                        bool mem[kStep];
#pragma unroll
                        for (int i = 0; i < kStep; ++i) {
                            eval_splat(g[i].x, g[i].y, g[i].z, g[i].w, o[i].x, o[i].y, fpx[p], fpy[p], e[i]);
                            mem[i] = e[i].power2 >= kPower2Floor && e[i].alpha >= kAlphaMin;
                        }
                        // Transmittance after each record: a non-member's factor is
                        // exactly 1, so Tp[i + 1] is the one-at-a-time walk's T
                        // after record i (the same product T (1 - alpha)) as long as
                        // that walk has not stopped.  T never rises, so the records
                        // before the first Tp[i + 1] < kTMin are the ones the walk
                        // takes and it stops at that record: one multiply per record
                        // is the only chain.
                        float om[kStep];
#pragma unroll
                        for (int i = 0; i < kStep; ++i) om[i] = mem[i] ? 1.0f - e[i].alpha : 1.0f;
                        float Tp[kStep + 1];
                        Tp[0] = T[p];
#pragma unroll
                        for (int i = 0; i < kStep; ++i) Tp[i + 1] = Tp[i] * om[i];
                        float Tc = Tp[0];
#pragma unroll
                        for (int i = 0; i < kStep; ++i) {
                            if (CNT) evals += (Tp[i] >= kTMin && i < nreal) ? 1u : 0u;   // a one-at-a-time walk's pairs
                            const bool ok = Tp[i + 1] >= kTMin;
                            const bool c = mem[i] && ok;                    // contributes
                            // the weight selected as float bits, then widened once
                            const float wf = __builtin_bit_cast(
                                float, c ? __builtin_bit_cast(uint32_t, e[i].alpha * Tp[i]) : 0u);
                            const double wd = (double)wf;
                            // a zero weight leaves the colour unchanged
                            C[p][0] = fma(rgb[i][0], wd, C[p][0]);
                            C[p][1] = fma(rgb[i][1], wd, C[p][1]);
                            C[p][2] = fma(rgb[i][2], wd, C[p][2]);
                            last[p] = c ? pos1[i] : last[p];
                            Tc = ok ? Tp[i + 1] : Tc;
                        }
                        const bool stop = Tp[kStep] < kTMin;
                        T[p] = Tc;
                        done[p] = stop;
                    }
                    all = all && done[p];
                }
                alldone = all;
            }
        }
    }
    if (CNT) {
        __syncthreads();
        if (evals) atomicAdd(&s_pairs, evals);
        __syncthreads();
        if (tid == 0 && s_pairs) atomicAdd(pairs + 0, (unsigned long long)s_pairs);
        // the wave runs as long as its longest lane
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) witer = max(witer, (uint32_t)__shfl_xor((int)witer, off, 64));
        if ((tid & 63) == 0 && witer) atomicAdd(pairs + 2, (unsigned long long)witer);
    }
    {
        uint32_t ml = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) ml = max(ml, last[p]);
        __syncthreads();
        if (ml) atomicMax(&s_last, ml);
        __syncthreads();
        if (tid == 0 && s_last) atomicMax(sc.tile_last + (int64_t)v * tiles + tile, s_last);
    }
    const int64_t HW = (int64_t)cm.width * cm.height;
    double la = 0.0, lb = 0.0;     // fused L1: sum |d| and sum of squared clamped errors
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!inside[p]) continue;
        int px, py;
        pixel_of<W, QUAD>(tid, p, quarter, tx0, ty0, px, py);
        const int64_t o = (int64_t)py * cm.width + px;
        float* img = image + (int64_t)v * 3 * HW + o;
        const float c3[3] = {(float)(C[p][0] + (double)(T[p] * bg0)), (float)(C[p][1] + (double)(T[p] * bg1)),
                             (float)(C[p][2] + (double)(T[p] * bg2))};
        img[0] = c3[0];
        img[HW] = c3[1];
        img[2 * HW] = c3[2];
        T_final[(int64_t)v * HW + o] = T[p];
        last_out[(int64_t)v * HW + o] = last[p];
        double* cf = cfg + (int64_t)v * 3 * HW + o;
        cf[0] = C[p][0];
        cf[HW] = C[p][1];
        cf[2 * HW] = C[p][2];
        if (l1.target) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const int64_t i = (int64_t)v * 3 * HW + ch * HW + o;
                const float t = l1.target[i];
                const float d = c3[ch] - t;
                l1.dL[i] = (d > 0.f) ? l1.inv : ((d < 0.f) ? -l1.inv : 0.f);
                la += (double)fabsf(d);
                const double e = (double)fminf(fmaxf(c3[ch], 0.f), 1.f) - (double)t;
                lb += e * e;
            }
        }
    }
    if (l1.target) {   // uniform: every thread takes part
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            la += __shfl_xor(la, off, 64);
            lb += __shfl_xor(lb, off, 64);
        }
        __shared__ double s_l1[W][2];
        if ((tid & 63) == 0) {
            s_l1[tid >> 6][0] = la;
            s_l1[tid >> 6][1] = lb;
        }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                a += s_l1[w][0];
                b += s_l1[w][1];
            }
            l1.part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(a, b);
        }
    }
}

// Splats per partial-sum flush in the backward.  32 rather than 64: the
// smaller LDS buffer of row totals lets 8 instead of 6 workgroups share a CU.
constexpr int kChunk = 32;

// Items per tile: ceil(tile_last / K) (one if segments are off), scanned by
// one workgroup of 1024 threads into item_off[0..nt] (item_off[nt] = total),
// two tiles per thread and round; item_tile[i] names the tile of item i.
// With a fused L1 loss (sums set) it also adds the forward's nparts
// per-workgroup loss sums in a fixed order (thread t: parts t, t + 1024, ...;
// the first kSegPre of them loaded before the scan).
constexpr int kSegPre = 8;
__global__ __launch_bounds__(1024) void k_seg_items(const uint32_t* __restrict__ tile_last, int nt, uint32_t shift,
                                                    uint32_t* __restrict__ item_off, uint32_t* __restrict__ item_tile,
                                                    uint32_t item_cap, const double2* __restrict__ lpart,
                                                    int nparts, double* __restrict__ sums) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double2 pre[kSegPre];
#pragma unroll
    for (int k = 0; k < kSegPre; ++k) {
        const int i = (int)threadIdx.x + 1024 * k;
        pre[k] = (sums && i < nparts) ? lpart[i] : make_double2(0.0, 0.0);
    }
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nt; base += 2048) {
        const int j0 = base + 2 * (int)threadIdx.x;
        uint32_t x[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            x[h] = 0;
            if (j0 + h < nt) {
                const uint32_t l = tile_last[j0 + h];
                x[h] = shift >= 31u ? (l ? 1u : 0u) : ((l + (1u << shift) - 1u) >> shift);
            }
        }
        const uint32_t xs = x[0] + x[1];
        uint32_t incl = xs;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint32_t wbase = s_carry;
        for (int k = 0; k < w; ++k) wbase += s_w[k];
        uint32_t off = wbase + incl - xs;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (j0 + h < nt) {
                item_off[j0 + h] = off;
                for (uint32_t i = 0; i < x[h]; ++i)
                    if (off + i < item_cap) item_tile[off + i] = (uint32_t)(j0 + h);
                off += x[h];
            }
        }
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = wbase + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) item_off[nt] = s_carry;
    if (sums) {   // uniform
        __shared__ double s_a[16], s_b[16];
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int k = 0; k < kSegPre; ++k) {
            a += pre[k].x;
            b += pre[k].y;
        }
#pragma unroll 4
        for (int i = (int)threadIdx.x + 1024 * kSegPre; i < nparts; i += 1024) {
            a += lpart[i].x;
            b += lpart[i].y;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
        if (lane == 0) {
            s_a[w] = a;
            s_b[w] = b;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0;
            for (int k = 0; k < 16; ++k) {
                ta += s_a[k];
                tb += s_b[k];
            }
            sums[0] = ta;
            sums[1] = tb;
        }
    }
}

// Two waves per tile (the default): at most 96 VGPRs, five waves per SIMD, so
// that nine of these workgroups (the LDS bound) fit a CU instead of eight.
template <int W, bool CNT>
__global__ __launch_bounds__(64 * W, W == 2 ? 5 : 1) void k_composite_bwd(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids, const uint32_t* __restrict__ gsort,
    const float4* __restrict__ geo, const float4* __restrict__ col, const float4* __restrict__ rgbv,
    int64_t stride, const uint8_t* __restrict__ frozen, CamArray cams, int nv, float bg0, float bg1, float bg2,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last_in, const double* __restrict__ cfg,
    const float* __restrict__ dL_dimage, float* __restrict__ partials, SegCkpt sc,
    unsigned long long* __restrict__ pairs) {
    constexpr int NT = 64 * W, P = 4 / W, B = NT;
    __shared__ float4 s_geo[B];
    __shared__ float4 s_co[B];
    __shared__ float4 s_rgb[B];
    __shared__ uint32_t s_idx[B];
    __shared__ uint32_t s_frz[B];
    __shared__ uint32_t s_pos[B];      // list position (from the tile's start) of each kept record
    __shared__ uint32_t s_wkept[W];
    // row totals; the chunk dimension is padded to kChunk + 1 words so that
    // the 36 words one write of a wave fills (rows 4 wid .. +3, values 0-8)
    // fall into nearly distinct LDS banks
    __shared__ float s_part[4 * W][9][kChunk + 1];
    __shared__ unsigned int s_pairs, s_grad;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tiles = cams.c[0].ntx * cams.c[0].nty;
    const int nt = nv * tiles;
    const uint32_t n_items = min(sc.item_off[nt], sc.item_cap);
    const bool seg = sc.shift < 31u;
    const uint32_t gen = *sc.gen;
    uint32_t evals = 0, witer = 0, wred = 0, ngrad = 0;
    if (tid == 0) {
        s_pairs = 0;
        s_grad = 0;
    }
    // row totals start at zero; only steps with gradient work write theirs,
    // and each flush clears what it has read
    for (int i = tid; i < 4 * W * 9 * (kChunk + 1); i += NT) (&s_part[0][0][0])[i] = 0.f;
    __syncthreads();

    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int gt = (int)sc.item_tile[item];     // the item's tile
        const uint32_t sgi = item - sc.item_off[gt];
        const int v = gt / tiles, tile = gt - v * tiles;
        const DevCam& cm = cams.c[v];
        const int tx0 = (tile % cm.ntx) * kTile, ty0 = (tile / cm.ntx) * kTile;
        const uint2 rg = ranges[gt];
        const int64_t vs = (int64_t)v * stride;
        const int64_t HW = (int64_t)cm.width * cm.height;
        const uint32_t tl = sc.tile_last[gt];
        const uint32_t p0 = seg ? (sgi << sc.shift) : 0u;                       // first position of the item
        const uint32_t p1 = seg ? min(tl, (sgi + 1u) << sc.shift) : tl;          // one past its last

        float fpx[P], fpy[P], dC[P][3], T[P];
        // Db = sum over channels of dL/dC (FB - A): FB the pixel's final
        // colour, background term included (the forward's double colour +
        // T_final bg), A the colour of the splats walked so far, so FB - A is
        // what lies behind the current splat.  A splat of colour c and weight
        // w takes w (dL/dC . c) off it.  dCd: dL/dC in double.
        double Db[P], dCd[P][3];
        uint32_t last[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            int px, py;
            pixel_of<W, false>(tid, p, 0, tx0, ty0, px, py);
            fpx[p] = (float)px;
            fpy[p] = (float)py;
            T[p] = 1.0f;
            dC[p][0] = dC[p][1] = dC[p][2] = 0.f;
            dCd[p][0] = dCd[p][1] = dCd[p][2] = 0.0;
            Db[p] = 0.0;
            last[p] = 0;
            if (px < cm.width && py < cm.height) {
                const int64_t o = (int64_t)py * cm.width + px;
                last[p] = last_in[(int64_t)v * HW + o];
                if (last[p] > p0) {
                    const float* dl = dL_dimage + (int64_t)v * 3 * HW + o;
                    dC[p][0] = dl[0];
                    dC[p][1] = dl[HW];
                    dC[p][2] = dl[2 * HW];
                    dCd[p][0] = (double)dC[p][0];
                    dCd[p][1] = (double)dC[p][1];
                    dCd[p][2] = (double)dC[p][2];
                    const float tf = T_final[(int64_t)v * HW + o];
                    const double* cf = cfg + (int64_t)v * 3 * HW + o;
                    Db[p] = dCd[p][0] * (cf[0] + (double)(tf * bg0)) + dCd[p][1] * (cf[HW] + (double)(tf * bg1)) +
                            dCd[p][2] * (cf[2 * HW] + (double)(tf * bg2));
                }
            }
        }
        if (p0 != 0u) {
            // resume from the forward's state at the segment boundary
            const size_t bucket = (size_t)((rg.x + p0) >> sc.shift);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (last[p] <= p0) continue;
                const uint32_t slot = sc.idx[bucket * kCkptGroups + wid + p * W];
                if (slot >= sc.pool_cap) {       // the forward ran out of slots (flagged)
                    last[p] = 0;
                    continue;
                }
                const double* d = sc.pool + (size_t)slot * 256;
                T[p] = (float)d[lane];
                Db[p] -= dCd[p][0] * d[64 + lane] + dCd[p][1] * d[128 + lane] + dCd[p][2] * d[192 + lane];
            }
        }
        const uint32_t beg = rg.x + p0, end = rg.x + p1;

        // Two-stage software pipeline as in the forward.
        Rec cur;
        uint32_t idx_cur = 0, frz_cur = 0, idx_nxt = 0, gid_nxt = 0;
        {
            const uint32_t j = beg + tid;
            if (j < end) {
                idx_cur = ids[j];
                const uint32_t gid = gsort[j];
                cur = fetch_rec(geo, col, rgbv, vs, gid);
                frz_cur = frozen ? (uint32_t)frozen[gid] : 0u;
            }
            if (j + B < end) {
                idx_nxt = ids[j + B];
                gid_nxt = gsort[j + B];
            }
        }
        for (uint32_t base = beg; base < end; base += B) {
            // Keep only the splats whose member ellipse reaches the tile (the
            // others are non-members of all its pixels: they would change
            // nothing and get no gradient), in list order.
            const bool hit = base + tid < end && splat_reaches_box(cur.g.x, cur.g.y, cur.g.z, cur.g.w, cur.co.x,
                                                                   cur.co.y, (float)tx0, (float)(tx0 + kTile - 1),
                                                                   (float)ty0, (float)(ty0 + kTile - 1));
            const uint64_t hm = __ballot(hit);
            __syncthreads();
            if (lane == 0) s_wkept[wid] = (uint32_t)__popcll(hm);
            __syncthreads();
            int cnt = 0, woff = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                woff += w < wid ? (int)s_wkept[w] : 0;
                cnt += (int)s_wkept[w];
            }
            if (hit) {
                const int r = woff + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(hm >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
                s_idx[r] = idx_cur;
                s_geo[r] = cur.g;
                s_co[r] = cur.co;
                s_rgb[r] = cur.c;
                s_frz[r] = frz_cur;
                s_pos[r] = base - rg.x + (uint32_t)tid;
            }
            __syncthreads();
            {
                const uint32_t jn = base + B + tid;
                if (jn < end) {
                    idx_cur = idx_nxt;
                    cur = fetch_rec(geo, col, rgbv, vs, gid_nxt);
                    frz_cur = frozen ? (uint32_t)frozen[gid_nxt] : 0u;
                }
                if (jn + B < end) {
                    idx_nxt = ids[jn + B];
                    gid_nxt = gsort[jn + B];
                }
            }
            for (int c0 = 0; c0 < cnt; c0 += kChunk) {
                const int c1 = min(cnt, c0 + kChunk);
                for (int k = c0; k < c1; ++k) {
                    const uint32_t pos = s_pos[k];
                    const float4 g = s_geo[k];
                    const float2 co = make_float2(s_co[k].x, s_co[k].y);
                    // uniform over the wave: a scalar branch
                    const bool frz = __builtin_amdgcn_readfirstlane(s_frz[k]) != 0u;
                    if (CNT) witer += 1u;
                    SplatEval e[P];
                    bool mem[P];
                    bool any = false;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const bool act = pos < last[p];
                        if (CNT) evals += act ? 1u : 0u;
                        eval_power(g.x, g.y, g.z, g.w, co.x, fpx[p], fpy[p], e[p]);
                        mem[p] = act && (e[p].power2 >= kPower2Floor);
                        any = any || mem[p];
                    }
                    if (__ballot(any) != 0ull) {
                        // Straight-line over the pixels: a non-member gets weight
                        // 0 and a zero dalpha, so it adds exact zeros and keeps
                        // its T and accumulated colour, without divergent branches.
                        const float4 c = s_rgb[k];
                        const double cx = (double)c.x, cy = (double)c.y, cz = (double)c.z;
                        bool contrib = false;
                        float g9[9];
#pragma unroll
                        for (int q = 0; q < 9; ++q) g9[q] = 0.f;
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            eval_alpha(co.y, e[p]);
                            const bool m = mem[p] && (e[p].alpha >= kAlphaMin);
                            const float w = m ? e[p].alpha * T[p] : 0.f;
                            const double wd = (double)w;
                            const double dcc = fma(dCd[p][2], cz, fma(dCd[p][1], cy, dCd[p][0] * cx));
                            Db[p] = fma(-wd, dcc, Db[p]);
                            if (!frz) {   // uniform
                                contrib = contrib || m;
                                if (CNT) ngrad += m ? 1u : 0u;
                                const float inv1m = __builtin_amdgcn_rcpf(1.0f - e[p].alpha);
                                // sum over channels of dL/dC (c T - behind / (1 - alpha))
                                const float da = fmaf(T[p], (float)dcc, -((float)Db[p] * inv1m));
                                g9[6] += dC[p][0] * w;
                                g9[7] += dC[p][1] * w;
                                g9[8] += dC[p][2] * w;
                                // alpha clamped at kAlphaMax: no gradient to opacity or power
                                const float dalpha = (m && e[p].oG <= kAlphaMax) ? da : 0.f;
                                // d power / d(u, v) = -(a dx + b dy, b dx + c dy)
                                //                   = ln 2 (2 A dx + B dy, B dx + 2 C dy)
                                // The splat's conic is the same for all its pixels: the
                                // pixels accumulate the moments of dpow = dalpha alpha,
                                // sum dpow (dx, dy, dx^2, dx dy, dy^2), and the flush
                                // forms the 2-D gradient from them.
                                const float dpow = dalpha * e[p].alpha;
                                g9[5] += dalpha * e[p].G;
                                const float tx = dpow * e[p].dx, ty = dpow * e[p].dy;
                                g9[0] += tx;
                                g9[1] += ty;
                                g9[2] = fmaf(tx, e[p].dx, g9[2]);
                                g9[3] = fmaf(tx, e[p].dy, g9[3]);
                                g9[4] = fmaf(ty, e[p].dy, g9[4]);
                            }
                            T[p] = m ? next_T(T[p], e[p].alpha) : T[p];
                        }
                        if (!frz && __ballot(contrib) != 0ull) {
                            if (CNT) wred += 1u;
                            float t, t8;
                            row_sum9(g9, lane, t, t8);
                            // one write per lane, no lane mask: lanes 0-7 of a row write
                            // values 0-7, lanes 8-15 all value 8 (the same word and value)
                            const bool hi8 = (lane & 8) != 0;
                            s_part[4 * wid + (lane >> 4)][hi8 ? 8 : (lane & 7)][k - c0] = hi8 ? t8 : t;
                        }
                    }
                }
                {
                    // the rows' totals added in a fixed order
                    __syncthreads();
                    if (tid < c1 - c0) {
                        const int k = c0 + tid;
                        if (!s_frz[k]) {
                            float sum[9];
                            bool nz = false;
#pragma unroll
                            for (int q = 0; q < 9; ++q) {
                                float acc = s_part[0][q][tid];
                                s_part[0][q][tid] = 0.f;
#pragma unroll
                                for (int w = 1; w < 4 * W; ++w) {
                                    acc += s_part[w][q][tid];
                                    s_part[w][q][tid] = 0.f;
                                }
                                sum[q] = acc;
                                nz = nz || (acc != 0.f);
                            }
                            if (nz) {   // a slot counts only with this call's stamp
                                // from the moments (sums of dpow dx, dpow dy, dpow dx^2,
                                // dpow dx dy, dpow dy^2) to the gradient of the mean,
                                // d power / d(u, v) = ln 2 (2 A dx + B dy, B dx + 2 C dy),
                                // and of the conic entries (-dx^2 / 2, -dx dy, -dy^2 / 2)
                                const float A = s_geo[k].z, B = s_geo[k].w, C = s_co[k].x;
                                const float X = sum[0], Y = sum[1];
                                sum[0] = kLn2 * fmaf(2.0f * A, X, B * Y);
                                sum[1] = kLn2 * fmaf(B, X, 2.0f * C * Y);
                                sum[2] = -0.5f * sum[2];
                                sum[3] = -sum[3];
                                sum[4] = -0.5f * sum[4];
                                float* dst = partials + (int64_t)s_idx[k] * 9;
#pragma unroll
                                for (int q = 0; q < 9; ++q) dst[q] = sum[q];
                                sc.stamps[s_idx[k]] = gen;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }
    if (CNT) {
        __syncthreads();
        if (evals) atomicAdd(&s_pairs, evals);
        if (ngrad) atomicAdd(&s_grad, ngrad);
        __syncthreads();
        if (tid == 0 && s_pairs) atomicAdd(pairs + 1, (unsigned long long)s_pairs);
        if (tid == 0 && s_grad) atomicAdd(pairs + 5, (unsigned long long)s_grad);
        if ((tid & 63) == 0 && witer) atomicAdd(pairs + 3, (unsigned long long)witer);
        if ((tid & 63) == 0 && wred) atomicAdd(pairs + 4, (unsigned long long)wred);
    }
}


}  // namespace

template <bool CNT>
void fwd_launch(int waves, const uint2* ranges, const uint32_t* gsort, const float4* geo,
                const float4* col, const float4* rgb, int64_t stride, const CamArray& cams, int nv, float bg0,
                float bg1, float bg2, float* image, float* T_final, uint32_t* last, double* cfg, const SegCkpt& sc,
                unsigned long long* pairs, const FusedL1& l1, hipStream_t s) {
    const int tiles = cams.c[0].ntx * cams.c[0].nty;
#define GSTA_FWD_ARGS ranges, gsort, geo, col, rgb, stride, cams, bg0, bg1, bg2, image, T_final, last, cfg, sc, pairs, l1
    if (waves == 0)   // one independent wave per 8x8 quarter of each tile
        k_composite_fwd<1, true, CNT><<<dim3(4 * tiles, nv), 64, 0, s>>>(GSTA_FWD_ARGS);
    else if (waves == 1)
        k_composite_fwd<1, false, CNT><<<dim3(tiles, nv), 64, 0, s>>>(GSTA_FWD_ARGS);
    else if (waves == 2)
        k_composite_fwd<2, false, CNT><<<dim3(tiles, nv), 128, 0, s>>>(GSTA_FWD_ARGS);
    else
        k_composite_fwd<4, false, CNT><<<dim3(tiles, nv), 256, 0, s>>>(GSTA_FWD_ARGS);
#undef GSTA_FWD_ARGS
}

template <bool CNT>
void bwd_launch(int waves, int blocks, const uint2* ranges, const uint32_t* ids, const uint32_t* gsort,
                const float4* geo, const float4* col, const float4* rgb, int64_t stride, const uint8_t* frozen,
                const CamArray& cams, int nv, float bg0, float bg1, float bg2, const float* T_final,
                const uint32_t* last, const double* cfg, const float* dL_dimage, float* partials, const SegCkpt& sc,
                unsigned long long* pairs, hipStream_t s) {
#define GSTA_BWD_ARGS ranges, ids, gsort, geo, col, rgb, stride, frozen, cams, nv, bg0, bg1, bg2, T_final, last, \
                      cfg, dL_dimage, partials, sc, pairs
    if (waves == 1)
        k_composite_bwd<1, CNT><<<blocks, 64, 0, s>>>(GSTA_BWD_ARGS);
    else if (waves == 2)
        k_composite_bwd<2, CNT><<<blocks, 128, 0, s>>>(GSTA_BWD_ARGS);
    else
        k_composite_bwd<4, CNT><<<blocks, 256, 0, s>>>(GSTA_BWD_ARGS);
#undef GSTA_BWD_ARGS
}

void launch_composite_fwd(int waves, const uint2* ranges, const uint32_t* gsort, const float4* geo, const float4* col, const float4* rgb, int64_t stride,
                          const CamArray& cams, int nv, float bg0, float bg1, float bg2, float* image,
                          float* T_final, uint32_t* last, double* cfg, const SegCkpt& sc, unsigned long long* pairs,
                          const FusedL1& l1, hipStream_t s) {
    // sc.tile_last and sc.ctr arrive zeroed (cleared by the binning)
    const int tiles = cams.c[0].ntx * cams.c[0].nty;
    if (pairs)
        fwd_launch<true>(waves, ranges, gsort, geo, col, rgb, stride, cams, nv, bg0, bg1, bg2, image, T_final,
                         last, cfg, sc, pairs, l1, s);
    else
        fwd_launch<false>(waves, ranges, gsort, geo, col, rgb, stride, cams, nv, bg0, bg1, bg2, image, T_final,
                          last, cfg, sc, pairs, l1, s);
    // the backward's work items: ceil(tile_last / K) per tile (and the fused loss's sums)
    const int nparts = tiles * nv * (waves == 0 ? 4 : 1);
    k_seg_items<<<1, 1024, 0, s>>>(sc.tile_last, tiles * nv, sc.shift, sc.item_off, sc.item_tile, sc.item_cap,
                                   l1.part, nparts, l1.target ? l1.sums : nullptr);
}

void launch_composite_bwd(int waves, int blocks, const uint2* ranges, const uint32_t* ids, const uint32_t* gsort,
                          const float4* geo, const float4* col, const float4* rgb, int64_t stride,
                          const uint8_t* frozen, const CamArray& cams, int nv, float bg0, float bg1, float bg2,
                          const float* T_final, const uint32_t* last, const double* cfg, const float* dL_dimage,
                          float* partials, const uint32_t* d_count, const SegCkpt& sc, unsigned long long* pairs,
                          hipStream_t s) {
    (void)d_count;
    if (pairs)
        bwd_launch<true>(waves, blocks, ranges, ids, gsort, geo, col, rgb, stride, frozen, cams, nv, bg0, bg1, bg2,
                         T_final, last, cfg, dL_dimage, partials, sc, pairs, s);
    else
        bwd_launch<false>(waves, blocks, ranges, ids, gsort, geo, col, rgb, stride, frozen, cams, nv, bg0, bg1,
                          bg2, T_final, last, cfg, dL_dimage, partials, sc, pairs, s);
}

int composite_bwd_blocks_per_cu(int waves) {
    int nb = 0;
    hipError_t e;
    if (waves == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_composite_bwd<1, false>, 64, 0);
    else if (waves == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_composite_bwd<2, false>, 128, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_composite_bwd<4, false>, 256, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace gsta
