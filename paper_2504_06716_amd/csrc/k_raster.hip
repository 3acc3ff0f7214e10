// Tile compositing, forward and backward.
//
// Forward (Section 3.1, eq. 2): one 256-thread workgroup per 16x16 tile,
// one thread per pixel.  The tile's depth-ordered splats are staged in LDS
// in batches of 256 (one record per thread, a gather by gid), then every
// pixel walks the batch front to back.  A workgroup stops fetching batches
// once every pixel has terminated (__syncthreads_count).  The colour is
// accumulated in double precision and kept per pixel for the backward.
//
// Backward (Section 3.2.4): same workgroup shape.  Each pixel re-walks its
// list up to its last member and recomputes the transmittance with the same
// instructions as the forward (shared eval_splat / next_T), so every
// membership and termination decision is identical.  The colour behind a
// member is the forward colour minus the recomputed prefix (both double).
// Frozen splats still attenuate the pixels behind them but get no gradient
// work.  Per splat the 9 partial derivatives are summed over the wave
// (skipped when no lane contributed), over the four waves in LDS, and added
// to the per-view 2-D gradient with one global atomic per value and tile.
#include "gsta_internal.h"

namespace gsta {
namespace {

constexpr int BATCH = kTilePix;

__global__ __launch_bounds__(kTilePix) void k_composite_fwd(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids, const float4* __restrict__ geo,
    const float4* __restrict__ col, const float4* __restrict__ rgbv, int64_t stride, CamArray cams,
    float bg0, float bg1, float bg2, float* __restrict__ image, float* __restrict__ T_final,
    uint32_t* __restrict__ last_out, double* __restrict__ cfg) {
    __shared__ float4 s_geo[BATCH];
    __shared__ float2 s_co[BATCH];
    __shared__ float4 s_rgb[BATCH];
    const int v = blockIdx.y;
    const DevCam& cm = cams.c[v];
    const int tiles = cm.ntx * cm.nty;
    const int tile = blockIdx.x;
    const int tid = threadIdx.x;
    const int px = (tile % cm.ntx) * kTile + (tid & (kTile - 1));
    const int py = (tile / cm.ntx) * kTile + (tid / kTile);
    const bool inside = px < cm.width && py < cm.height;
    const uint2 rg = ranges[(int64_t)v * tiles + tile];
    const int64_t vs = (int64_t)v * stride;
    const float fpx = (float)px, fpy = (float)py;

    float T = 1.0f;
    double C0 = 0.0, C1 = 0.0, C2 = 0.0;
    uint32_t last = 0;
    bool done = !inside;
    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t j = base + tid;
        if (j < rg.y) {
            const uint32_t gid = ids[j];
            s_geo[tid] = geo[vs + gid];
            const float4 c = col[vs + gid];
            s_co[tid] = make_float2(c.x, c.y);
            s_rgb[tid] = rgbv[vs + gid];
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)BATCH, rg.y - base);
        if (!done) {
            for (int k = 0; k < cnt; ++k) {
                const float4 g = s_geo[k];
                const float2 co = s_co[k];
                SplatEval e;
                eval_splat(g.x, g.y, g.z, g.w, co.x, co.y, fpx, fpy, e);
                if (e.power < kPowerFloor) continue;
                if (e.alpha < kAlphaMin) continue;
                const float Tn = next_T(T, e.alpha);
                if (Tn < kTMin) {
                    done = true;
                    break;
                }
                const float4 c = s_rgb[k];
                const double w = (double)(e.alpha * T);
                C0 = fma((double)c.x, w, C0);
                C1 = fma((double)c.y, w, C1);
                C2 = fma((double)c.z, w, C2);
                T = Tn;
                last = base - rg.x + (uint32_t)k + 1u;
            }
        }
    }
    if (inside) {
        const int64_t HW = (int64_t)cm.width * cm.height;
        const int64_t pix = (int64_t)py * cm.width + px;
        float* img = image + (int64_t)v * 3 * HW + pix;
        img[0] = (float)(C0 + (double)(T * bg0));
        img[HW] = (float)(C1 + (double)(T * bg1));
        img[2 * HW] = (float)(C2 + (double)(T * bg2));
        T_final[(int64_t)v * HW + pix] = T;
        last_out[(int64_t)v * HW + pix] = last;
        double* cf = cfg + (int64_t)v * 3 * HW + pix;
        cf[0] = C0;
        cf[HW] = C1;
        cf[2 * HW] = C2;
    }
}

__global__ __launch_bounds__(kTilePix) void k_composite_bwd(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids, const float4* __restrict__ geo,
    const float4* __restrict__ col, const float4* __restrict__ rgbv, int64_t stride,
    const uint8_t* __restrict__ frozen, CamArray cams, float bg0, float bg1, float bg2,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last_in, const double* __restrict__ cfg,
    const float* __restrict__ dL_dimage, float* __restrict__ grad2d) {
    __shared__ float4 s_geo[BATCH];
    __shared__ float2 s_co[BATCH];
    __shared__ float4 s_rgb[BATCH];
    __shared__ uint32_t s_gid[BATCH];
    __shared__ uint32_t s_frz[BATCH];
    __shared__ float s_acc[9][BATCH];
    __shared__ uint32_t s_hit[BATCH];
    __shared__ uint32_t s_maxlast;

    const int v = blockIdx.y;
    const DevCam& cm = cams.c[v];
    const int tiles = cm.ntx * cm.nty;
    const int tile = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int px = (tile % cm.ntx) * kTile + (tid & (kTile - 1));
    const int py = (tile / cm.ntx) * kTile + (tid / kTile);
    const bool inside = px < cm.width && py < cm.height;
    const uint2 rg = ranges[(int64_t)v * tiles + tile];
    const int64_t vs = (int64_t)v * stride;
    const float fpx = (float)px, fpy = (float)py;
    const int64_t HW = (int64_t)cm.width * cm.height;
    const int64_t pix = (int64_t)py * cm.width + px;

    float dC0 = 0.f, dC1 = 0.f, dC2 = 0.f, Tf = 1.f;
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;   // forward colour (background excluded)
    uint32_t last = 0;
    if (inside) {
        const float* dl = dL_dimage + (int64_t)v * 3 * HW + pix;
        dC0 = dl[0];
        dC1 = dl[HW];
        dC2 = dl[2 * HW];
        Tf = T_final[(int64_t)v * HW + pix];
        last = last_in[(int64_t)v * HW + pix];
        const double* cf = cfg + (int64_t)v * 3 * HW + pix;
        F0 = cf[0];
        F1 = cf[HW];
        F2 = cf[2 * HW];
    }
    if (tid == 0) s_maxlast = 0;
    __syncthreads();
    if (last) atomicMax(&s_maxlast, last);
    __syncthreads();
    const uint32_t end = rg.x + s_maxlast;
    const float tb0 = Tf * bg0, tb1 = Tf * bg1, tb2 = Tf * bg2;

    float T = 1.0f;
    double A0 = 0.0, A1 = 0.0, A2 = 0.0;   // colour of the members walked so far
    for (uint32_t base = rg.x; base < end; base += BATCH) {
        __syncthreads();
        const uint32_t j = base + tid;
        if (j < end) {
            const uint32_t gid = ids[j];
            s_gid[tid] = gid;
            s_geo[tid] = geo[vs + gid];
            const float4 c = col[vs + gid];
            s_co[tid] = make_float2(c.x, c.y);
            s_rgb[tid] = rgbv[vs + gid];
            s_frz[tid] = frozen ? (uint32_t)frozen[gid] : 0u;
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) s_acc[q][tid] = 0.f;
        s_hit[tid] = 0;
        __syncthreads();
        const int cnt = (int)min((uint32_t)BATCH, end - base);
        for (int k = 0; k < cnt; ++k) {
            const uint32_t idx = base - rg.x + (uint32_t)k;
            float g9[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) g9[q] = 0.f;
            bool contrib = false;
            if (idx < last) {
                const float4 g = s_geo[k];
                const float2 co = s_co[k];
                SplatEval e;
                eval_splat(g.x, g.y, g.z, g.w, co.x, co.y, fpx, fpy, e);
                if (e.power >= kPowerFloor && e.alpha >= kAlphaMin) {
                    const float4 c = s_rgb[k];
                    const float w = e.alpha * T;
                    const double wd = (double)w;
                    A0 = fma((double)c.x, wd, A0);
                    A1 = fma((double)c.y, wd, A1);
                    A2 = fma((double)c.z, wd, A2);
                    if (!s_frz[k]) {
                        contrib = true;
                        const float inv1m = 1.0f / (1.0f - e.alpha);
                        const float b0 = (float)(F0 - A0) + tb0;
                        const float b1 = (float)(F1 - A1) + tb1;
                        const float b2 = (float)(F2 - A2) + tb2;
                        const float dalpha = dC0 * (c.x * T - b0 * inv1m) + dC1 * (c.y * T - b1 * inv1m) +
                                             dC2 * (c.z * T - b2 * inv1m);
                        g9[6] = dC0 * w;
                        g9[7] = dC1 * w;
                        g9[8] = dC2 * w;
                        if (e.oG <= kAlphaMax) {
                            const float dpow = dalpha * e.alpha;
                            g9[5] = dalpha * e.G;
                            g9[0] = -dpow * (g.z * e.dx + g.w * e.dy);
                            g9[1] = -dpow * (g.w * e.dx + co.x * e.dy);
                            g9[2] = -0.5f * dpow * e.dx * e.dx;
                            g9[3] = -dpow * e.dx * e.dy;
                            g9[4] = -0.5f * dpow * e.dy * e.dy;
                        }
                    }
                    T = next_T(T, e.alpha);
                }
            }
            if (__ballot(contrib) != 0ull) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const float sum = wave_sum(g9[q]);
                    if (lane == 0) atomicAdd(&s_acc[q][k], sum);
                }
                if (lane == 0) s_hit[k] = 1u;
            }
        }
        __syncthreads();
        if (tid < cnt && s_hit[tid]) {
            const uint32_t gid = s_gid[tid];
            float* out = grad2d + (int64_t)v * 9 * stride + gid;
#pragma unroll
            for (int q = 0; q < 9; ++q) unsafeAtomicAdd(out + (int64_t)q * stride, s_acc[q][tid]);
        }
    }
}

}  // namespace

void launch_composite_fwd(const uint2* ranges, const uint32_t* ids, const float4* geo,
                          const float4* col, const float4* rgb, int64_t stride, const CamArray& cams,
                          int nv, float bg0, float bg1, float bg2, float* image, float* T_final,
                          uint32_t* last, double* cfg, hipStream_t s) {
    const int tiles = cams.c[0].ntx * cams.c[0].nty;
    k_composite_fwd<<<dim3(tiles, nv), kTilePix, 0, s>>>(ranges, ids, geo, col, rgb, stride, cams, bg0,
                                                          bg1, bg2, image, T_final, last, cfg);
}

void launch_composite_bwd(const uint2* ranges, const uint32_t* ids, const float4* geo,
                          const float4* col, const float4* rgb, int64_t stride, const uint8_t* frozen,
                          const CamArray& cams, int nv, float bg0, float bg1, float bg2,
                          const float* T_final, const uint32_t* last, const double* cfg,
                          const float* dL_dimage, float* grad2d, hipStream_t s) {
    const int tiles = cams.c[0].ntx * cams.c[0].nty;
    k_composite_bwd<<<dim3(tiles, nv), kTilePix, 0, s>>>(ranges, ids, geo, col, rgb, stride, frozen, cams,
                                                          bg0, bg1, bg2, T_final, last, cfg, dL_dimage,
                                                          grad2d);
}

}  // namespace gsta
