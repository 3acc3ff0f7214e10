// Backward compositing, per-splat variant (Section 3.2.4: the paper's
// rasterizer parallelises the backward over the splats of a tile, keeping
// per-splat state in its threads and passing per-pixel state between them).
//
// One 64-lane workgroup per work item (tile, segment of list positions), the
// same items as the per-pixel variant.  The segment is taken 64 splats at a
// time, one splat per lane; the tile's pixels that are still walking at the
// sub-segment's start stream through the wave: at step t lane l meets pixel
// t - l, and the pixel's transmittance and colour behind move one lane to
// the right between steps (DPP wave shift), so each pixel meets the splats in
// list order with the forward's exact transmittance sequence.  A lane sums
// its own splat's nine 2-D gradient terms over every pixel it meets: no
// cross-lane reductions and no atomics.  A pixel's constant data (dL/dC, its
// last member, its coordinates) is read by every lane from LDS; lane 0 also
// takes the pixel's starting state from there, and the sub-segment's last
// splat lane writes the state back for the next sub-segment.
//
// Per pair the arithmetic is the per-pixel variant's (shared evaluation,
// same transmittance and colour updates in list order); only the order in
// which a splat's terms over pixels are added differs, so the two variants
// agree to rounding.  A lane whose splat is frozen still applies its
// (1 - alpha) but does no gradient work; on SIMD hardware that saves time
// only when the whole wave's splats are frozen, which is why the per-pixel
// variant, which skips a frozen splat for all its pixels at once, stays the
// default inside a freezing window.
#include "gsta_internal.h"

namespace gsta {
namespace {

constexpr int kSplatLanes = 64;

__device__ __forceinline__ float shr1f(float v, float lane0) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, lane0),
                                                                 __builtin_bit_cast(int, v), 0x138, 0xF, 0xF,
                                                                 false));
}

__device__ __forceinline__ double shr1d(double v, double lane0) {
    const uint64_t a = __builtin_bit_cast(uint64_t, v), b = __builtin_bit_cast(uint64_t, lane0);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)b, (int)(uint32_t)a, 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(b >> 32), (int)(uint32_t)(a >> 32), 0x138, 0xF, 0xF,
                                               false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ __launch_bounds__(kSplatLanes) void k_composite_bwd_splat(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids, const uint32_t* __restrict__ gsort,
    const float4* __restrict__ geo, const float4* __restrict__ col, const float4* __restrict__ rgbv,
    int64_t stride, const uint8_t* __restrict__ frozen, CamArray cams, int nv, float bg0, float bg1, float bg2,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last_in, const double* __restrict__ cfg,
    const float* __restrict__ dL_dimage, float* __restrict__ partials, SegCkpt sc) {
    // the walking pixels of the current sub-segment, compacted in tile order
    __shared__ float4 s_pc[kTilePix];       // dL/dC r, g, b and the last member (bits)
    __shared__ uint32_t s_xy[kTilePix];     // x | y << 16
    __shared__ float s_T[kTilePix];         // transmittance before the sub-segment
    __shared__ double s_B[3][kTilePix];     // colour behind the sub-segment's first splat (background included)

    const int lane = threadIdx.x;
    const int tiles = cams.c[0].ntx * cams.c[0].nty;
    const int nt = nv * tiles;
    const uint32_t n_items = min(sc.item_off[nt], sc.item_cap);
    const bool seg = sc.shift < 31u;
    const uint32_t gen = *sc.gen;

    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int gt = (int)sc.item_tile[item];
        const uint32_t sgi = item - sc.item_off[gt];
        const int v = gt / tiles, tile = gt - v * tiles;
        const DevCam& cm = cams.c[v];
        const int tx0 = (tile % cm.ntx) * kTile, ty0 = (tile / cm.ntx) * kTile;
        const uint2 rg = ranges[gt];
        const int64_t vs = (int64_t)v * stride;
        const int64_t HW = (int64_t)cm.width * cm.height;
        const uint32_t tl = sc.tile_last[gt];
        const uint32_t p0 = seg ? (sgi << sc.shift) : 0u;
        const uint32_t p1 = seg ? min(tl, (sgi + 1u) << sc.shift) : tl;

        // ---- stage the pixels that walk past p0: 64-pixel group g = 8x8 quarter ----
        __syncthreads();   // the previous item's last reads are done
        uint32_t np = 0;
        const size_t bucket = (size_t)((rg.x + p0) >> sc.shift);
#pragma unroll
        for (int g = 0; g < kCkptGroups; ++g) {
            const int px = tx0 + (g & 1) * 8 + (lane & 7), py = ty0 + (g >> 1) * 8 + (lane >> 3);
            uint32_t last = 0;
            int64_t o = 0;
            if (px < cm.width && py < cm.height) {
                o = (int64_t)py * cm.width + px;
                last = last_in[(int64_t)v * HW + o];
            }
            bool keep = last > p0;
            float T = 1.0f;
            double A[3] = {0.0, 0.0, 0.0};
            if (keep && p0 != 0u) {   // resume from the forward's state at the segment boundary
                const uint32_t slot = sc.idx[bucket * kCkptGroups + g];
                if (slot >= sc.pool_cap) {
                    keep = false;       // the forward ran out of slots (flagged)
                } else {
                    const double* d = sc.pool + (size_t)slot * 256;
                    T = (float)d[lane];
                    A[0] = d[64 + lane];
                    A[1] = d[128 + lane];
                    A[2] = d[192 + lane];
                }
            }
            const uint64_t m = __ballot(keep);
            const uint32_t r = np + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (keep) {
                const float* dl = dL_dimage + (int64_t)v * 3 * HW + o;
                const float tf = T_final[(int64_t)v * HW + o];
                const double* cf = cfg + (int64_t)v * 3 * HW + o;
                s_pc[r] = make_float4(dl[0], dl[HW], dl[2 * HW], __builtin_bit_cast(float, last));
                s_xy[r] = (uint32_t)px | ((uint32_t)py << 16);
                s_T[r] = T;
                s_B[0][r] = (cf[0] + (double)(tf * bg0)) - A[0];
                s_B[1][r] = (cf[HW] + (double)(tf * bg1)) - A[1];
                s_B[2][r] = (cf[2 * HW] + (double)(tf * bg2)) - A[2];
            }
            np += (uint32_t)__popcll(m);
        }
        __syncthreads();

        for (uint32_t s0 = p0; s0 < p1 && np > 0u; s0 += kSplatLanes) {
            const int ns = (int)min((uint32_t)kSplatLanes, p1 - s0);
            // this lane's splat
            const bool has = lane < ns;
            const uint32_t pos = s0 + (uint32_t)lane;          // its list position
            float4 g = make_float4(0.f, 0.f, 0.f, 0.f), c = make_float4(0.f, 0.f, 0.f, 0.f);
            float2 co = make_float2(0.f, 0.f);
            uint32_t idx = 0;
            bool frz = true;
            if (has) {
                const uint32_t j = rg.x + pos;
                const uint32_t gid = gsort[j];
                idx = ids[j];
                g = geo[vs + gid];
                const float4 cc = col[vs + gid];
                co = make_float2(cc.x, cc.y);
                c = rgbv[vs + gid];
                frz = frozen ? frozen[gid] != 0 : false;
            }
            const double cx = (double)c.x, cy = (double)c.y, cz = (double)c.z;
            float g9[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) g9[q] = 0.f;
            float T = 1.0f;
            double B0 = 0.0, B1 = 0.0, B2 = 0.0;
            const int steps = (int)np + ns - 1;
            for (int t = 0; t < steps; ++t) {
                const int jc = t - lane;
                const bool inr = (unsigned)jc < np;
                const int jr = inr ? jc : 0;
                const float4 pc = s_pc[jr];
                const uint32_t xy = s_xy[jr];
                // lane 0 starts pixel t from its staged state; the others take
                // the state their left neighbour left after its splat
                T = shr1f(T, s_T[jr]);
                B0 = shr1d(B0, s_B[0][jr]);
                B1 = shr1d(B1, s_B[1][jr]);
                B2 = shr1d(B2, s_B[2][jr]);
                const uint32_t last = __builtin_bit_cast(uint32_t, pc.w);
                const bool act = inr && has && pos < last;
                SplatEval e;
                eval_power(g.x, g.y, g.z, g.w, co.x, (float)(xy & 0xFFFFu), (float)(xy >> 16), e);
                eval_alpha(co.y, e);
                const bool m = act && e.power2 >= kPower2Floor && e.alpha >= kAlphaMin;
                const float w = m ? e.alpha * T : 0.f;
                const double wd = (double)w;
                B0 = fma(-cx, wd, B0);
                B1 = fma(-cy, wd, B1);
                B2 = fma(-cz, wd, B2);
                if (!frz) {
                    const float inv1m = __builtin_amdgcn_rcpf(1.0f - e.alpha);
                    const float b0 = (float)B0, b1 = (float)B1, b2 = (float)B2;
                    const float da = pc.x * (c.x * T - b0 * inv1m) + pc.y * (c.y * T - b1 * inv1m) +
                                     pc.z * (c.z * T - b2 * inv1m);
                    g9[6] += pc.x * w;
                    g9[7] += pc.y * w;
                    g9[8] += pc.z * w;
                    // alpha clamped at kAlphaMax: no gradient to opacity or power
                    const float dalpha = (m && e.oG <= kAlphaMax) ? da : 0.f;
                    const float dpow = dalpha * e.alpha;
                    const float dpl = dpow * kLn2;
                    g9[5] += dalpha * e.G;
                    g9[0] += dpl * (2.0f * g.z * e.dx + g.w * e.dy);
                    g9[1] += dpl * (g.w * e.dx + 2.0f * co.x * e.dy);
                    g9[2] -= 0.5f * dpow * e.dx * e.dx;
                    g9[3] -= dpow * e.dx * e.dy;
                    g9[4] -= 0.5f * dpow * e.dy * e.dy;
                }
                T = m ? next_T(T, e.alpha) : T;
                if (lane == ns - 1 && inr) {   // the pixel's state after this sub-segment
                    s_T[jc] = T;
                    s_B[0][jc] = B0;
                    s_B[1][jc] = B1;
                    s_B[2][jc] = B2;
                }
            }
            if (has && !frz) {
                bool nz = false;
#pragma unroll
                for (int q = 0; q < 9; ++q) nz = nz || (g9[q] != 0.f);
                if (nz) {   // a slot counts only with this call's stamp
                    float* dst = partials + (int64_t)idx * 9;
#pragma unroll
                    for (int q = 0; q < 9; ++q) dst[q] = g9[q];
                    sc.stamps[idx] = gen;
                }
            }
            // keep the pixels still walking past the next sub-segment's start (stable, in place)
            const uint32_t s1 = s0 + (uint32_t)kSplatLanes;
            if (s1 < p1) {
                __syncthreads();
                float4 kpc[kTilePix / kSplatLanes];
                uint32_t kxy[kTilePix / kSplatLanes];
                float kT[kTilePix / kSplatLanes];
                double kB[kTilePix / kSplatLanes][3];
                bool kk[kTilePix / kSplatLanes];
#pragma unroll
                for (int q = 0; q < kTilePix / kSplatLanes; ++q) {
                    const uint32_t j = (uint32_t)(q * kSplatLanes + lane);
                    kk[q] = false;
                    if (j < np) {
                        kpc[q] = s_pc[j];
                        kxy[q] = s_xy[j];
                        kT[q] = s_T[j];
                        kB[q][0] = s_B[0][j];
                        kB[q][1] = s_B[1][j];
                        kB[q][2] = s_B[2][j];
                        kk[q] = __builtin_bit_cast(uint32_t, kpc[q].w) > s1;
                    }
                }
                __syncthreads();
                uint32_t n2 = 0;
#pragma unroll
                for (int q = 0; q < kTilePix / kSplatLanes; ++q) {
                    const uint64_t m = __ballot(kk[q]);
                    const uint32_t r = n2 + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (kk[q]) {
                        s_pc[r] = kpc[q];
                        s_xy[r] = kxy[q];
                        s_T[r] = kT[q];
                        s_B[0][r] = kB[q][0];
                        s_B[1][r] = kB[q][1];
                        s_B[2][r] = kB[q][2];
                    }
                    n2 += (uint32_t)__popcll(m);
                }
                np = n2;
                __syncthreads();
            }
        }
    }
}

}  // namespace

void launch_composite_bwd_splat(int blocks, const uint2* ranges, const uint32_t* ids, const uint32_t* gsort,
                                const float4* geo, const float4* col, const float4* rgb, int64_t stride,
                                const uint8_t* frozen, const CamArray& cams, int nv, float bg0, float bg1, float bg2,
                                const float* T_final, const uint32_t* last, const double* cfg,
                                const float* dL_dimage, float* partials, const SegCkpt& sc, hipStream_t s) {
    k_composite_bwd_splat<<<blocks, kSplatLanes, 0, s>>>(ranges, ids, gsort, geo, col, rgb, stride, frozen, cams, nv,
                                                         bg0, bg1, bg2, T_final, last, cfg, dL_dimage, partials, sc);
}

int composite_bwd_splat_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_composite_bwd_splat, kSplatLanes, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace gsta
