// Per-Gaussian projection (forward) and its chain rule (backward).
//
// Forward (Section 3.1, eq. 1 -- EWA splatting): one thread per Gaussian,
// looping over the views of the call so the SoA parameter rows are read once.
// Writes the 2-D splat record (mean, conic, colour, opacity), the tile
// rectangle of its 3-sigma ellipse and the depth sort key.
//
// Backward (Section 3.2.4): one thread per active Gaussian; frozen ones
// return at once and their gradient rows are never touched.  Chains the
// per-view 2-D gradients to every parameter, sums over views, and updates the
// gradient-norm moving averages used by the freeze rule (Section 3.2.1).
#include "gsta_internal.h"

namespace gsta {
namespace {

// Real SH basis (unit-norm on the sphere, positive sign), k = l*l + l + m.
constexpr float C0 = 0.28209479177387814f;
constexpr float C1 = 0.4886025119029199f;
constexpr float C2a = 1.0925484305920792f;   // xy, yz, xz
constexpr float C2b = 0.31539156525252005f;  // 2z^2 - x^2 - y^2
constexpr float C2c = 0.5462742152960396f;   // x^2 - y^2
constexpr float C3a = 0.5900435899266435f;   // y(3x^2 - y^2), x(x^2 - 3y^2)
constexpr float C3b = 2.890611442640554f;    // xyz
constexpr float C3c = 0.4570457994644658f;   // y(4z^2 - x^2 - y^2), x(4z^2 - x^2 - y^2)
constexpr float C3d = 0.3731763325901154f;   // z(2z^2 - 3x^2 - 3y^2)
constexpr float C3e = 1.445305721320277f;    // z(x^2 - y^2)

template <int D>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* B) {
    B[0] = C0;
    if (D >= 1) {
        B[1] = C1 * y;
        B[2] = C1 * z;
        B[3] = C1 * x;
    }
    if (D >= 2) {
        float xx = x * x, yy = y * y, zz = z * z;
        B[4] = C2a * x * y;
        B[5] = C2a * y * z;
        B[6] = C2b * (2.f * zz - xx - yy);
        B[7] = C2a * x * z;
        B[8] = C2c * (xx - yy);
        if (D >= 3) {
            B[9] = C3a * y * (3.f * xx - yy);
            B[10] = C3b * x * y * z;
            B[11] = C3c * y * (4.f * zz - xx - yy);
            B[12] = C3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
            B[13] = C3c * x * (4.f * zz - xx - yy);
            B[14] = C3e * z * (xx - yy);
            B[15] = C3a * x * (xx - 3.f * yy);
        }
    }
}

// g = d/d(x,y,z) of sum_k w[k] B_k(x, y, z).
template <int D>
__device__ __forceinline__ void sh_grad_weighted(const float* w, float x, float y, float z, float* g) {
    g[0] = g[1] = g[2] = 0.f;
    if (D >= 1) {
        g[1] += C1 * w[1];
        g[2] += C1 * w[2];
        g[0] += C1 * w[3];
    }
    if (D >= 2) {
        float xx = x * x, yy = y * y, zz = z * z;
        g[0] += C2a * (w[4] * y + w[7] * z) + C2b * w[6] * (-2.f * x) + C2c * w[8] * (2.f * x);
        g[1] += C2a * (w[4] * x + w[5] * z) + C2b * w[6] * (-2.f * y) + C2c * w[8] * (-2.f * y);
        g[2] += C2a * (w[5] * y + w[7] * x) + C2b * w[6] * (4.f * z);
        if (D >= 3) {
            g[0] += C3a * w[9] * (6.f * x * y) + C3b * w[10] * (y * z) + C3c * w[11] * (-2.f * x * y) +
                    C3d * w[12] * (-6.f * x * z) + C3c * w[13] * (4.f * zz - 3.f * xx - yy) +
                    C3e * w[14] * (2.f * x * z) + C3a * w[15] * (3.f * xx - 3.f * yy);
            g[1] += C3a * w[9] * (3.f * xx - 3.f * yy) + C3b * w[10] * (x * z) +
                    C3c * w[11] * (4.f * zz - xx - 3.f * yy) + C3d * w[12] * (-6.f * y * z) +
                    C3c * w[13] * (-2.f * x * y) + C3e * w[14] * (-2.f * y * z) +
                    C3a * w[15] * (-6.f * x * y);
            g[2] += C3b * w[10] * (x * y) + C3c * w[11] * (8.f * y * z) +
                    C3d * w[12] * (6.f * zz - 3.f * xx - 3.f * yy) + C3c * w[13] * (8.f * x * z) +
                    C3e * w[14] * (xx - yy);
        }
    }
}

// Camera-space position.  The dot products run in double precision and are
// rounded once, so the float32 depth (the sort key) is the correctly rounded
// camera depth of the float32 inputs.
__device__ __forceinline__ void to_camera(const DevCam& c, const float* mu, float* xc) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double acc = (double)c.t[r];
        acc = fma((double)c.R[3 * r + 2], (double)mu[2], acc);
        acc = fma((double)c.R[3 * r + 1], (double)mu[1], acc);
        acc = fma((double)c.R[3 * r + 0], (double)mu[0], acc);
        xc[r] = (float)acc;
    }
}

// Rotation of the unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(const float* q, float* R) {
    float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.f - 2.f * (y * y + z * z);
    R[1] = 2.f * (x * y - w * z);
    R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);
    R[4] = 1.f - 2.f * (x * x + z * z);
    R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);
    R[7] = 2.f * (y * z + w * x);
    R[8] = 1.f - 2.f * (x * x + y * y);
}

// Geometry of one view shared by forward and backward: 2-D covariance via
// P = J W R S (2x3), A = P P^T + 0.3 I.  det(A) is formed from the 2x2 minors
// of P (Cauchy-Binet) plus the dilation terms, which avoids the cancellation
// of a*c - b*b for thin splats.
struct Geo {
    float xc[3];
    float rx, ry, rxc, ryc;
    bool clx, cly;
    float T0[3], T1[3];   // rows of J W
    float P0[3], P1[3];   // rows of J W M
    float a, b, c, det, inv;
    float u, v;
};

__device__ __forceinline__ bool project_geo(const DevCam& cm, const float* mu, const float* Rq,
                                            const float* s, Geo& g) {
    to_camera(cm, mu, g.xc);
    float z = g.xc[2];
    if (!(z > cm.near_z)) return false;
    float iz = 1.0f / z;
    g.rx = g.xc[0] * iz;
    g.ry = g.xc[1] * iz;
    g.clx = fabsf(g.rx) > cm.limx;
    g.cly = fabsf(g.ry) > cm.limy;
    g.rxc = g.clx ? copysignf(cm.limx, g.rx) : g.rx;
    g.ryc = g.cly ? copysignf(cm.limy, g.ry) : g.ry;
    float j00 = cm.fx * iz, j02 = -cm.fx * g.rxc * iz;
    float j11 = cm.fy * iz, j12 = -cm.fy * g.ryc * iz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.T0[k] = j00 * cm.R[k] + j02 * cm.R[6 + k];
        g.T1[k] = j11 * cm.R[3 + k] + j12 * cm.R[6 + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {   // column k of M = R S is s_k * R[:, k]
        g.P0[k] = (g.T0[0] * Rq[k] + g.T0[1] * Rq[3 + k] + g.T0[2] * Rq[6 + k]) * s[k];
        g.P1[k] = (g.T1[0] * Rq[k] + g.T1[1] * Rq[3 + k] + g.T1[2] * Rq[6 + k]) * s[k];
    }
    float a0 = g.P0[0] * g.P0[0] + g.P0[1] * g.P0[1] + g.P0[2] * g.P0[2];
    float c0 = g.P1[0] * g.P1[0] + g.P1[1] * g.P1[1] + g.P1[2] * g.P1[2];
    g.b = g.P0[0] * g.P1[0] + g.P0[1] * g.P1[1] + g.P0[2] * g.P1[2];
    float m01 = g.P0[0] * g.P1[1] - g.P0[1] * g.P1[0];
    float m02 = g.P0[0] * g.P1[2] - g.P0[2] * g.P1[0];
    float m12 = g.P0[1] * g.P1[2] - g.P0[2] * g.P1[1];
    g.a = a0 + kDilate;
    g.c = c0 + kDilate;
    g.det = (m01 * m01 + m02 * m02 + m12 * m12) + kDilate * (a0 + c0) + kDilate * kDilate;
    if (!(g.det > 0.f)) return false;
    g.inv = 1.0f / g.det;
    g.u = cm.fx * g.rx + cm.cx;
    g.v = cm.fy * g.ry + cm.cy;
    return true;
}

// Opacity activation: sigmoid of the logit (opact 0), or the absolute value
// of the parameter (opact 1), which the finetune stage switches to
// (Section 4.1: the "absolute" activation of Taming 3DGS; opacities above 1
// then make high-opacity Gaussians, alpha still capped at 0.99).
__device__ __forceinline__ void load_core(const float* __restrict__ P, int64_t ld, int64_t i, float* mu,
                                          float* s, float* qn, float* Rq, float& qinv, float& o, int opact) {
    mu[0] = P[i];
    mu[1] = P[ld + i];
    mu[2] = P[2 * ld + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = expf(P[(3 + k) * ld + i]);
    float q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = P[(6 + k) * ld + i];
    qinv = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) qn[k] = q[k] * qinv;
    quat_rot(qn, Rq);
    const float x = P[10 * ld + i];
    o = opact ? fabsf(x) : 1.0f / (1.0f + expf(-x));
}

// SH-band masks (Section 3.3): band l = 1..D of Gaussian i is kept where its
// logit exceeds the threshold's logit (sigmoid(logit) > threshold), else its
// coefficients count as zero.  gate[l] is 1 or 0 (gate[0] = 1).
template <int D>
__device__ __forceinline__ void band_gates(const ShMask& sm, int64_t ld, int64_t i, float* gate) {
    gate[0] = 1.f;
#pragma unroll
    for (int l = 1; l <= D; ++l) gate[l] = (sm.logit && !(sm.logit[(l - 1) * ld + i] > sm.thr_logit)) ? 0.f : 1.f;
}

__device__ __forceinline__ constexpr int sh_band(int k) { return k < 1 ? 0 : (k < 4 ? 1 : (k < 9 ? 2 : 3)); }

template <int D>
// hist0 (optional): the depth sort's first-pass (low 8 bits) digit counts of
// the block's keys (its 256 Gaussians), at hist0[v * hv + digit * hd +
// (blockIdx.x >> hshift) * hc]: stored when hshift is 0, else added (the
// 2^hshift blocks of a chunk share its counters).
__global__ __launch_bounds__(256) void k_preprocess_fwd(
    const float* __restrict__ P, int64_t ld, int64_t n, CamArray cams, int nv,
    float4* __restrict__ geo, float4* __restrict__ col, float4* __restrict__ rgbo,
    ushort4* __restrict__ rect, uint32_t* __restrict__ dkey, uint32_t* __restrict__ dval,
    int64_t stride, uint32_t* __restrict__ hist0, int64_t hv, int64_t hd, int64_t hc, int hshift, int opact,
    ShMask sm) {
    constexpr int K = (D + 1) * (D + 1);
    __shared__ uint32_t s_h[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    if (!valid && !hist0) return;    // with hist0 every thread reaches the barriers
    float mu[3], s[3], qn[4], Rq[9], qinv, o;
    float f[K][3];
    if (valid) {
        load_core(P, ld, i, mu, s, qn, Rq, qinv, o, opact);
        float gate[D + 1];
        band_gates<D>(sm, ld, i, gate);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) f[k][ch] = gate[sh_band(k)] * P[(11 + 3 * k + ch) * ld + i];
    }

    for (int v = 0; v < nv; ++v) {
        if (hist0) {
            s_h[threadIdx.x] = 0;
            __syncthreads();
        }
        if (valid) {
            const DevCam& cm = cams.c[v];
            const int64_t o_idx = (int64_t)v * stride + i;
            Geo g;
            bool vis = project_geo(cm, mu, Rq, s, g);
            ushort4 r = make_ushort4(0, 0, 0, 0);
            float4 rg = make_float4(0.f, 0.f, 0.f, 0.f);
            if (vis) {
                float ex = 3.0f * sqrtf(g.a), ey = 3.0f * sqrtf(g.c);
                float x0 = ceilf((g.u - ex - (float)(kTile - 1)) * (1.0f / kTile));
                float x1 = floorf((g.u + ex) * (1.0f / kTile)) + 1.0f;
                float y0 = ceilf((g.v - ey - (float)(kTile - 1)) * (1.0f / kTile));
                float y1 = floorf((g.v + ey) * (1.0f / kTile)) + 1.0f;
                int tx0 = (int)fminf(fmaxf(x0, 0.f), (float)cm.ntx);
                int tx1 = (int)fminf(fmaxf(x1, 0.f), (float)cm.ntx);
                int ty0 = (int)fminf(fmaxf(y0, 0.f), (float)cm.nty);
                int ty1 = (int)fminf(fmaxf(y1, 0.f), (float)cm.nty);
                vis = (tx0 < tx1) && (ty0 < ty1);
                if (vis) {
                    r = make_ushort4((unsigned short)tx0, (unsigned short)tx1, (unsigned short)ty0,
                                     (unsigned short)ty1);
                    // SH colour with the unit direction from the camera centre.
                    float d[3] = {mu[0] - cm.pos[0], mu[1] - cm.pos[1], mu[2] - cm.pos[2]};
                    float il = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    float B[16];
                    sh_eval<D>(d[0] * il, d[1] * il, d[2] * il, B);
                    float cc[3];
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        float acc = 0.f;
#pragma unroll
                        for (int k = 0; k < K; ++k) acc += f[k][ch] * B[k];
                        cc[ch] = fmaxf(acc + 0.5f, 0.f);
                    }
                    rg = make_float4(cc[0], cc[1], cc[2], g.xc[2]);
                    // conic (a, b, c) = (c', -b', a') / det, stored pre-scaled (kConicScale*)
                    geo[o_idx] = make_float4(g.u, g.v, (g.c * g.inv) * kConicScaleAC, (-g.b * g.inv) * kConicScaleB);
                    // Screen half-extent outside which no pixel can be a member:
                    // power >= -4.5 and o exp(power) >= 1/255 bound d^T conic d by
                    // 2 min(4.5, ln(255 o)).  Inflated by 1% + 0.5 px so float32
                    // rounding never makes a skipped splat a member.
                    const float lo = logf(255.0f * o);
                    float ex2 = -1e30f, ey2 = -1e30f;
                    if (lo > 0.f) {
                        const float kf = sqrtf(2.0f * fminf(4.5f, lo));
                        ex2 = kf * sqrtf(g.a) * 1.01f + 0.5f;
                        ey2 = kf * sqrtf(g.c) * 1.01f + 0.5f;
                    }
                    col[o_idx] = make_float4((g.a * g.inv) * kConicScaleAC, o, ex2, ey2);
                }
            }
            if (!vis) {
                geo[o_idx] = make_float4(0.f, 0.f, 0.f, 0.f);
                col[o_idx] = make_float4(0.f, 0.f, -1e30f, -1e30f);
                if (g.xc[2] > cm.near_z) rg.w = g.xc[2];
            }
            rgbo[o_idx] = rg;
            rect[o_idx] = r;
            const uint32_t key = vis ? __float_as_uint(g.xc[2]) : 0xFFFFFFFFu;
            dkey[o_idx] = key;
            dval[o_idx] = (uint32_t)i;
            if (hist0) atomicAdd(&s_h[key & 0xFFu], 1u);
        }
        if (hist0) {
            __syncthreads();
            uint32_t* h = hist0 + (int64_t)v * hv + (int64_t)threadIdx.x * hd + (int64_t)(blockIdx.x >> hshift) * hc;
            if (hshift == 0)
                *h = s_h[threadIdx.x];
            else if (s_h[threadIdx.x])
                atomicAdd(h, s_h[threadIdx.x]);
            __syncthreads();
        }
    }
}

// Sum over each row of 16 lanes with DPP (pairs, quads, then rotations by
// 4 and 8 within the row); every lane of a row holds its row's total.
__device__ __forceinline__ float row16_sum(float v) {
    int x = __builtin_bit_cast(int, v);
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
    x = __builtin_bit_cast(int, v);
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
    x = __builtin_bit_cast(int, v);
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false));
    x = __builtin_bit_cast(int, v);
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));
    return v;
}

// 2-D gradient of each (view, active visible Gaussian): the sum of the
// per-tile totals of the compositing backward, into d2sum[v][9][stride].  A
// slot without this call's stamp (the current generation) was not written by
// it (nothing reached the splat there) and counts as zero.  A Gaussian's slots are contiguous, so a
// row of 16 lanes takes one Gaussian and reads 16 consecutive slots per
// step (coalesced); lane l adds slots l, l+16, ... and the row is then
// summed in a fixed order.
constexpr int kSumRows = 16;   // Gaussians per 256-thread block

__global__ __launch_bounds__(256) void k_sum_partials(const ushort4* __restrict__ rect,
                                                      const uint32_t* __restrict__ inst_off, int64_t stride,
                                                      int64_t n, const float* __restrict__ partials,
                                                      const uint32_t* __restrict__ stamps,
                                                      const uint32_t* __restrict__ genp,
                                                      const uint32_t* __restrict__ d_count,
                                                      const uint8_t* __restrict__ frozen,
                                                      float* __restrict__ d2sum) {
    const int l16 = threadIdx.x & 15;
    const int64_t i = (int64_t)blockIdx.x * kSumRows + (threadIdx.x >> 4);
    const int v = blockIdx.y;
    const int64_t o_idx = (int64_t)v * stride + i;
    // the independent loads first, so that their latencies overlap
    const bool inb = i < n;
    const bool fz = inb && frozen && frozen[i];
    const ushort4 r = inb ? rect[o_idx] : make_ushort4(0, 0, 0, 0);
    const uint64_t j0 = inb ? inst_off[o_idx] : 0ull;
    // `work` is uniform over each row of 16 lanes
    const bool work = inb && !fz && r.x < r.y;
    if (work) {
        const uint32_t cnt = (uint32_t)(r.y - r.x) * (uint32_t)(r.w - r.z);
        const uint32_t gen = *genp;
        float d2[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) d2[k] = 0.f;
        if (j0 + cnt <= (uint64_t)(*d_count)) {
            // lane l adds slots l, l + 16, l + 32, ... in that order, two per step
            uint32_t base = 0;
            for (; base + 16u < cnt; base += 32u) {
                const uint32_t t0 = base + (uint32_t)l16, t1 = t0 + 16u;
                const bool s0 = stamps[j0 + t0] == gen;
                const bool s1 = t1 < cnt && stamps[j0 + t1] == gen;
                if (s0) {
                    const float* src = partials + (j0 + t0) * 9;
#pragma unroll
                    for (int k = 0; k < 9; ++k) d2[k] += src[k];
                }
                if (s1) {
                    const float* src = partials + (j0 + t1) * 9;
#pragma unroll
                    for (int k = 0; k < 9; ++k) d2[k] += src[k];
                }
            }
            if (base < cnt) {
                const uint32_t t = base + (uint32_t)l16;
                if (t < cnt && stamps[j0 + t] == gen) {
                    const float* src = partials + (j0 + t) * 9;
#pragma unroll
                    for (int k = 0; k < 9; ++k) d2[k] += src[k];
                }
            }
        }
        float out = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float tot = row16_sum(d2[k]);
            if (l16 == k) out = tot;
        }
        if (l16 < 9) d2sum[((int64_t)v * 9 + l16) * stride + i] = out;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_preprocess_bwd(
    const float* __restrict__ P, int64_t ld, int64_t n, CamArray cams, int nv,
    const ushort4* __restrict__ rect, int64_t stride, const float* __restrict__ d2sum,
    const uint8_t* __restrict__ frozen,
    float* __restrict__ G, int64_t gld, float* __restrict__ ema, float beta, float* __restrict__ grad2d_out,
    float* __restrict__ dstats, uint32_t* __restrict__ genp, int opact, ShMask sm) {
    constexpr int K = (D + 1) * (D + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // Every reader of this backward's generation (the compositing backward
    // and the partial sums) has finished before this kernel starts, so one
    // thread moves the generation on for the next backward.
    if (i == 0) *genp = *genp + 1u;
    if (i >= n) return;
    if (frozen && frozen[i]) return;
    float mu[3], s[3], qn[4], Rq[9], qinv, o;
    load_core(P, ld, i, mu, s, qn, Rq, qinv, o, opact);
    // f: the coefficients as used (a closed band's are zero); fr: as stored
    float gate[D + 1];
    band_gates<D>(sm, ld, i, gate);
    float f[K][3], fr[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            fr[k][ch] = P[(11 + 3 * k + ch) * ld + i];
            f[k][ch] = gate[sh_band(k)] * fr[k][ch];
        }

    float gmu[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gqn[4] = {0.f, 0.f, 0.f, 0.f};
    float glogit = 0.f;
    float gsh[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    bool any_vis = false;
    float dsum = 0.f, dcnt = 0.f;   // densification: screen-gradient norms, visible views

    for (int v = 0; v < nv; ++v) {
        const int64_t o_idx = (int64_t)v * stride + i;
        ushort4 r = rect[o_idx];
        if (!(r.x < r.y)) continue;    // culled in this view by the forward
        any_vis = true;
        const DevCam& cm = cams.c[v];
        // 2-D gradient of this view: the per-tile totals of the compositing
        // backward, summed in row-major tile order.
        float d2[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) d2[k] = d2sum[((int64_t)v * 9 + k) * stride + i];
        if (grad2d_out) {
#pragma unroll
            for (int k = 0; k < 9; ++k) grad2d_out[((int64_t)v * 9 + k) * n + i] = d2[k];
        }
        if (dstats) {
            // gradient with respect to the normalised device coordinates of the mean
            const float nx = d2[0] * (0.5f * (float)cm.width), ny = d2[1] * (0.5f * (float)cm.height);
            dsum += sqrtf(nx * nx + ny * ny);
            dcnt += 1.f;
        }
        Geo g;
        project_geo(cm, mu, Rq, s, g);
        float z = g.xc[2], iz = 1.0f / z, iz2 = iz * iz;

        // ---- colour: rgb = max(0, sum_k f_k B_k(dir) + 0.5) ----
        float d[3] = {mu[0] - cm.pos[0], mu[1] - cm.pos[1], mu[2] - cm.pos[2]};
        float il = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float dn[3] = {d[0] * il, d[1] * il, d[2] * il};
        float B[16];
        sh_eval<D>(dn[0], dn[1], dn[2], B);
        float draw[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) acc += f[k][ch] * B[k];
            draw[ch] = (acc + 0.5f < 0.f) ? 0.f : d2[6 + ch];
        }
        float wk[16];
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gsh[k][ch] += draw[ch] * B[k];
            wk[k] = draw[0] * f[k][0] + draw[1] * f[k][1] + draw[2] * f[k][2];
        }
        if (D > 0) {
            float gd[3];
            sh_grad_weighted<D>(wk, dn[0], dn[1], dn[2], gd);
            float dot = gd[0] * dn[0] + gd[1] * dn[1] + gd[2] * dn[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) gmu[a] += (gd[a] - dn[a] * dot) * il;
        }

        // ---- opacity ----
        if (opact) {   // d|x|/dx = sign(x), 0 at x = 0
            const float x = P[10 * ld + i];
            glogit += x > 0.f ? d2[5] : (x < 0.f ? -d2[5] : 0.f);
        } else {
            glogit += d2[5] * o * (1.f - o);
        }

        // ---- conic = A^-1:  GA = -K GK K with GK = [[dca, dcb/2], [dcb/2, dcc]] ----
        float pk = g.c * g.inv, qk = -g.b * g.inv, rk = g.a * g.inv;
        float al = d2[2], be = 0.5f * d2[3], ga = d2[4];
        float ga00 = -(pk * pk * al + 2.f * pk * qk * be + qk * qk * ga);
        float ga01 = -(pk * qk * al + (pk * rk + qk * qk) * be + qk * rk * ga);
        float ga11 = -(qk * qk * al + 2.f * qk * rk * be + rk * rk * ga);
        // ---- A = P P^T + 0.3 I: dP = 2 GA P ----
        float dP0[3], dP1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dP0[k] = 2.f * (ga00 * g.P0[k] + ga01 * g.P1[k]);
            dP1[k] = 2.f * (ga01 * g.P0[k] + ga11 * g.P1[k]);
        }
        // ---- P = T M with M = R S:  dM = T^T dP,  dT = dP M^T ----
        float dT0[3] = {0.f, 0.f, 0.f}, dT1[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float dsk = 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float Mjk = Rq[3 * j + k] * s[k];
                float dMjk = g.T0[j] * dP0[k] + g.T1[j] * dP1[k];
                dT0[j] += dP0[k] * Mjk;
                dT1[j] += dP1[k] * Mjk;
                dsk += dMjk * Rq[3 * j + k];
                // dR_jk = dM_jk * s_k  -> quaternion below
                float dR = dMjk * s[k];
                // R(q) partials, accumulated per entry (row j, column k)
                float w = qn[0], x = qn[1], y = qn[2], zq = qn[3];
                switch (3 * j + k) {
                    case 0: gqn[2] += -4.f * y * dR; gqn[3] += -4.f * zq * dR; break;
                    case 1: gqn[0] += -2.f * zq * dR; gqn[1] += 2.f * y * dR; gqn[2] += 2.f * x * dR; gqn[3] += -2.f * w * dR; break;
                    case 2: gqn[0] += 2.f * y * dR; gqn[1] += 2.f * zq * dR; gqn[2] += 2.f * w * dR; gqn[3] += 2.f * x * dR; break;
                    case 3: gqn[0] += 2.f * zq * dR; gqn[1] += 2.f * y * dR; gqn[2] += 2.f * x * dR; gqn[3] += 2.f * w * dR; break;
                    case 4: gqn[1] += -4.f * x * dR; gqn[3] += -4.f * zq * dR; break;
                    case 5: gqn[0] += -2.f * x * dR; gqn[1] += -2.f * w * dR; gqn[2] += 2.f * zq * dR; gqn[3] += 2.f * y * dR; break;
                    case 6: gqn[0] += -2.f * y * dR; gqn[1] += 2.f * zq * dR; gqn[2] += -2.f * w * dR; gqn[3] += 2.f * x * dR; break;
                    case 7: gqn[0] += 2.f * x * dR; gqn[1] += 2.f * w * dR; gqn[2] += 2.f * zq * dR; gqn[3] += 2.f * y * dR; break;
                    default: gqn[1] += -4.f * x * dR; gqn[2] += -4.f * y * dR; break;
                }
            }
            gls[k] += dsk * s[k];
        }
        // ---- T = J W: dJ = dT W^T (entries 00, 02, 11, 12 are variable) ----
        float dJ00 = dT0[0] * cm.R[0] + dT0[1] * cm.R[1] + dT0[2] * cm.R[2];
        float dJ02 = dT0[0] * cm.R[6] + dT0[1] * cm.R[7] + dT0[2] * cm.R[8];
        float dJ11 = dT1[0] * cm.R[3] + dT1[1] * cm.R[4] + dT1[2] * cm.R[5];
        float dJ12 = dT1[0] * cm.R[6] + dT1[1] * cm.R[7] + dT1[2] * cm.R[8];
        float dxc[3] = {0.f, 0.f, 0.f};
        dxc[2] += -(dJ00 * cm.fx + dJ11 * cm.fy) * iz2;
        if (!g.clx) {
            dxc[0] += -dJ02 * cm.fx * iz2;
            dxc[2] += 2.f * dJ02 * cm.fx * g.rx * iz2;
        } else {
            dxc[2] += dJ02 * cm.fx * g.rxc * iz2;
        }
        if (!g.cly) {
            dxc[1] += -dJ12 * cm.fy * iz2;
            dxc[2] += 2.f * dJ12 * cm.fy * g.ry * iz2;
        } else {
            dxc[2] += dJ12 * cm.fy * g.ryc * iz2;
        }
        // ---- u = fx x/z + cx, v = fy y/z + cy ----
        dxc[0] += d2[0] * cm.fx * iz;
        dxc[1] += d2[1] * cm.fy * iz;
        dxc[2] += -(d2[0] * cm.fx * g.rx + d2[1] * cm.fy * g.ry) * iz;
        // ---- x_cam = W mu + t ----
#pragma unroll
        for (int a = 0; a < 3; ++a) gmu[a] += cm.R[a] * dxc[0] + cm.R[3 + a] * dxc[1] + cm.R[6 + a] * dxc[2];
    }

    // Quaternion normalisation: dq = (dqn - qn (qn . dqn)) / |q|.
    float qd = qn[0] * gqn[0] + qn[1] * gqn[1] + qn[2] * gqn[2] + qn[3] * gqn[3];
    G[i] = gmu[0];
    G[gld + i] = gmu[1];
    G[2 * gld + i] = gmu[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) G[(3 + k) * gld + i] = gls[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) G[(6 + k) * gld + i] = (gqn[k] - qn[k] * qd) * qinv;
    G[10 * gld + i] = glogit;
    // gsh is dL/d(gate f): a stored coefficient gets it times its gate, and
    // each band's logit the straight-through dL/dgate sigmoid'(logit)
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) G[(11 + 3 * k + ch) * gld + i] = gate[sh_band(k)] * gsh[k][ch];
    if (sm.logit && sm.grad) {
#pragma unroll
        for (int l = 1; l <= D; ++l) {
            float dM = 0.f;
#pragma unroll
            for (int k = l * l; k < (l + 1) * (l + 1); ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) dM += gsh[k][ch] * fr[k][ch];
            const float x = sm.logit[(l - 1) * ld + i];
            const float sg = 1.0f / (1.0f + expf(-x));
            sm.grad[(l - 1) * gld + i] = dM * (sg * (1.0f - sg));
        }
    }

    if (dstats && any_vis) {
        dstats[i] += dsum;
        dstats[n + i] += dcnt;
        dstats[2 * n + i] += sqrtf(gsh[0][0] * gsh[0][0] + gsh[0][1] * gsh[0][1] + gsh[0][2] * gsh[0][2]);
        dstats[3 * n + i] += 1.f;
    }
    if (ema && any_vis) {
        float sc[4];
        sc[0] = sqrtf(gmu[0] * gmu[0] + gmu[1] * gmu[1] + gmu[2] * gmu[2]);
        sc[1] = sqrtf(gsh[0][0] * gsh[0][0] + gsh[0][1] * gsh[0][1] + gsh[0][2] * gsh[0][2]);
        sc[2] = fabsf(glogit);
        sc[3] = sqrtf(gls[0] * gls[0] + gls[1] * gls[1] + gls[2] * gls[2]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float prev = ema[(int64_t)k * n + i];
            ema[(int64_t)k * n + i] = (prev >= 3.402823466e38f) ? sc[k] : beta * prev + (1.f - beta) * sc[k];
        }
    }
}

}  // namespace

void launch_preprocess_fwd(const float* P, int64_t ld, int64_t n, int degree, const CamArray& cams,
                           int nv, float4* geo, float4* col, float4* rgb, ushort4* rect,
                           uint32_t* dkey, uint32_t* dval, int64_t stride, uint32_t* hist0, bool hist_chunks,
                           int opact, const ShMask& sm, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const int64_t hp = (n + 255) / 256;   // blocks of 256 keys
    int hshift = 0;
    while ((256 << hshift) < kSmallSortChunkKeys) ++hshift;
    const int64_t hv = hist_chunks ? (int64_t)kSmallSortChunks * 256 : 256 * hp;
    const int64_t hd = hist_chunks ? 1 : hp, hc = hist_chunks ? 256 : 1;
    if (!hist_chunks) hshift = 0;
#define GSTA_PRE_ARGS P, ld, n, cams, nv, geo, col, rgb, rect, dkey, dval, stride, hist0, hv, hd, hc, hshift, opact, sm
    switch (degree) {
        case 0: k_preprocess_fwd<0><<<grid, block, 0, s>>>(GSTA_PRE_ARGS); break;
        case 1: k_preprocess_fwd<1><<<grid, block, 0, s>>>(GSTA_PRE_ARGS); break;
        case 2: k_preprocess_fwd<2><<<grid, block, 0, s>>>(GSTA_PRE_ARGS); break;
        default: k_preprocess_fwd<3><<<grid, block, 0, s>>>(GSTA_PRE_ARGS); break;
    }
#undef GSTA_PRE_ARGS
}

void launch_preprocess_bwd(const float* P, int64_t ld, int64_t n, int degree, const CamArray& cams,
                           int nv, const ushort4* rect, const uint32_t* inst_off, int64_t stride,
                           const float* partials, const uint32_t* stamps, uint32_t* gen,
                           const uint32_t* d_count, const uint8_t* frozen, float* d2sum, float* G,
                           int64_t gld, float* ema, float beta, float* grad2d_out, float* dstats, int opact,
                           const ShMask& sm, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    k_sum_partials<<<dim3((unsigned)((n + kSumRows - 1) / kSumRows), (unsigned)nv), block, 0, s>>>(
        rect, inst_off, stride, n, partials, stamps, gen, d_count, frozen, d2sum);
#define GSTA_BWD_ARGS P, ld, n, cams, nv, rect, stride, d2sum, frozen, G, gld, ema, beta, grad2d_out, dstats, gen, opact, sm
    switch (degree) {
        case 0: k_preprocess_bwd<0><<<grid, block, 0, s>>>(GSTA_BWD_ARGS); break;
        case 1: k_preprocess_bwd<1><<<grid, block, 0, s>>>(GSTA_BWD_ARGS); break;
        case 2: k_preprocess_bwd<2><<<grid, block, 0, s>>>(GSTA_BWD_ARGS); break;
        default: k_preprocess_bwd<3><<<grid, block, 0, s>>>(GSTA_BWD_ARGS); break;
    }
#undef GSTA_BWD_ARGS
}

}  // namespace gsta
