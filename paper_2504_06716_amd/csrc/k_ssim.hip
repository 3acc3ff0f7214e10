// D-SSIM term of the loss (eq. 3, lambda_SSIM = 0.2): SSIM with an 11 x 11
// Gaussian window (sigma 1.5, normalised, zero padding), C1 = 0.01^2,
// C2 = 0.03^2, per channel; L_D-SSIM = 1 - mean SSIM.  The window is
// separable, so each 2-D filter runs as a row pass and a column pass over a
// tile staged in LDS (the paper's accelerated SSIM replaces each 2-D
// convolution by two 1-D ones and fuses the map computation after them).
//
// Forward (k_ssim_fwd): one workgroup per (32 x 16 tile, view, channel)
// stages the tile and its 5-pixel halo of image x and target y, filters the
// five moments x, y, x^2, y^2, x y (row pass into LDS, column pass in
// registers; double accumulation, which costs the same as float on this GPU
// without packed FP32 and keeps the variance differences exact enough), then
// per pixel forms the SSIM map S and the three partial derivatives of the
// loss with respect to the filtered moments m = G*x, s = G*x^2, c = G*(x y):
//   g_m = k S (2 mu_y / A - 2 mu_y / B - 2 mu_x / C + 2 mu_x / D),
//   g_s = -k S / D,   g_c = 2 k S / B,   k = -lambda / count,
// written as three float maps, and adds S into the workgroup's partial sum.
// Backward (k_ssim_bwd): the same tiling filters the three maps (the filter
// is its own adjoint) and writes
//   dL = (1 - lambda) dL_L1 + G*g_m + 2 x G*g_s + y G*g_c.
#include "gsta_internal.h"

#include <cmath>

namespace gsta {
namespace {

constexpr int TW = 32, TH = 16, R = 5, K = 2 * R + 1;
constexpr int IW = TW + 2 * R, IH = TH + 2 * R;   // staged tile with halo: 42 x 26
constexpr double kC1 = 1e-4, kC2 = 9e-4;          // (0.01)^2, (0.03)^2

// Stages plane[y][x] (zero outside [0, H) x [0, W)) for the tile at (x0, y0).
__device__ __forceinline__ void stage(const float* __restrict__ plane, int W, int H, int x0, int y0,
                                      float (*dst)[IW]) {
    for (int i = threadIdx.x; i < IH * IW; i += 256) {
        const int r = i / IW, c = i - r * IW;
        const int gy = y0 + r - R, gx = x0 + c - R;
        dst[r][c] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? plane[(int64_t)gy * W + gx] : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ img, const float* __restrict__ tgt,
                                                  int W, int H, SsimTaps wt, double k,
                                                  float* __restrict__ gmap, int64_t plane_stride,
                                                  double* __restrict__ part) {
    __shared__ float sx[IH][IW], sy[IH][IW];
    __shared__ double hrow[5][IH][TW];
    __shared__ double s_w[4];
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
    const int64_t plane = (int64_t)blockIdx.z * H * W;     // (view, channel) plane
    stage(img + plane, W, H, x0, y0, sx);
    stage(tgt + plane, W, H, x0, y0, sy);
    __syncthreads();
    // row pass: the five moments filtered along x for every staged row
    for (int i = threadIdx.x; i < IH * TW; i += 256) {
        const int r = i / TW, c = i - r * TW;
        double ax = 0, ay = 0, axx = 0, ayy = 0, axy = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double xv = sx[r][c + t], yv = sy[r][c + t], w = wt.w[t];
            ax = fma(w, xv, ax);
            ay = fma(w, yv, ay);
            axx = fma(w, xv * xv, axx);
            ayy = fma(w, yv * yv, ayy);
            axy = fma(w, xv * yv, axy);
        }
        hrow[0][r][c] = ax;
        hrow[1][r][c] = ay;
        hrow[2][r][c] = axx;
        hrow[3][r][c] = ayy;
        hrow[4][r][c] = axy;
    }
    __syncthreads();
    // column pass, SSIM and the partial derivatives: 2 pixels per thread
    double ssum = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int r = i / TW, c = i - r * TW;
        const int gy = y0 + r, gx = x0 + c;
        double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double w = wt.w[t];
            mx = fma(w, hrow[0][r + t][c], mx);
            my = fma(w, hrow[1][r + t][c], my);
            exx = fma(w, hrow[2][r + t][c], exx);
            eyy = fma(w, hrow[3][r + t][c], eyy);
            exy = fma(w, hrow[4][r + t][c], exy);
        }
        if (gy < H && gx < W) {
            const double vx = exx - mx * mx, vy = eyy - my * my, cxy = exy - mx * my;
            const double A = 2.0 * mx * my + kC1, B = 2.0 * cxy + kC2;
            const double C = mx * mx + my * my + kC1, D = vx + vy + kC2;
            const double S = (A * B) / (C * D);
            ssum += S;
            const double ks = k * S;
            const int64_t o = plane + (int64_t)gy * W + gx;
            gmap[o] = (float)(ks * (2.0 * my / A - 2.0 * my / B - 2.0 * mx / C + 2.0 * mx / D));
            gmap[plane_stride + o] = (float)(-ks / D);
            gmap[2 * plane_stride + o] = (float)(2.0 * ks / B);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ssum += __shfl_xor(ssum, off, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = ssum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[b] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ img, const float* __restrict__ tgt,
                                                  int W, int H, SsimTaps wt, float l1_weight,
                                                  const float* __restrict__ gmap, int64_t plane_stride,
                                                  float* __restrict__ dL) {
    __shared__ float sg[3][IH][IW];
    __shared__ double hrow[3][IH][TW];
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
    const int64_t plane = (int64_t)blockIdx.z * H * W;
#pragma unroll
    for (int m = 0; m < 3; ++m) stage(gmap + m * plane_stride + plane, W, H, x0, y0, sg[m]);
    __syncthreads();
    for (int i = threadIdx.x; i < IH * TW; i += 256) {
        const int r = i / TW, c = i - r * TW;
        double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double w = wt.w[t];
            a0 = fma(w, (double)sg[0][r][c + t], a0);
            a1 = fma(w, (double)sg[1][r][c + t], a1);
            a2 = fma(w, (double)sg[2][r][c + t], a2);
        }
        hrow[0][r][c] = a0;
        hrow[1][r][c] = a1;
        hrow[2][r][c] = a2;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int r = i / TW, c = i - r * TW;
        const int gy = y0 + r, gx = x0 + c;
        if (gy >= H || gx >= W) continue;
        double fm = 0, fs = 0, fc = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double w = wt.w[t];
            fm = fma(w, hrow[0][r + t][c], fm);
            fs = fma(w, hrow[1][r + t][c], fs);
            fc = fma(w, hrow[2][r + t][c], fc);
        }
        const int64_t o = plane + (int64_t)gy * W + gx;
        const double xv = img[o], yv = tgt[o];
        dL[o] = (float)((double)l1_weight * (double)dL[o] + fm + 2.0 * xv * fs + yv * fc);
    }
}

// Sum of the workgroups' partial sums in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_ssim_final(const double* __restrict__ part, int64_t nb,
                                                    double* __restrict__ out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) a += part[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

}  // namespace

int64_t ssim_blocks(int nv, int H, int W) {
    return (int64_t)((W + TW - 1) / TW) * ((H + TH - 1) / TH) * nv * 3;
}

void launch_dssim(const float* img, const float* tgt, int nv, int H, int W, float lambda, float* dL, double* ssim_sum,
                  float* gmap, double* part, hipStream_t s) {
    SsimTaps wt;
    double sum = 0.0;
    for (int t = 0; t < K; ++t) {
        const double d = (double)(t - R);
        wt.w[t] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
        sum += wt.w[t];
    }
    for (int t = 0; t < K; ++t) wt.w[t] /= sum;
    const int64_t count = (int64_t)nv * 3 * H * W;
    const int64_t plane_stride = count;
    const dim3 grid((unsigned)((W + TW - 1) / TW), (unsigned)((H + TH - 1) / TH), (unsigned)(nv * 3));
    k_ssim_fwd<<<grid, 256, 0, s>>>(img, tgt, W, H, wt, -(double)lambda / (double)count, gmap, plane_stride, part);
    k_ssim_final<<<1, 256, 0, s>>>(part, ssim_blocks(nv, H, W), ssim_sum);
    k_ssim_bwd<<<grid, 256, 0, s>>>(img, tgt, W, H, wt, 1.0f - lambda, gmap, plane_stride, dL);
}

}  // namespace gsta
