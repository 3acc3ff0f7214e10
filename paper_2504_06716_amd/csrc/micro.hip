// Peak microbenchmarks for the roofline fractions of the training kernels
// (built into their own library, libgsta_micro.so; measurement only).
// Each probe runs a kernel shaped to saturate one resource and reports the
// elapsed time of `reps` launches (HIP events on the caller's stream):
//   0 HBM copy           4 float4 per thread (nontemporal), bytes = 2 * size per launch
//   1 FP32 FMA           8 independent FMA chains per lane, flops = 2 per FMA
//   2 v_exp_f32          8 independent exp2 chains per lane
//   3 LDS ds_read_b128   float4 reads of a 16 KiB LDS array, conflict-free
//   4 BF16 MFMA          4 independent 16x16x32 accumulation chains per wave
//   5 FP32 atomics       atomicAdd to distinct addresses (one per thread)
//   6 FP32 atomics       atomicAdd contended: 64 addresses per launch
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// four float4 per thread, all loads issued before the stores (n a multiple
// of 1024; one workgroup per 16 KiB)
typedef float f32v4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src4, float4* __restrict__ dst4, int64_t n) {
    const f32v4* src = reinterpret_cast<const f32v4*>(src4);
    f32v4* dst = reinterpret_cast<f32v4*>(dst4);
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    f32v4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(src + base + 256 * k);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], dst + base + 256 * k);
    (void)n;
}

__global__ __launch_bounds__(256) void k_fma(float* out, int iters, float a, float b) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (float)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == 12345.678f) out[0] = s;     // keeps the chains alive, never true in practice
}

__global__ __launch_bounds__(256) void k_exp(float* out, int iters) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = -1e-3f * (float)(threadIdx.x & 7) - 1e-4f * k;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(x[k]) - 1.0f;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == 12345.678f) out[0] = s;
}

__global__ __launch_bounds__(256) void k_lds(float* out, int iters) {
    __shared__ float4 buf[1024];
    for (int k = threadIdx.x; k < 1024; k += 256) buf[k] = make_float4((float)k, 1.f, 2.f, 3.f);
    __syncthreads();
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int idx = threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 v = buf[(idx + 256 * k) & 1023];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        idx = (idx + 64) & 1023;
    }
    if (acc.x + acc.y + acc.z + acc.w == 12345.678f) out[0] = acc.x;
}

__global__ __launch_bounds__(256) void k_mfma(float* out, int iters) {
    const int lane = threadIdx.x & 63;
    bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(0.001f * (float)(lane + k));
        b[k] = (__bf16)(0.002f * (float)(lane - k));
    }
    f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
    }
    const float s = c0[0] + c1[1] + c2[2] + c3[3];
    if (s == 12345.678f) out[0] = s;
}

__global__ __launch_bounds__(256) void k_atomic(float* dst, int64_t n, int64_t mask, int iters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < iters; ++r) atomicAdd(dst + (i & mask), 1.0f);
}

}  // namespace

extern "C" {

// Runs probe `kind` `reps` times after one untimed launch on `stream` and
// returns the elapsed milliseconds of the timed launches in *ms and the
// work they did in *work (bytes for 0 and 3, flops for 1 and 4, exps for 2,
// atomic operations for 5 and 6).  buf0, buf1: device buffers of `bytes`
// bytes (probes 0, 5, 6).  Returns 0 or a HIP error code.
int gsta_micro_probe(int kind, void* buf0, void* buf1, int64_t bytes, int reps, hipStream_t stream, float* ms,
                     double* work) {
    hipDevice_t dev = 0;
    int cus = 1;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 2;
    const int blocks = cus * 8;
    const int iters = 4096;
    double w = 0.0;
    auto launch = [&]() {
        switch (kind) {
            case 0: {
                const int64_t n = bytes / 16 / 1024 * 1024;
                k_copy<<<(unsigned)(n / 1024), 256, 0, stream>>>((const float4*)buf0, (float4*)buf1, n);
                w = 2.0 * (double)(n * 16);
                break;
            }
            case 1:
                k_fma<<<blocks, 256, 0, stream>>>((float*)buf0, iters, 0.999f, 1e-3f);
                w = 2.0 * 8.0 * iters * (double)blocks * 256.0;
                break;
            case 2:
                k_exp<<<blocks, 256, 0, stream>>>((float*)buf0, iters);
                w = 8.0 * iters * (double)blocks * 256.0;
                break;
            case 3:
                k_lds<<<blocks, 256, 0, stream>>>((float*)buf0, iters / 4);
                w = 16.0 * 4.0 * (iters / 4) * (double)blocks * 256.0;
                break;
            case 4:
                k_mfma<<<blocks, 256, 0, stream>>>((float*)buf0, iters / 4);
                w = 16.0 * 16.0 * 32.0 * 2.0 * 4.0 * (iters / 4) * (double)blocks * 4.0;
                break;
            case 5:
            case 6: {
                const int64_t n = bytes / 4;
                k_atomic<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>((float*)buf0, n, kind == 5 ? -1 : 63, 4);
                w = 4.0 * (double)n;
                break;
            }
            default:
                break;
        }
    };
    if (kind < 0 || kind > 6) return 3;
    launch();
    if (hipEventRecord(e0, stream) != hipSuccess) return 4;
    for (int r = 0; r < reps; ++r) launch();
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 5;
    float t = 0.f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return 6;
    *ms = t;
    *work = w * reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

}  // extern "C"
