// Microbenchmarks of the two on-chip resources that bound the samplers: the float32 vector
// ALU (fused multiply-adds per lane per cycle) and the LDS read bandwidth (bytes per CU per
// cycle) for the access widths and sharing patterns the samplers use.  Built into its own
// small library (libasm_micro.so); bench.py --micro reports the rates.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// 16 independent fused multiply-add chains per thread
__global__ __launch_bounds__(256) void k_valu(int iters, float x, float y, float *sink) {
    float a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = threadIdx.x * 1e-3f + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = fmaf(a[k], x, y);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += a[k];
    if (s == 1234.5f) sink[blockIdx.x] = s;   // keeps the chains live
}

// LDS reads of W bytes per lane (W = 4, 8, 16) in rows of 64 lanes: `share` lanes in a row
// read the same word (share = 1: every lane its own word; 4: the four 16-lane groups of a
// wavefront read the same 16 words, as the samplers' chains read one mode row).  Eight
// independent reads per iteration, addresses advancing by one row each iteration.
template <int W>
__global__ __launch_bounds__(256) void k_lds(int iters, int share, float *sink) {
    constexpr int WORDS = 16384;   // 64 KiB
    __shared__ __align__(16) uint32_t buf[WORDS];
    for (int i = threadIdx.x; i < WORDS; i += blockDim.x) buf[i] = i * 2654435761u;
    __syncthreads();
    const int lane = threadIdx.x % 64;
    const int col = (share == 1 ? lane : lane % (64 / share)) * (W / 4);
    const int rowlen = 64 * (W / 4);
    uint32_t acc = 0;
    int base = (threadIdx.x / 64) * rowlen * 8;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = (base + k * rowlen + col) & (WORDS - 1);
            if constexpr (W == 4) {
                acc ^= buf[idx];
            } else if constexpr (W == 8) {
                const uint2 v = *reinterpret_cast<const uint2 *>(buf + idx);
                acc ^= v.x + v.y;
            } else {
                const uint4 v = *reinterpret_cast<const uint4 *>(buf + idx);
                acc ^= (v.x + v.y) ^ (v.z + v.w);
            }
        }
        base += rowlen;
    }
    if (acc == 0x12345678u) sink[blockIdx.x] = (float)acc;
}

// 16 independent float64 fused multiply-add chains per thread
__global__ __launch_bounds__(256) void k_valu64(int iters, double x, double y, float *sink) {
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = threadIdx.x * 1e-3 + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = fma(a[k], x, y);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += a[k];
    if (s == 1234.5) sink[blockIdx.x] = (float)s;
}

// float64 MFMA 16x16x4: 8 independent accumulators per wavefront
typedef double d4m __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_mfma64(int iters, float *sink) {
    d4m acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = d4m{0, 0, 0, 0};
    const double a = 1e-3 * (threadIdx.x % 64), b = 0.999;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (s == 1234.5) sink[blockIdx.x] = (float)s;
}

// HBM: dst = src over n float4 words, grid-stride
__global__ __launch_bounds__(256) void k_copy(const float4 *src, float4 *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

// kind 4: float64 VALU (16 fused multiply-adds per thread per iteration); kind 5: float64 MFMA
// (8 MFMA f64 16x16x4 per wavefront per iteration); kind 6: a copy of n = iters float4 words
// from src to dst (device buffers of at least that size), grid x 256 threads.  As micro_run.
int micro_run2(int kind, int iters, int grid, const void *src, void *dst, float *sink, double *ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return (int)e;
    for (int rep = 0; rep < 2; ++rep) {
        if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) return (int)e;
        if (kind == 4)
            hipLaunchKernelGGL(k_valu64, dim3(grid), dim3(256), 0, nullptr, iters, 0.999, 1e-3, sink);
        else if (kind == 5)
            hipLaunchKernelGGL(k_mfma64, dim3(grid), dim3(256), 0, nullptr, iters, sink);
        else if (kind == 6)
            hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, nullptr, static_cast<const float4 *>(src),
                               static_cast<float4 *>(dst), (int64_t)iters);
        else
            return (int)hipErrorInvalidValue;
        if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) return (int)e;
    }
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return (int)e;
    float t = 0.0f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return (int)e;
    *ms = t;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (int)hipGetLastError();
}

// kind 0: VALU (16 fused multiply-adds per thread per iteration); kind 1, 2, 3: LDS reads of
// 4, 8, 16 bytes per lane (eight per iteration), `share` lanes reading each word.  Times one
// launch of grid x 256 threads with HIP events on the null stream; writes the milliseconds.
// sink: device, >= grid floats.  Returns 0, or the HIP error code.
int micro_run(int kind, int iters, int grid, int share, float *sink, double *ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return (int)e;
    for (int rep = 0; rep < 2; ++rep) {   // the first launch warms up
        if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) return (int)e;
        if (kind == 0)
            hipLaunchKernelGGL(k_valu, dim3(grid), dim3(256), 0, nullptr, iters, 0.999f, 1e-3f, sink);
        else if (kind == 1)
            hipLaunchKernelGGL(k_lds<4>, dim3(grid), dim3(256), 0, nullptr, iters, share, sink);
        else if (kind == 2)
            hipLaunchKernelGGL(k_lds<8>, dim3(grid), dim3(256), 0, nullptr, iters, share, sink);
        else if (kind == 3)
            hipLaunchKernelGGL(k_lds<16>, dim3(grid), dim3(256), 0, nullptr, iters, share, sink);
        else
            return (int)hipErrorInvalidValue;
        if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) return (int)e;
    }
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return (int)e;
    float t = 0.0f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return (int)e;
    *ms = t;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (int)hipGetLastError();
}

}  // extern "C"
