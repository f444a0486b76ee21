// Machine peaks for the rooflines of the solver's kernels, measured with the
// same compiler flags as the solver (no packed FP32): HBM stream copy, LDS
// 16-byte reads, FP32 vector FMA and FP32 matrix-core (MFMA) throughput.
// Not part of the method; the kernels only touch the buffers the caller
// passes (copy) or their own registers and LDS.

#include <hip/hip_runtime.h>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"

namespace tilt {
namespace {

constexpr int kPeakThreads = 256;
constexpr int kLdsFloat4 = 2048;  // 32 KiB of LDS per workgroup

// dst[i] = src[i] for i < n (float4), grid-stride over 4 workgroups per
// compute unit: the fastest of the copy forms measured on MI355X (1-8 loads
// in flight per thread, 4-64 workgroups per unit, plain or nontemporal
// accesses: 4.3-5.5 TB/s for 2 GiB).
__global__ __launch_bounds__(kPeakThreads) void k_peak_copy(const float4* __restrict__ src,
                                                           float4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kPeakThreads;
    for (size_t i = (size_t)blockIdx.x * kPeakThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Each lane reads 16 bytes per step from LDS; consecutive lanes read
// consecutive 16-byte words (no bank conflicts).  The words are folded with
// integer XORs (one VALU operation per 4-byte word, as in the Jacobi where
// every loaded float feeds at least one multiply-add), so the figure is the
// LDS read rate a kernel consuming what it reads can reach; out gets one
// word per thread.
__global__ __launch_bounds__(kPeakThreads) void k_peak_lds(unsigned* __restrict__ out, int iters) {
    __shared__ uint4 buf[kLdsFloat4];
    const int t = threadIdx.x;
    for (int i = t; i < kLdsFloat4; i += kPeakThreads) buf[i] = make_uint4(i, 3 * i + 1, 5 * i + 2, 7 * i + 3);
    __syncthreads();
    unsigned acc = 0;
    int base = t;
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint4 v = buf[(base + u * kPeakThreads) & (kLdsFloat4 - 1)];
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
        base = (base + 8 * kPeakThreads + 64) & (kLdsFloat4 - 1);
    }
    out[(size_t)blockIdx.x * kPeakThreads + t] = acc;
}

// Eight independent FP32 FMA chains per lane (2 flops each per step).
__global__ __launch_bounds__(kPeakThreads) void k_peak_fma(float* __restrict__ out, int iters) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = 1e-3f * (float)(threadIdx.x + u);
    const float a = 0.999f, b = 1e-4f;
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = fmaf(x[u], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
    out[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

typedef float peak_floatx4 __attribute__((ext_vector_type(4)));

// Four independent FP32 MFMA 16x16x4 accumulators per wavefront (2 x 16 x 16
// x 4 flops per instruction and wavefront).
__global__ __launch_bounds__(kPeakThreads) void k_peak_mfma(float* __restrict__ out, int iters) {
    peak_floatx4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = peak_floatx4{0.f, 0.f, 0.f, 0.f};
    const float a = 1e-3f * (float)(threadIdx.x & 63), b = 0.5f;
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[u], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
    out[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace tilt

using namespace tilt;

extern "C" {

int tilt_peak_probe(int kind, const void* src, void* dst, size_t bytes, int iters, double* ms_out,
                    double* work_out, void* hip_stream) {
    if (!dst || !ms_out || !work_out || kind < 0 || kind > 3) return TILT_ERR_ARG;
    if (kind == 0 && (!src || bytes < 16)) return TILT_ERR_ARG;
    if (kind != 0 && iters < 1) return TILT_ERR_ARG;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    // 8 workgroups of 256 threads per compute unit for the compute probes
    const int grid = 8 * cus;
    const size_t out_bytes = (size_t)grid * kPeakThreads * sizeof(float);
    if (kind != 0 && bytes < out_bytes) return TILT_ERR_ARG;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TILT_ERR_DEVICE;
    }
    double work = 0.0;
    hipError_t err = hipEventRecord(e0, stream);
    if (err == hipSuccess) {
        switch (kind) {
            case 0: {
                const size_t n = bytes / 16;
                k_peak_copy<<<4 * cus, kPeakThreads, 0, stream>>>(static_cast<const float4*>(src),
                                                                   static_cast<float4*>(dst), n);
                work = 2.0 * 16.0 * (double)n;  // bytes read + written
                break;
            }
            case 1:
                k_peak_lds<<<grid, kPeakThreads, 0, stream>>>(static_cast<unsigned*>(dst), iters);
                work = 16.0 * 8.0 * (double)iters * grid * kPeakThreads;  // LDS bytes read
                break;
            case 2:
                k_peak_fma<<<grid, kPeakThreads, 0, stream>>>(static_cast<float*>(dst), iters);
                work = 2.0 * 8.0 * (double)iters * grid * kPeakThreads;  // flops
                break;
            default:
                k_peak_mfma<<<grid, kPeakThreads, 0, stream>>>(static_cast<float*>(dst), iters);
                work = 4.0 * 2.0 * 16 * 16 * 4 * (double)iters * grid * (kPeakThreads / 64);  // flops
                break;
        }
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return host::record_hip_error(err, "peak probe", __LINE__);
    *ms_out = ms;
    *work_out = work;
    return TILT_OK;
}

}  // extern "C"
