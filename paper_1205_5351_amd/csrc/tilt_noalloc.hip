// Allocation-free singular value shrinkage: tilt_svt_batch_noalloc.
//
// Same computation and kernels as tilt_svt_batch (the one-sided Jacobi SVT
// of the solver), but every device buffer beyond the caller's inputs and
// outputs -- the job table, the per-job work counters, the ranks and the
// per-job working planes -- lives in one fixed device array, `scratch`,
// declared below.  Its device address is taken once per device with
// hipGetSymbolAddress, on the first call made with that device current;
// host code uses that address only, never the array's name.  No call of
// this entry point allocates device memory.
//
// Every call on a device shares that device's array, which keeps the
// previous call's contents; calls that overlap on one device race.  Nothing
// here needs the array to start at zero: each kernel writes every word it
// reads later in the same call.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"

namespace tilt {

// 64 MiB per device (float words).
constexpr size_t kNoallocWords = (size_t)16 << 20;

static __device__ __align__(256) float scratch[kNoallocWords];

namespace {

// Job table of one call: matrix i of the batch at M + i m n, A + i m n,
// sigma + i min(m, n), shrinkage threshold eps[i].
__global__ void __launch_bounds__(NT) k_noalloc_jobs(const float* M, float* A, float* sigma, int m, int n,
                                                     const float* eps, SvtJob* jobs, int count) {
    const size_t mn = (size_t)m * n;
    const int k = m < n ? m : n;
    for (int i = blockIdx.x * NT + threadIdx.x; i < count; i += gridDim.x * NT) {
        SvtJob j;
        j.M = M + (size_t)i * mn;
        j.A = A + (size_t)i * mn;
        j.sigma = sigma ? sigma + (size_t)i * k : nullptr;
        j.m = m;
        j.n = n;
        j.eps = eps[i];
        j.pad = 0;
        jobs[i] = j;
    }
}

// Ranks (kept singular values) per job and the counters summed over the
// batch in job order: sweeps, pairs, rotations, kept rows.
__global__ void __launch_bounds__(NT) k_noalloc_tally(const long long* counters, int count, int* ranks,
                                                      long long* sums) {
    for (int i = threadIdx.x; i < count; i += NT) ranks[i] = (int)counters[4 * i + 3];
    if (threadIdx.x == 0) {
        long long s[4] = {0, 0, 0, 0};
        for (int i = 0; i < count; ++i)
            for (int c = 0; c < 4; ++c) s[c] += counters[4 * i + c];
        for (int c = 0; c < 4; ++c) sums[c] = s[c];
    }
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken once).
hipError_t scratch_address(int device, float** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = static_cast<float*>(p);
    }
    *out = g_ptr[device];
    return hipSuccess;
}

size_t align_words(size_t w) { return (w + 63) & ~(size_t)63; }

}  // namespace
}  // namespace tilt

using namespace tilt;
using namespace tilt::host;

static_assert(kNoallocWords * sizeof(float) == TILT_SVT_NOALLOC_BYTES, "the header states the limit");

int tilt_svt_batch_noalloc(const float* M, float* A, float* sigma, int count, int m, int n, const float* eps,
                           const tilt_params* prm, int* ranks, tilt_counters* counters, void* hip_stream) {
    if (!M || !A || !eps || !prm || count < 0 || m < 1 || n < 1) return TILT_ERR_ARG;
    int st = validate_params(prm);
    if (st != TILT_OK) return st;
    if (count == 0) return TILT_OK;
    for (int i = 0; i < count; ++i)
        if (!std::isfinite(eps[i]) || eps[i] < 0.f) return TILT_ERR_ARG;
    ShapeCfg sc{};
    st = shape_config(m, n, &sc);
    if (st != TILT_OK) return st;
    // layout of the words used: eps | jobs | counters (4 per job) | ranks |
    // sums (4) | working planes (per job: two nc x ldg planes, plus the
    // ncp x ldg Jacobi plane when tiled)
    const size_t np = (size_t)sc.nc * sc.ldg;
    const size_t per_job = 2 * np + (sc.sb > 0 ? (size_t)sc.ncp * sc.ldg : 0);
    const size_t w_eps = align_words((size_t)count);
    const size_t w_jobs = align_words((sizeof(SvtJob) * (size_t)count + 3) / 4);
    const size_t w_cnt = align_words((size_t)8 * count);
    const size_t w_ranks = align_words((size_t)count);
    const size_t w_sums = 64;
    const size_t need = w_eps + w_jobs + w_cnt + w_ranks + w_sums + per_job * (size_t)count;
    if (need > kNoallocWords) return TILT_ERR_TOO_LARGE;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return TILT_ERR_DEVICE;
    float* base = nullptr;
    HIP_TRY(scratch_address(dev, &base));
    float* d_eps = base;
    SvtJob* d_jobs = reinterpret_cast<SvtJob*>(d_eps + w_eps);
    long long* d_cnt = reinterpret_cast<long long*>(reinterpret_cast<float*>(d_jobs) + w_jobs);
    int* d_ranks = reinterpret_cast<int*>(reinterpret_cast<float*>(d_cnt) + w_cnt);
    long long* d_sums = reinterpret_cast<long long*>(reinterpret_cast<float*>(d_ranks) + w_ranks);
    float* d_planes = reinterpret_cast<float*>(d_sums) + w_sums;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(d_eps, eps, sizeof(float) * count, hipMemcpyHostToDevice, stream));
    const int fill_grid = std::min(1024, (count + NT - 1) / NT);
    hipLaunchKernelGGL(k_noalloc_jobs, dim3(fill_grid), dim3(NT), 0, stream, M, A, sigma, m, n, d_eps, d_jobs,
                       count);
    HIP_TRY(hipGetLastError());
    const SvtShape shape{sc.cfg, sc.ld, sc.tb, sc.sb, sc.nsb, sc.ncp};
    HIP_TRY(launch_svt_jobs(d_jobs, count, shape, prm->jacobi_tol, prm->max_sweeps, d_cnt, d_planes, sc.lds, stream));
    hipLaunchKernelGGL(k_noalloc_tally, dim3(1), dim3(NT), 0, stream, d_cnt, count, d_ranks, d_sums);
    HIP_TRY(hipGetLastError());
    long long sums[4] = {0, 0, 0, 0};
    if (ranks) HIP_TRY(hipMemcpyAsync(ranks, d_ranks, sizeof(int) * count, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(sums, d_sums, sizeof(sums), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (counters) {
        std::memset(counters, 0, sizeof(*counters));
        counters->svt_calls = count;
        counters->jacobi_sweeps = sums[0];
        counters->jacobi_pairs = sums[1];
        counters->jacobi_rotations = sums[2];
        counters->recon_rows = sums[3];
    }
    return TILT_OK;
}
