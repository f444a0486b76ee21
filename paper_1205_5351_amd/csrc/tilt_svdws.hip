// SVD with warm start (Sec. 5, Alg. 2; derivatives of Appendix A) as a
// component entry point: one Cayley step per matrix for a batch of
// matrices of one shape, one workgroup per matrix (the step itself is in
// tilt_svdws.inc).

#include <hip/hip_runtime.h>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"
#include <cmath>
#include <vector>

namespace tilt {

namespace {

#include "tilt_svdws.inc"

__global__ void __launch_bounds__(NT) k_svdws(SvdwsJob* jobs, int m, int n, float* scratch) {
    SvdwsJob& jb = jobs[blockIdx.x];
    float* w = scratch + (size_t)blockIdx.x * svdws_scratch_words(m, n);
    double t, f0, ft;
    const int st = svdws_step(m, n, jb.U, jb.S, jb.V, jb.M, jb.U_out, jb.S_out, jb.V_out, jb.A_out, jb.eps, w, t, f0,
                              ft);
    if (threadIdx.x == 0) {
        jb.t = t;
        jb.f0 = f0;
        jb.ft = ft;
        jb.status = st;
    }
}

}  // namespace

size_t svdws_scratch_bytes(int m, int n) { return sizeof(float) * svdws_scratch_words(m, n); }

hipError_t launch_svdws(SvdwsJob* jobs, int count, int m, int n, float* scratch, hipStream_t s) {
    hipLaunchKernelGGL(k_svdws, dim3(count), dim3(NT), 0, s, jobs, m, n, scratch);
    return hipGetLastError();
}

}  // namespace tilt

using namespace tilt;
using namespace tilt::host;

int tilt_svdws_batch(tilt_ctx* ctx, int count, int m, int n, const float* U, const float* S, const float* V,
                     const float* M, float* U_out, float* S_out, float* V_out, float* A_out, const float* eps,
                     double* t_out, double* f0_out, double* ft_out, int* status, void* hip_stream) {
    if (!ctx || count < 0 || n < 1 || m < n || n > 256 || m > 4096) return TILT_ERR_ARG;
    if (!U || !S || !V || !M || !U_out || !S_out || !V_out || (A_out && !eps)) return TILT_ERR_ARG;
    if (count == 0) return TILT_OK;
    if (A_out)
        for (int i = 0; i < count; ++i)
            if (!std::isfinite(eps[i]) || eps[i] < 0.f) return TILT_ERR_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    std::vector<SvdwsJob> jobs(count);
    for (int i = 0; i < count; ++i) {
        SvdwsJob& j = jobs[i];
        j.U = U + i * mn;
        j.S = S + (size_t)i * n;
        j.V = V + i * nn;
        j.M = M + i * mn;
        j.U_out = U_out + i * mn;
        j.S_out = S_out + (size_t)i * n;
        j.V_out = V_out + i * nn;
        j.A_out = A_out ? A_out + i * mn : nullptr;
        j.eps = A_out ? eps[i] : 0.f;
        j.status = -3;
        j.t = j.f0 = j.ft = 0.0;
    }
    if (ctx->jobs.reserve(sizeof(SvdwsJob) * count) != hipSuccess ||
        ctx->scratch.reserve(svdws_scratch_bytes(m, n) * count) != hipSuccess)
        return TILT_ERR_NOMEM;
    HIP_TRY(hipMemcpyAsync(ctx->jobs.p, jobs.data(), sizeof(SvdwsJob) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(launch_svdws(reinterpret_cast<SvdwsJob*>(ctx->jobs.p), count, m, n,
                         reinterpret_cast<float*>(ctx->scratch.p), stream));
    HIP_TRY(hipMemcpyAsync(jobs.data(), ctx->jobs.p, sizeof(SvdwsJob) * count, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    // status 1 (no step: f''(0) <= 0) is the caller's cue for a full SVD,
    // reported per matrix only; the return value carries the worst error
    int worst = TILT_OK;
    for (int i = 0; i < count; ++i) {
        if (t_out) t_out[i] = jobs[i].t;
        if (f0_out) f0_out[i] = jobs[i].f0;
        if (ft_out) ft_out[i] = jobs[i].ft;
        if (status) status[i] = jobs[i].status;
        if (jobs[i].status < 0) worst = worse(worst, jobs[i].status);
    }
    return worst;
}

