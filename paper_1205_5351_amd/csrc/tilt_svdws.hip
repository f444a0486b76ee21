// SVD with warm start (Sec. 5, Alg. 2; derivatives of Appendix A): one
// Cayley step from the previous decomposition, for a batch of matrices of
// one shape, one workgroup per matrix.
//
// Given U (m x n, orthonormal columns), Sigma (n) and V (n x n, orthogonal)
// of the previous matrix and the next matrix M (m >= n), with
// X = U Sigma V^T:
//   P_U = X M^T - M X^T (m x m, skew, rank <= 2n)
//   P_V = X^T M - M^T X (n x n, skew)
//   P_Sigma = Sigma - diag(U^T M V)
// The step size is t* = -f'(0)/f''(0) of the second-order model of
// f(t) = 1/2 ||M - U(t) Sigma(t) V(t)^T||_F^2, with the closed forms
//   h0 = M - X, h1 = P_U X + U P_Sigma V^T - X P_V,
//   Z = h1 + U P_Sigma V^T, h2 = -P_U Z + Z P_V,
//   f'(0) = <h0, h1>, f''(0) = <h1, h1> + <h0, h2>.
// P_U is never formed: P_U Y = X (M^T Y) - M (X^T Y).  The m x m Cayley
// factor is applied through the Sherman-Morrison-Woodbury identity with
// P_U = A B^T, A = [X, -M], B = [M, X] (m x 2n) and c = t/2:
//   (I + c P_U)^{-1} (I - c P_U) U = 2 (I + c A B^T)^{-1} U - U
//                                 = U - t A W,   (I_2n + c B^T A) W = B^T U,
// a 2n x 2n system; V(t) solves (I + c P_V) V(t) = (I - c P_V) V (n x n).
// Sigma(t) = Sigma - t P_Sigma.  When f''(0) <= 0 the quadratic model has
// no minimum: no step is taken (status 1) and the caller computes a full
// SVD, as Alg. 2 does when the matrices differ too much.
//
// FP32 data, FP32 products with FP32 accumulation (fmaf), FP64 for the
// inner products f'(0), f''(0), f(0), f(t); LU with partial pivoting for
// both systems.  Matrices are row-major; every workspace array lives in
// the per-matrix scratch the host hands over.

#include <hip/hip_runtime.h>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"
#include <cmath>
#include <vector>

namespace tilt {

namespace {

struct SvdwsDims {
    int m, n;
};

// C (r x c) = op(A) op(B) over k, all row-major in device memory, with
// A^T taken when TA (A stored k x r) and B^T when TB (B stored c x k);
// alpha scales the product, beta the old C (beta = 0: C is not read).
template <bool TA, bool TB>
__device__ void gemm(int r, int c, int k, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                     float alpha, float beta) {
    for (int e = threadIdx.x; e < r * c; e += NT) {
        const int i = e / c, j = e - i * c;
        float acc = 0.f;
        for (int q = 0; q < k; ++q) {
            const float a = TA ? A[(size_t)q * lda + i] : A[(size_t)i * lda + q];
            const float b = TB ? B[(size_t)j * ldb + q] : B[(size_t)q * ldb + j];
            acc = fmaf(a, b, acc);
        }
        const float old = beta != 0.f ? beta * C[(size_t)i * ldc + j] : 0.f;
        C[(size_t)i * ldc + j] = fmaf(alpha, acc, old);
    }
    __syncthreads();
}

// Sum over the workgroup of a per-thread FP64 value (same bits everywhere).
__device__ double wg_sum(double v) {
    __shared__ double part[NWAVE];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NWAVE; ++w) s += part[w];
    __syncthreads();
    return s;
}

// <P, Q> over r x c row-major arrays (FP64 accumulation).
__device__ double dot_mat(const float* P, const float* Q, int count) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < count; e += NT) acc += (double)P[e] * (double)Q[e];
    return wg_sum(acc);
}

// Solve T X = R in place (T: N x N, R: N x nrhs, both row-major in device
// memory; T is overwritten by its LU factors, R by the solution), by
// Gaussian elimination with partial pivoting.  Returns false if a pivot is
// zero.
__device__ bool lu_solve(float* T, int N, float* R, int nrhs) {
    __shared__ int sh_piv;
    __shared__ float sh_val[NT];
    __shared__ int sh_idx[NT];
    for (int k = 0; k < N; ++k) {
        // pivot: largest |T[i][k]|, i >= k (ties to the smaller row)
        float best = -1.f;
        int bi = k;
        for (int i = k + threadIdx.x; i < N; i += NT) {
            const float v = fabsf(T[(size_t)i * N + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        sh_val[threadIdx.x] = best;
        sh_idx[threadIdx.x] = bi;
        __syncthreads();
        if (threadIdx.x == 0) {
            float bv = -1.f;
            int b = k;
            for (int u = 0; u < NT; ++u)
                if (sh_val[u] > bv || (sh_val[u] == bv && sh_idx[u] < b)) {
                    bv = sh_val[u];
                    b = sh_idx[u];
                }
            sh_piv = bv > 0.f ? b : -1;
        }
        __syncthreads();
        const int p = sh_piv;
        if (p < 0) return false;
        if (p != k) {
            for (int j = threadIdx.x; j < N; j += NT) {
                const float a = T[(size_t)k * N + j];
                T[(size_t)k * N + j] = T[(size_t)p * N + j];
                T[(size_t)p * N + j] = a;
            }
            for (int j = threadIdx.x; j < nrhs; j += NT) {
                const float a = R[(size_t)k * nrhs + j];
                R[(size_t)k * nrhs + j] = R[(size_t)p * nrhs + j];
                R[(size_t)p * nrhs + j] = a;
            }
        }
        __syncthreads();
        const float piv = T[(size_t)k * N + k];
        // multipliers, then the trailing update of T and R
        for (int i = k + 1 + threadIdx.x; i < N; i += NT) T[(size_t)i * N + k] /= piv;
        __syncthreads();
        const int rows = N - k - 1;
        const int cols = N - k - 1 + nrhs;
        for (int e = threadIdx.x; e < rows * cols; e += NT) {
            const int i = k + 1 + e / cols, jj = e - (e / cols) * cols;
            const float l = T[(size_t)i * N + k];
            if (jj < N - k - 1) {
                const int j = k + 1 + jj;
                T[(size_t)i * N + j] = fmaf(-l, T[(size_t)k * N + j], T[(size_t)i * N + j]);
            } else {
                const int j = jj - (N - k - 1);
                R[(size_t)i * nrhs + j] = fmaf(-l, R[(size_t)k * nrhs + j], R[(size_t)i * nrhs + j]);
            }
        }
        __syncthreads();
    }
    // back substitution, one right-hand side per thread
    for (int j = threadIdx.x; j < nrhs; j += NT) {
        for (int i = N - 1; i >= 0; --i) {
            float s = R[(size_t)i * nrhs + j];
            for (int q = i + 1; q < N; ++q) s = fmaf(-T[(size_t)i * N + q], R[(size_t)q * nrhs + j], s);
            R[(size_t)i * nrhs + j] = s / T[(size_t)i * N + i];
        }
    }
    __syncthreads();
    return true;
}

// Words of per-matrix scratch.
__host__ __device__ inline size_t svdws_scratch_words(int m, int n) {
    return (size_t)8 * m * n + (size_t)4 * n * n + (size_t)4 * n * n + (size_t)2 * n * n + (size_t)2 * n * n +
           (size_t)2 * n;
}

__global__ void __launch_bounds__(NT) k_svdws(SvdwsJob* jobs, int m, int n, float* scratch) {
    SvdwsJob& jb = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    float* w = scratch + (size_t)blockIdx.x * svdws_scratch_words(m, n);
    float* X = w;           // m x n
    float* H0 = X + mn;     // M - X
    float* H1 = H0 + mn;    // h1
    float* Zp = H1 + mn;    // Z = h1 + U P_S V^T
    float* H2 = Zp + mn;    // h2
    float* T1 = H2 + mn;    // m x n temporaries
    float* T2 = T1 + mn;
    float* UPV = T2 + mn;   // U P_S V^T
    float* K = UPV + mn;    // 2n x 2n
    float* G1 = K + 4 * nn;  // M^T X (n x n)
    float* G2 = G1 + nn;     // X^T X
    float* PV = G2 + nn;     // P_V
    float* G3 = PV + nn;     // n x n temporaries
    float* WZ = G3 + nn;     // 2n x n: B^T U, then W
    float* VS = WZ + 2 * nn; // n x n system of V(t)
    float* VR = VS + nn;     // its right-hand side, then V(t)
    float* PS = VR + nn;     // P_Sigma (n)
    float* Sv = PS + n;      // Sigma as given (n)
    const float* U = jb.U;
    const float* V = jb.V;
    const float* M = jb.M;
    for (int j = tid; j < n; j += NT) Sv[j] = jb.S[j];
    __syncthreads();
    // X = U Sigma V^T: T1 = U diag(Sigma), X = T1 V^T
    for (size_t e = tid; e < mn; e += NT) T1[e] = U[e] * Sv[e % n];
    __syncthreads();
    gemm<false, true>(m, n, n, T1, n, V, n, X, n, 1.f, 0.f);
    for (size_t e = tid; e < mn; e += NT) H0[e] = M[e] - X[e];
    // P_Sigma = Sigma - diag(U^T M V): T2 = M V, d_j = sum_i U_ij T2_ij
    gemm<false, false>(m, n, n, M, n, V, n, T2, n, 1.f, 0.f);
    for (int j = tid; j < n; j += NT) {
        float d = 0.f;
        for (int i = 0; i < m; ++i) d = fmaf(U[(size_t)i * n + j], T2[(size_t)i * n + j], d);
        PS[j] = Sv[j] - d;
    }
    __syncthreads();
    // U P_Sigma V^T
    for (size_t e = tid; e < mn; e += NT) T1[e] = U[e] * PS[e % n];
    __syncthreads();
    gemm<false, true>(m, n, n, T1, n, V, n, UPV, n, 1.f, 0.f);
    // G1 = M^T X, G2 = X^T X, P_V = G1^T - G1
    gemm<true, false>(n, n, m, M, n, X, n, G1, n, 1.f, 0.f);
    gemm<true, false>(n, n, m, X, n, X, n, G2, n, 1.f, 0.f);
    for (size_t e = tid; e < nn; e += NT) {
        const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
        PV[e] = G1[(size_t)j * n + i] - G1[e];
    }
    __syncthreads();
    // h1 = P_U X + U P_S V^T - X P_V, with P_U X = X G1 - M G2
    gemm<false, false>(m, n, n, X, n, G1, n, H1, n, 1.f, 0.f);
    gemm<false, false>(m, n, n, M, n, G2, n, H1, n, -1.f, 1.f);
    gemm<false, false>(m, n, n, X, n, PV, n, H1, n, -1.f, 1.f);
    for (size_t e = tid; e < mn; e += NT) H1[e] += UPV[e];
    __syncthreads();
    for (size_t e = tid; e < mn; e += NT) Zp[e] = H1[e] + UPV[e];
    __syncthreads();
    // h2 = -P_U Z + Z P_V, P_U Z = X (M^T Z) - M (X^T Z)
    gemm<true, false>(n, n, m, M, n, Zp, n, G3, n, 1.f, 0.f);   // G3 = M^T Z
    gemm<false, false>(m, n, n, X, n, G3, n, H2, n, -1.f, 0.f);  // H2 = -X M^T Z
    gemm<true, false>(n, n, m, X, n, Zp, n, G3, n, 1.f, 0.f);   // G3 = X^T Z
    gemm<false, false>(m, n, n, M, n, G3, n, H2, n, 1.f, 1.f);   // H2 += M X^T Z
    gemm<false, false>(m, n, n, Zp, n, PV, n, H2, n, 1.f, 1.f);  // H2 += Z P_V
    const double f1 = dot_mat(H0, H1, (int)mn);
    const double f2 = dot_mat(H1, H1, (int)mn) + dot_mat(H0, H2, (int)mn);
    const double f0 = 0.5 * dot_mat(H0, H0, (int)mn);
    if (!(f2 > 0.0)) {
        // no minimum along the curve: hand back the previous decomposition
        for (size_t e = tid; e < mn; e += NT) jb.U_out[e] = U[e];
        for (size_t e = tid; e < nn; e += NT) jb.V_out[e] = V[e];
        for (int j = tid; j < n; j += NT) jb.S_out[j] = Sv[j];
        if (tid == 0) {
            jb.t = 0.0;
            jb.f0 = f0;
            jb.ft = f0;
            jb.status = 1;
        }
        return;
    }
    const double t = -f1 / f2;
    const float tf = (float)t, c = (float)(0.5 * t);
    // K = B^T A = [[M^T X, -M^T M], [X^T X, -X^T M]]  (2n x 2n), then I + c K
    const int N2 = 2 * n;
    gemm<true, false>(n, n, m, M, n, M, n, G3, n, 1.f, 0.f);    // G3 = M^T M
    for (size_t e = tid; e < 4 * nn; e += NT) {
        const int i = (int)(e / N2), j = (int)(e - (size_t)i * N2);
        float v;
        if (i < n)
            v = j < n ? G1[(size_t)i * n + j] : -G3[(size_t)i * n + (j - n)];
        else
            v = j < n ? G2[(size_t)(i - n) * n + j] : -G1[(size_t)(j - n) * n + (i - n)];  // -X^T M = -(M^T X)^T
        K[e] = c * v + (i == j ? 1.f : 0.f);
    }
    __syncthreads();
    // right-hand side B^T U = [M^T U; X^T U]
    gemm<true, false>(n, n, m, M, n, U, n, WZ, n, 1.f, 0.f);
    gemm<true, false>(n, n, m, X, n, U, n, WZ + nn, n, 1.f, 0.f);
    bool ok = lu_solve(K, N2, WZ, n);
    // U(t) = U - t (X W1 - M W2)
    if (ok) {
        gemm<false, false>(m, n, n, X, n, WZ, n, T1, n, 1.f, 0.f);
        gemm<false, false>(m, n, n, M, n, WZ + nn, n, T1, n, -1.f, 1.f);
        for (size_t e = tid; e < mn; e += NT) jb.U_out[e] = fmaf(-tf, T1[e], U[e]);
        __syncthreads();
    }
    // V(t): (I + c P_V) V(t) = (I - c P_V) V
    if (ok) {
        for (size_t e = tid; e < nn; e += NT) {
            const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
            VS[e] = c * PV[e] + (i == j ? 1.f : 0.f);
        }
        gemm<false, false>(n, n, n, PV, n, V, n, VR, n, -c, 0.f);
        for (size_t e = tid; e < nn; e += NT) VR[e] += V[e];
        __syncthreads();
        ok = lu_solve(VS, n, VR, n);
    }
    if (!ok) {
        if (tid == 0) jb.status = -4;
        return;
    }
    for (size_t e = tid; e < nn; e += NT) jb.V_out[e] = VR[e];
    for (int j = tid; j < n; j += NT) jb.S_out[j] = fmaf(-tf, PS[j], Sv[j]);
    __syncthreads();
    // f(t) = 1/2 ||M - U(t) Sigma(t) V(t)^T||^2, and the shrinkage
    for (size_t e = tid; e < mn; e += NT) T1[e] = jb.U_out[e] * jb.S_out[e % n];
    __syncthreads();
    gemm<false, true>(m, n, n, T1, n, VR, n, T2, n, 1.f, 0.f);
    for (size_t e = tid; e < mn; e += NT) T1[e] = M[e] - T2[e];
    __syncthreads();
    const double ft = 0.5 * dot_mat(T1, T1, (int)mn);
    if (jb.A_out) {
        // A = U(t) T_eps(Sigma(t)) V(t)^T with the signed soft threshold
        const float eps = jb.eps;
        for (size_t e = tid; e < mn; e += NT) {
            const float s = jb.S_out[e % n];
            const float sh = s > eps ? s - eps : (s < -eps ? s + eps : 0.f);
            T1[e] = jb.U_out[e] * sh;
        }
        __syncthreads();
        gemm<false, true>(m, n, n, T1, n, VR, n, jb.A_out, n, 1.f, 0.f);
    }
    if (tid == 0) {
        jb.t = t;
        jb.f0 = f0;
        jb.ft = ft;
        jb.status = 0;
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
    int worst = TILT_OK;
    for (int i = 0; i < count; ++i) {
        if (t_out) t_out[i] = jobs[i].t;
        if (f0_out) f0_out[i] = jobs[i].f0;
        if (ft_out) ft_out[i] = jobs[i].ft;
        if (status) status[i] = jobs[i].status;
        worst = worse(worst, jobs[i].status == 1 ? TILT_WARN_MAXITER : jobs[i].status);
    }
    return worst < 0 ? worst : TILT_OK;
}

