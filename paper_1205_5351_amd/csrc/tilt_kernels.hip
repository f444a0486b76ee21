// HIP kernels for TILT solved by LADMAP with variable warm start (gfx950).
//
// One workgroup of 256 threads owns one patch at a time.  Every step of
// Alg. 1 is a device function that the whole workgroup calls:
//
//   dev_setup    Alg. 1 Step 1 + Sec. 4.3 constraints + Sec. 4.2 warm start:
//                bilinear warp and exact interpolant gradient, normalisation,
//                Jacobian of the normalised warp, reduced Jacobian J~ = J N_Q,
//                orthonormal basis Qb of span(J~) (Cholesky-QR twice, FP64
//                factors), Y <- J~perp Y, R <- J~perp(A + E - I),
//                c = ||J~perp I||_F, mu_0 = 1.25 / ||I||_2.
//   dev_svt      M = A - R - Y/mu and A <- S_{1/mu}(M) (Eqs. A, A_1,
//                S_operator): one-sided Jacobi on the rows of M held in LDS,
//                then S(M) = sum_j (1 - eps/s_j)/s_j^2 (M b_j) b_j^T over the
//                orthogonalised rows b_j with s_j = ||b_j|| > eps.
//   dev_update   N, E <- T_{lam/mu}(N) (Eq. E_1), R <- J~perp(A + E - I),
//                Y <- Y + mu R (Eq. Y), Cond1/Cond2 (Eqs. Cond1, Cond2) and
//                the adaptive penalty (Eqs. mu, rho).
//   dev_dtau     Delta tau = N_Q R^{-1} Qb^T (A + E - I) (Eq. Delta_tau with
//                the constraints eliminated), tau += Delta tau (FP64).
//
// The plain path launches one kernel per step; the batched path runs all
// steps of whole patches in one persistent kernel.  Both call the same
// device functions with the same workgroup shape, so a patch gives the same
// bits either way.

#include "tilt_internal.h"

namespace tilt {

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

__device__ inline float wave_sum_f(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One LDS scratch buffer for every workgroup reduction (one slot per value
// per wavefront).
constexpr int RED_MAX = 24;
__shared__ double tilt_red_scratch[RED_MAX * NWAVE];

// Sum K values over the workgroup; every thread receives the same bits.
template <int K>
__device__ inline void block_sum_f(float (&v)[K]) {
    static_assert(K <= RED_MAX, "reduction too wide");
    float* red = reinterpret_cast<float*>(tilt_red_scratch);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_f(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * NWAVE + w] = v[k];
    }
    __syncthreads();
    // thread k combines the per-wave partials of value k (fixed order)
    if ((int)threadIdx.x < K) {
        const int k = threadIdx.x;
        float s = red[k * NWAVE];
        for (int i = 1; i < NWAVE; ++i) s += red[k * NWAVE + i];
        red[k * NWAVE] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[k * NWAVE];
    __syncthreads();
}

template <int K>
__device__ inline void block_sum_d(double (&v)[K]) {
    static_assert(K <= RED_MAX, "reduction too wide");
    double* red = tilt_red_scratch;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_d(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * NWAVE + w] = v[k];
    }
    __syncthreads();
    // thread k combines the per-wave partials of value k (fixed order)
    if ((int)threadIdx.x < K) {
        const int k = threadIdx.x;
        double s = red[k * NWAVE];
        for (int i = 1; i < NWAVE; ++i) s += red[k * NWAVE + i];
        red[k * NWAVE] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[k * NWAVE];
    __syncthreads();
}

__device__ inline long long block_sum_ll(long long v) {
    long long* red = reinterpret_cast<long long*>(tilt_red_scratch);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[w] = v;
    __syncthreads();
    long long s = 0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Cross-lane moves inside a group of 4 or 8 consecutive lanes (DPP).
__device__ inline float dpp_xor1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline float dpp_xor2(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ inline float dpp_half_mirror(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
}

__device__ inline float dpp_mirror(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
}

// Sum over the LPP (4, 8, 16, 32 or 64) lanes of a group; all lanes get
// identical bits (each step adds two equal partial sums in either order).
// Groups wider than a 16-lane row exchange halves through lane shuffles.
template <int LPP>
__device__ inline float group_sum(float v) {
    v += dpp_xor1(v);
    v += dpp_xor2(v);
    if (LPP >= 8) v += dpp_half_mirror(v);
    if (LPP >= 16) v += dpp_mirror(v);
    if (LPP >= 32) v += __shfl_xor(v, 16, 64);
    if (LPP >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ inline float4 f4(float a) { return make_float4(a, a, a, a); }

// ---------------------------------------------------------------------------
// One-sided Jacobi on the rows of B (LDS), round-robin ordering of blocks
// of BS rows (BS = 1: single rows, BS = 2: pairs of rows).
//
// Rows 0..nc4-1 (nc rounded up to a multiple of 4 with zero rows) with
// stride ld; every row is zero-padded to LPP*(4*NCH + TL) floats so each of
// the LPP lanes of a group reads exactly NCH float4 chunks (lane q owns
// chunks q, q+LPP, ...) and TL single floats after them.  Each round pairs every block with another (circle
// method: the last block is fixed, pair k of round r is (r+k, r-k) mod
// (nb-1)); a group owns one block pair, holds its 2 BS rows in registers
// and rotates its cross pairs -- for BS = 2 in the order (a1,b1), (a2,b2),
// (a1,b2), (a2,b1), plus (a1,a2), (b1,b2) in the first round of a sweep --
// so every pair of rows is met once per sweep.  A pair is rotated when
// |a.b| > tol ||a|| ||b||; the sweeps stop when a whole sweep rotates
// nothing.  Squared row norms are recomputed exactly at the start of each
// sweep and updated through each rotation (||a'||^2 = ||a||^2 - t a.b,
// ||b'||^2 = ||b||^2 + t a.b), so the final sweep, which rotates nothing,
// tests every pair against exact norms.
// ---------------------------------------------------------------------------

struct JacobiStats {
    long long sweeps, pairs, rotations;
};

// Rotation that zeroes a.b for norms al = ||a||^2, be = ||b||^2 and
// ga = a.b (Hestenes / Rutishauser), returned as t = tan of the angle,
// s = sin = t/r and the half-angle tangent tau = s/(1 + c) = t/(1 + r),
// r = sqrt(1 + t^2).  With d = be - al, t = sgn(d) 2 ga/(|d| + sqrt(d^2 +
// 4 ga^2)), the smaller root of the rotation's quadratic.  The rows are
// updated as a' = a - s (b + tau a), b' = b + s (a - tau b), whose effective
// cosine 1 - s tau never rounds to 1 for small angles.  Any t is a valid
// rotation, so t comes straight from hardware estimates; 1/r (reciprocal
// square-root estimate) and tau (reciprocal estimate) each get one Newton
// correction, which keeps the transformation orthogonal to rounding level
// with no systematic shrink or growth of the rows over the thousands of
// rotations of a decomposition.  Four transcendental instructions per pair.
// t = 0 gives s = tau = 0 exactly (and leaves the tracked norms unchanged),
// so a pair that needs no rotation only has its t replaced by 0.
__device__ inline float rotation_tangent(float al, float be, float ga) {
    const float d = be - al;
    const float dd = __builtin_amdgcn_sqrtf(fmaf(d, d, 4.0f * ga * ga));
    return copysignf(1.0f, d) * (2.0f * ga) * __builtin_amdgcn_rcpf(fabsf(d) + dd);
}

__device__ inline void rotation_sin_halftan(float t, float& sn, float& ta) {
    const float q = fmaf(t, t, 1.0f);
    float y = __builtin_amdgcn_rsqf(q);
    y = fmaf(y, fmaf(-0.5f * q * y, y, 0.5f), y);
    const float r = q * y;
    const float op = 1.0f + r;
    const float ro = __builtin_amdgcn_rcpf(op);
    const float h = t * ro;
    sn = t * y;
    ta = fmaf(fmaf(-h, op, t), ro, h);
}

__device__ inline void jacobi_rotation(float al, float be, float ga, float& sn, float& ta, float& tn) {
    tn = rotation_tangent(al, be, ga);
    rotation_sin_halftan(tn, sn, ta);
}

// Rotation test: |a.b| > tol ||a|| ||b||, squared (no square roots).
__device__ inline bool needs_rotation(float ga, float nx, float ny, float tol) {
    return ga * ga > (tol * tol) * (nx * ny);
}

__device__ inline float dot4(const float4& a, const float4& b, float acc) {
    acc = fmaf(a.x, b.x, acc);
    acc = fmaf(a.y, b.y, acc);
    acc = fmaf(a.z, b.z, acc);
    acc = fmaf(a.w, b.w, acc);
    return acc;
}

// A lane's part of one row: NCH float4 chunks (lane q of a group owns chunks
// q, q + LPP, ...), then TL single floats (lane q owns floats
// 4 LPP NCH + q TL + t).  The single floats let a row whose length is not a
// multiple of 4 LPP avoid a last chunk that would be mostly zero padding.
template <int NCH, int TL>
struct RowPart {
    float4 c[NCH];
    float t[TL > 0 ? TL : 1];
};

template <int LPP, int NCH, int TL>
__device__ inline void load_row(const float* row, int q, RowPart<NCH, TL>& x) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) x.c[c] = *reinterpret_cast<const float4*>(row + 4 * q + 4 * LPP * c);
    if constexpr (TL == 1) x.t[0] = row[4 * LPP * NCH + q];
    if constexpr (TL == 2) {
        const float2 v = *reinterpret_cast<const float2*>(row + 4 * LPP * NCH + 2 * q);
        x.t[0] = v.x;
        x.t[1] = v.y;
    }
}

template <int LPP, int NCH, int TL>
__device__ inline void store_row(float* row, int q, const RowPart<NCH, TL>& x) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) *reinterpret_cast<float4*>(row + 4 * q + 4 * LPP * c) = x.c[c];
    if constexpr (TL == 1) row[4 * LPP * NCH + q] = x.t[0];
    if constexpr (TL == 2) *reinterpret_cast<float2*>(row + 4 * LPP * NCH + 2 * q) = make_float2(x.t[0], x.t[1]);
}

// a.b summed over the group (two partial sums per lane for shorter chains:
// even chunks, then odd chunks and the single floats).
template <int LPP, int NCH, int TL>
__device__ inline float group_dot(const RowPart<NCH, TL>& a, const RowPart<NCH, TL>& b) {
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; c += 2) s0 = dot4(a.c[c], b.c[c], s0);
#pragma unroll
    for (int c = 1; c < NCH; c += 2) s1 = dot4(a.c[c], b.c[c], s1);
#pragma unroll
    for (int i = 0; i < TL; ++i) s1 = fmaf(a.t[i], b.t[i], s1);
    return group_sum<LPP>(s0 + s1);
}

// Rotate two rows in place by (s, tau): a' = a - s (b + tau a),
// b' = b + s (a - tau b).  Both temporaries are formed before either row is
// overwritten, so the update needs no register copies; s = tau = 0 leaves
// the rows bit-for-bit unchanged.
__device__ inline void rotate_values(float& a, float& b, float s, float h) {
    const float u = fmaf(h, a, b);
    const float v = fmaf(-h, b, a);
    a = fmaf(-s, u, a);
    b = fmaf(s, v, b);
}

template <int NCH, int TL>
__device__ inline void apply_rotation(RowPart<NCH, TL>& x, RowPart<NCH, TL>& y, float s, float h) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        float4 u, v;
        u.x = fmaf(h, x.c[c].x, y.c[c].x);
        u.y = fmaf(h, x.c[c].y, y.c[c].y);
        u.z = fmaf(h, x.c[c].z, y.c[c].z);
        u.w = fmaf(h, x.c[c].w, y.c[c].w);
        v.x = fmaf(-h, y.c[c].x, x.c[c].x);
        v.y = fmaf(-h, y.c[c].y, x.c[c].y);
        v.z = fmaf(-h, y.c[c].z, x.c[c].z);
        v.w = fmaf(-h, y.c[c].w, x.c[c].w);
        x.c[c].x = fmaf(-s, u.x, x.c[c].x);
        x.c[c].y = fmaf(-s, u.y, x.c[c].y);
        x.c[c].z = fmaf(-s, u.z, x.c[c].z);
        x.c[c].w = fmaf(-s, u.w, x.c[c].w);
        y.c[c].x = fmaf(s, v.x, y.c[c].x);
        y.c[c].y = fmaf(s, v.y, y.c[c].y);
        y.c[c].z = fmaf(s, v.z, y.c[c].z);
        y.c[c].w = fmaf(s, v.w, y.c[c].w);
    }
#pragma unroll
    for (int i = 0; i < TL; ++i) rotate_values(x.t[i], y.t[i], s, h);
}

// Rotate rows x, y (registers of the group) if they are not yet orthogonal
// to tolerance; updates their squared norms.  The decision is uniform over
// the group (all lanes hold identical sums).
template <int LPP, int NCH, int TL>
__device__ inline bool rotate_rows(RowPart<NCH, TL>& x, RowPart<NCH, TL>& y, float& nx, float& ny, float tol,
                                   float& sn, float& ta) {
    sn = ta = 0.f;
    const float ga = group_dot<LPP, NCH, TL>(x, y);
    if (!needs_rotation(ga, nx, ny, tol)) return false;
    float t;
    jacobi_rotation(nx, ny, ga, sn, ta, t);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const float4 a = x.c[c], b = y.c[c];
        x.c[c].x = fmaf(-sn, fmaf(ta, a.x, b.x), a.x);
        x.c[c].y = fmaf(-sn, fmaf(ta, a.y, b.y), a.y);
        x.c[c].z = fmaf(-sn, fmaf(ta, a.z, b.z), a.z);
        x.c[c].w = fmaf(-sn, fmaf(ta, a.w, b.w), a.w);
        y.c[c].x = fmaf(sn, fmaf(-ta, b.x, a.x), b.x);
        y.c[c].y = fmaf(sn, fmaf(-ta, b.y, a.y), b.y);
        y.c[c].z = fmaf(sn, fmaf(-ta, b.z, a.z), b.z);
        y.c[c].w = fmaf(sn, fmaf(-ta, b.w, a.w), b.w);
    }
#pragma unroll
    for (int i = 0; i < TL; ++i) rotate_values(x.t[i], y.t[i], sn, ta);
    // Tracked norms; clamped at 0 (cancellation can only make a small norm
    // inaccurate until the exact recomputation at the next sweep start).
    nx = fmaxf(fmaf(-t, ga, nx), 0.f);
    ny = fmaxf(fmaf(t, ga, ny), 0.f);
    return true;
}

// Two independent rotations (disjoint rows) computed side by side so that
// their dependency chains (dot, cross-lane sum, rotation parameters)
// overlap.  The skip test is uniform over the wavefront (no group of the
// wave rotates either pair); otherwise both updates run for every lane,
// with s = tau = 0 for a pair that is already orthogonal to tolerance,
// which leaves its rows and norms bit-for-bit unchanged.  Keeping the
// updates free of divergent branches lets the rows stay in their
// registers.
template <int LPP, int NCH, int TL>
__device__ inline void rotate_two(RowPart<NCH, TL>& x1, RowPart<NCH, TL>& y1, float& nx1, float& ny1, bool& f1,
                                  RowPart<NCH, TL>& x2, RowPart<NCH, TL>& y2, float& nx2, float& ny2, bool& f2,
                                  float tol, float& s1, float& h1, float& s2, float& h2) {
    s1 = h1 = s2 = h2 = 0.f;
    float p0 = 0.f, p1 = 0.f, q0 = 0.f, q1 = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; c += 2) {
        p0 = dot4(x1.c[c], y1.c[c], p0);
        q0 = dot4(x2.c[c], y2.c[c], q0);
    }
#pragma unroll
    for (int c = 1; c < NCH; c += 2) {
        p1 = dot4(x1.c[c], y1.c[c], p1);
        q1 = dot4(x2.c[c], y2.c[c], q1);
    }
#pragma unroll
    for (int i = 0; i < TL; ++i) {
        p1 = fmaf(x1.t[i], y1.t[i], p1);
        q1 = fmaf(x2.t[i], y2.t[i], q1);
    }
    const float g1 = group_sum<LPP>(p0 + p1);
    const float g2 = group_sum<LPP>(q0 + q1);
    f1 = needs_rotation(g1, nx1, ny1, tol);
    f2 = needs_rotation(g2, nx2, ny2, tol);
    if (!__any(f1 || f2)) return;
    // both tangents are computed (a = b = 1 stand in for a pair that stays,
    // whose own norms may both be 0) and the tangent of a pair that stays is
    // replaced by 0: s = tau = 0 and its norms keep their values
    float t1 = rotation_tangent(nx1, ny1, f1 ? g1 : 1.0f);
    float t2 = rotation_tangent(nx2, ny2, f2 ? g2 : 1.0f);
    t1 = f1 ? t1 : 0.f;
    t2 = f2 ? t2 : 0.f;
    rotation_sin_halftan(t1, s1, h1);
    rotation_sin_halftan(t2, s2, h2);
    apply_rotation<NCH, TL>(x1, y1, s1, h1);
    apply_rotation<NCH, TL>(x2, y2, s2, h2);
    nx1 = fmaxf(fmaf(-t1, g1, nx1), 0.f);
    ny1 = fmaxf(fmaf(t1, g1, ny1), 0.f);
    nx2 = fmaxf(fmaf(-t2, g2, nx2), 0.f);
    ny2 = fmaxf(fmaf(t2, g2, ny2), 0.f);
}

// Squared norms of rows 0..nrows-1 of B into s2 (LDS).
template <int LPP, int NCH, int TL>
__device__ void row_norms(const float* B, int nrows, int ld, float* s2) {
    const int tid = threadIdx.x;
    const int g = tid / LPP, q = tid % LPP;
    constexpr int G = NT / LPP;
    for (int j = g; j < nrows; j += G) {
        RowPart<NCH, TL> x;
        load_row<LPP, NCH, TL>(B + j * ld, q, x);
        const float v = group_dot<LPP, NCH, TL>(x, x);
        if (q == 0) s2[j] = v;
    }
    __syncthreads();
}

// Squared row norms during the sweeps: one LDS array for every variant.
__shared__ float tilt_jacobi_nrm[SVT_MAX_ROWS];

// Block pair k of round r of the circle ordering over Nb + 1 blocks (Nb
// odd): block Nb meets block r, and blocks r + k and r - k (mod Nb) meet.
struct CirclePairs {
    int r, Nb;
    __device__ inline void operator()(int k, int& I, int& J) const {
        if (k == 0) {
            I = Nb;
            J = r;
        } else {
            I = r + k;
            if (I >= Nb) I -= Nb;
            J = r - k;
            if (J < 0) J += Nb;
        }
    }
};

// One round of block pairs: every lane group takes pairs k = g, g + G, ...
// of the Pb pairs that `pairs` maps to block indices.  FIRST also rotates
// the pairs inside each block of two rows; it is a separate instance so the
// other rounds carry no conditional stage.
template <int BS, int LPP, int NCH, int TL, bool WARM, bool FIRST, class Pairs>
__device__ inline void jacobi_round_of(float* B, float* Rm, float* nrm, int ld, const Pairs& pairs, int Pb, int g,
                                       int q, float tol, int& any, long long& rots) {
    constexpr int G = NT / LPP;
    // WARM: the rotation rows of the block pair (same layout as the Jacobi
    // rows) stay in registers for the round and take the same rotations.
    constexpr int RN = WARM ? NCH : 1;
    constexpr int RT = WARM ? TL : 0;
    using Row = RowPart<NCH, TL>;
    using RRow = RowPart<RN, RT>;
    for (int k = g; k < Pb; k += G) {
        int I, J;
        pairs(k, I, J);
        float* pa = B + (BS * I) * ld;
        float* pb = B + (BS * J) * ld;
        if (BS == 1) {
            Row a1, b1;
            RRow ra, rb;
            load_row<LPP, NCH, TL>(pa, q, a1);
            load_row<LPP, NCH, TL>(pb, q, b1);
            float* qa = WARM ? Rm + I * ld : nullptr;
            float* qb = WARM ? Rm + J * ld : nullptr;
            if (WARM) {
                load_row<LPP, RN, RT>(qa, q, ra);
                load_row<LPP, RN, RT>(qb, q, rb);
            }
            float na1 = nrm[I], nb1 = nrm[J];
            float sr, hr;
            const bool f = rotate_rows<LPP, NCH, TL>(a1, b1, na1, nb1, tol, sr, hr);
            if (WARM && __any(f)) apply_rotation<RN, RT>(ra, rb, sr, hr);
            if (f) {
                any = 1;
                rots += 1;
                store_row<LPP, NCH, TL>(pa, q, a1);
                store_row<LPP, NCH, TL>(pb, q, b1);
                if (WARM) {
                    store_row<LPP, RN, RT>(qa, q, ra);
                    store_row<LPP, RN, RT>(qb, q, rb);
                }
                if (q == 0) {
                    nrm[I] = na1;
                    nrm[J] = nb1;
                }
            }
        } else {
            Row a1, a2, b1, b2;
            RRow ra1, ra2, rb1, rb2;
            load_row<LPP, NCH, TL>(pa, q, a1);
            load_row<LPP, NCH, TL>(pa + ld, q, a2);
            load_row<LPP, NCH, TL>(pb, q, b1);
            load_row<LPP, NCH, TL>(pb + ld, q, b2);
            float* qa = WARM ? Rm + (BS * I) * ld : nullptr;
            float* qb = WARM ? Rm + (BS * J) * ld : nullptr;
            if (WARM) {
                load_row<LPP, RN, RT>(qa, q, ra1);
                load_row<LPP, RN, RT>(qa + ld, q, ra2);
                load_row<LPP, RN, RT>(qb, q, rb1);
                load_row<LPP, RN, RT>(qb + ld, q, rb2);
            }
            float na1 = nrm[2 * I], na2 = nrm[2 * I + 1], nb1 = nrm[2 * J], nb2 = nrm[2 * J + 1];
            bool d0 = false, d1 = false, d2 = false, d3 = false, f, h;
            float s1, h1, s2, h2;
            if (FIRST) {
                rotate_two<LPP, NCH, TL>(a1, a2, na1, na2, f, b1, b2, nb1, nb2, h, tol, s1, h1, s2, h2);
                if (WARM && __any(f || h)) {
                    apply_rotation<RN, RT>(ra1, ra2, s1, h1);
                    apply_rotation<RN, RT>(rb1, rb2, s2, h2);
                }
                d0 |= f; d1 |= f; d2 |= h; d3 |= h; rots += f; rots += h;
            }
            rotate_two<LPP, NCH, TL>(a1, b1, na1, nb1, f, a2, b2, na2, nb2, h, tol, s1, h1, s2, h2);
            if (WARM && __any(f || h)) {
                apply_rotation<RN, RT>(ra1, rb1, s1, h1);
                apply_rotation<RN, RT>(ra2, rb2, s2, h2);
            }
            d0 |= f; d2 |= f; d1 |= h; d3 |= h; rots += f; rots += h;
            rotate_two<LPP, NCH, TL>(a1, b2, na1, nb2, f, a2, b1, na2, nb1, h, tol, s1, h1, s2, h2);
            if (WARM && __any(f || h)) {
                apply_rotation<RN, RT>(ra1, rb2, s1, h1);
                apply_rotation<RN, RT>(ra2, rb1, s2, h2);
            }
            d0 |= f; d3 |= f; d1 |= h; d2 |= h; rots += f; rots += h;
            if (d0 | d1 | d2 | d3) any = 1;
            if (d0) store_row<LPP, NCH, TL>(pa, q, a1);
            if (d1) store_row<LPP, NCH, TL>(pa + ld, q, a2);
            if (d2) store_row<LPP, NCH, TL>(pb, q, b1);
            if (d3) store_row<LPP, NCH, TL>(pb + ld, q, b2);
            if (WARM) {
                if (d0) store_row<LPP, RN, RT>(qa, q, ra1);
                if (d1) store_row<LPP, RN, RT>(qa + ld, q, ra2);
                if (d2) store_row<LPP, RN, RT>(qb, q, rb1);
                if (d3) store_row<LPP, RN, RT>(qb + ld, q, rb2);
            }
            if (q == 0) {
                nrm[2 * I] = na1;
                nrm[2 * I + 1] = na2;
                nrm[2 * J] = nb1;
                nrm[2 * J + 1] = nb2;
            }
        }
    }
}

// Round r of the circle ordering over the Nb + 1 blocks of B; FIRST in
// round 0 of a sweep.
template <int BS, int LPP, int NCH, int TL, bool WARM, bool FIRST>
__device__ inline void jacobi_round(float* B, float* Rm, float* nrm, int ld, int r, int Nb, int Pb, int g, int q,
                                    float tol, int& any, long long& rots) {
    jacobi_round_of<BS, LPP, NCH, TL, WARM, FIRST>(B, Rm, nrm, ld, CirclePairs{r, Nb}, Pb, g, q, tol, any, rots);
}

// Returns 1 (uniform over the workgroup) if any pair was rotated.  WARM:
// every rotation is also applied to the rows of Rm (same layout), which
// accumulates the product of the rotations.
template <int BS, int LPP, int NCH, int TL, bool WARM>
__device__ int jacobi_rows(float* B, float* Rm, int nc, int ld, float tol, int max_sweeps, JacobiStats& js) {
    float* nrm = tilt_jacobi_nrm;
    const int tid = threadIdx.x;
    const int g = tid / LPP, q = tid % LPP;
    const int nc4 = (nc + 3) & ~3;
    const int nb = nc4 / BS;          // blocks (even)
    const int Pb = nb >> 1, Nb = nb - 1;
    long long rots = 0;
    int sweeps = 0, rotated = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        row_norms<LPP, NCH, TL>(B, nc4, ld, nrm);
        int any = 0;
        jacobi_round<BS, LPP, NCH, TL, WARM, true>(B, Rm, nrm, ld, 0, Nb, Pb, g, q, tol, any, rots);
        __syncthreads();
        for (int r = 1; r < Nb; ++r) {
            jacobi_round<BS, LPP, NCH, TL, WARM, false>(B, Rm, nrm, ld, r, Nb, Pb, g, q, tol, any, rots);
            __syncthreads();
        }
        ++sweeps;
        const int a = __syncthreads_or(any);
        rotated |= a;
        if (!a) break;
    }
    // every pair of the nc4 rows is examined once per sweep
    js.sweeps += sweeps;
    js.pairs += (long long)sweeps * ((long long)nc4 * (nc4 - 1) / 2);
    js.rotations += block_sum_ll(q == 0 ? rots : 0);
    return rotated;
}

template <int BS, int LPP, int NCH, int TL, bool WARM>
__device__ void jacobi_svd_rows(float* B, float* Rm, int nc, int ld, float tol, int max_sweeps, JacobiStats& js,
                                float* s2) {
    jacobi_rows<BS, LPP, NCH, TL, WARM>(B, Rm, nc, ld, tol, max_sweeps, js);
    row_norms<LPP, NCH, TL>(B, nc, ld, s2);
}

// Staged super-block pair of the tiled Jacobi: rows 0..sb-1 of B are
// super-block I, rows sb..2sb-1 super-block J, h = sb / BS blocks each (h
// even).  The pairs inside the two super-blocks (when `inner`: the circle
// ordering run in both at once, h - 1 rounds of h block pairs) and then
// every cross pair (h rounds; round s joins block a of I with block
// (a + s) mod h of J).
struct InnerPairs {
    int r, Nb, Pb, h;  // circle round r over the h = Nb + 1 blocks of each super-block, Pb = h / 2
    __device__ inline void operator()(int k, int& I, int& J) const {
        const int half = k >= Pb ? 1 : 0;
        CirclePairs{r, Nb}(k - half * Pb, I, J);
        I += half * h;
        J += half * h;
    }
};

struct CrossPairs {
    int s, h;
    __device__ inline void operator()(int k, int& I, int& J) const {
        I = k;
        J = k + s;
        if (J >= h) J -= h;
        J += h;
    }
};

template <int BS, int LPP, int NCH, int TL, bool WARM>
__device__ int jacobi_pair_rows(float* B, float* Rm, int sb, int ld, float tol, bool inner, JacobiStats& js) {
    float* nrm = tilt_jacobi_nrm;
    const int tid = threadIdx.x;
    const int g = tid / LPP, q = tid % LPP;
    const int h = sb / BS;
    long long rots = 0;
    int any = 0;
    row_norms<LPP, NCH, TL>(B, 2 * sb, ld, nrm);
    if (inner) {
        const int Nb = h - 1, Pb = h >> 1;
        jacobi_round_of<BS, LPP, NCH, TL, WARM, true>(B, Rm, nrm, ld, InnerPairs{0, Nb, Pb, h}, h, g, q, tol, any,
                                                      rots);
        __syncthreads();
        for (int r = 1; r < Nb; ++r) {
            jacobi_round_of<BS, LPP, NCH, TL, WARM, false>(B, Rm, nrm, ld, InnerPairs{r, Nb, Pb, h}, h, g, q, tol,
                                                           any, rots);
            __syncthreads();
        }
    }
    for (int s = 0; s < h; ++s) {
        jacobi_round_of<BS, LPP, NCH, TL, WARM, false>(B, Rm, nrm, ld, CrossPairs{s, h}, h, g, q, tol, any, rots);
        __syncthreads();
    }
    const int a = __syncthreads_or(any);
    js.pairs += (long long)sb * sb + (inner ? (long long)sb * (sb - 1) : 0);
    js.rotations += block_sum_ll(q == 0 ? rots : 0);
    return a;
}

// Layout codes from svt_make_cfg(BS, LPP, NCH, TL).
#define TILT_SVT_CASE_T(S, L, C, T)                                                       \
    case svt_make_cfg(S, L, C, T):                                                        \
        jacobi_svd_rows<S, L, C, T, false>(B, nullptr, nc, ld, tol, max_sweeps, js, s2);  \
        break;
#define TILT_SVT_CASE(S, L, C) TILT_SVT_CASE_T(S, L, C, 0)
#define TILT_SVT_CASES8(S, L)                                                              \
    TILT_SVT_CASE(S, L, 1) TILT_SVT_CASE(S, L, 2) TILT_SVT_CASE(S, L, 3) TILT_SVT_CASE(S, L, 4) \
    TILT_SVT_CASE(S, L, 5) TILT_SVT_CASE(S, L, 6) TILT_SVT_CASE(S, L, 7) TILT_SVT_CASE(S, L, 8)
#define TILT_SVT_CASES4(S, L) \
    TILT_SVT_CASE(S, L, 1) TILT_SVT_CASE(S, L, 2) TILT_SVT_CASE(S, L, 3) TILT_SVT_CASE(S, L, 4)
// Two-row blocks of 8 or 16 lanes with 1-3 chunks and 1 or 2 single floats
// per lane (the layouts the host offers for the one-workgroup SVT).
#define TILT_SVT_TAILS(S, L)                                                                      \
    TILT_SVT_CASE_T(S, L, 1, 1) TILT_SVT_CASE_T(S, L, 2, 1) TILT_SVT_CASE_T(S, L, 3, 1)           \
    TILT_SVT_CASE_T(S, L, 1, 2) TILT_SVT_CASE_T(S, L, 2, 2) TILT_SVT_CASE_T(S, L, 3, 2)

// Kept out of line (as is the warm variant): inlined into dev_svt, its
// switch made the 256 x 100x100 batch 30 % slower, with the same code for
// the Jacobi itself.
__device__ void jacobi_dispatch(int cfg, float* B, int nc, int ld, float tol, int max_sweeps, JacobiStats& js,
                                float* s2) {
    switch (cfg) {
        TILT_SVT_CASES8(1, 4) TILT_SVT_CASES8(1, 8) TILT_SVT_CASES8(1, 16)
        TILT_SVT_CASES4(2, 4) TILT_SVT_CASES4(2, 8) TILT_SVT_CASES4(2, 16)
        TILT_SVT_TAILS(2, 8) TILT_SVT_TAILS(2, 16)
        // rows longer than 512: the layouts the cost model may choose there
        TILT_SVT_CASE(1, 32, 5) TILT_SVT_CASE(1, 32, 6) TILT_SVT_CASE(1, 32, 7) TILT_SVT_CASE(1, 32, 8)
        TILT_SVT_CASE(1, 64, 3) TILT_SVT_CASE(1, 64, 4) TILT_SVT_CASE(1, 64, 5) TILT_SVT_CASE(1, 64, 6)
        TILT_SVT_CASE(1, 64, 7) TILT_SVT_CASE(1, 64, 8) TILT_SVT_CASE(2, 64, 3) TILT_SVT_CASE(2, 64, 4)
        default:
            break;
    }
}

// Warm variants (rotation rows Rm in LDS, same layout as B): chunks per
// lane up to 4.
#define TILT_WARM_CASE_T(S, L, C, T)                                                      \
    case svt_make_cfg(S, L, C, T):                                                        \
        jacobi_svd_rows<S, L, C, T, true>(B, Rm, nc, ld, tol, max_sweeps, js, s2);        \
        break;
#define TILT_WARM_CASE(S, L, C) TILT_WARM_CASE_T(S, L, C, 0)
#define TILT_WARM_CASES4(S, L) \
    TILT_WARM_CASE(S, L, 1) TILT_WARM_CASE(S, L, 2) TILT_WARM_CASE(S, L, 3) TILT_WARM_CASE(S, L, 4)
#define TILT_WARM_TAILS(S, L)                                                                       \
    TILT_WARM_CASE_T(S, L, 1, 1) TILT_WARM_CASE_T(S, L, 2, 1) TILT_WARM_CASE_T(S, L, 3, 1)          \
    TILT_WARM_CASE_T(S, L, 1, 2) TILT_WARM_CASE_T(S, L, 2, 2) TILT_WARM_CASE_T(S, L, 3, 2)

__device__ void jacobi_dispatch_warm(int cfg, float* B, float* Rm, int nc, int ld, float tol, int max_sweeps,
                                     JacobiStats& js, float* s2) {
    switch (cfg) {
        TILT_WARM_CASES4(1, 4) TILT_WARM_CASES4(1, 8) TILT_WARM_CASES4(1, 16)
        TILT_WARM_CASES4(2, 4) TILT_WARM_CASES4(2, 8) TILT_WARM_CASES4(2, 16)
        TILT_WARM_TAILS(2, 8) TILT_WARM_TAILS(2, 16)
        default:
            break;
    }
}
#undef TILT_WARM_TAILS
#undef TILT_WARM_CASES4
#undef TILT_WARM_CASE
#undef TILT_WARM_CASE_T
#undef TILT_SVT_TAILS
#undef TILT_SVT_CASES4
#undef TILT_SVT_CASES8
#undef TILT_SVT_CASE
#undef TILT_SVT_CASE_T

// The rounds of one staged super-block pair (jacobi_pair_rows) for the
// layout code cfg, with the rotation rows Rm (same layout as B; chunks per
// lane up to 4) in the _warm variant; 1 if any pair rotated.  The tiled
// paths use layouts without single floats.
#define TILT_PAIR_CASE(S, L, C) \
    case svt_make_cfg(S, L, C): \
        return jacobi_pair_rows<S, L, C, 0, false>(B, nullptr, sb, ld, tol, inner, js);
#define TILT_PAIR_CASES8(S, L)                                                                  \
    TILT_PAIR_CASE(S, L, 1) TILT_PAIR_CASE(S, L, 2) TILT_PAIR_CASE(S, L, 3) TILT_PAIR_CASE(S, L, 4) \
    TILT_PAIR_CASE(S, L, 5) TILT_PAIR_CASE(S, L, 6) TILT_PAIR_CASE(S, L, 7) TILT_PAIR_CASE(S, L, 8)
#define TILT_PAIR_CASES4(S, L) \
    TILT_PAIR_CASE(S, L, 1) TILT_PAIR_CASE(S, L, 2) TILT_PAIR_CASE(S, L, 3) TILT_PAIR_CASE(S, L, 4)
#define TILT_WPAIR_CASE(S, L, C) \
    case svt_make_cfg(S, L, C):  \
        return jacobi_pair_rows<S, L, C, 0, true>(B, Rm, sb, ld, tol, inner, js);
#define TILT_WPAIR_CASES4(S, L) \
    TILT_WPAIR_CASE(S, L, 1) TILT_WPAIR_CASE(S, L, 2) TILT_WPAIR_CASE(S, L, 3) TILT_WPAIR_CASE(S, L, 4)

__device__ int jacobi_pair_dispatch(int cfg, float* B, int sb, int ld, float tol, bool inner, JacobiStats& js) {
    switch (cfg) {
        TILT_PAIR_CASES8(1, 4) TILT_PAIR_CASES8(1, 8) TILT_PAIR_CASES8(1, 16)
        TILT_PAIR_CASES4(2, 4) TILT_PAIR_CASES4(2, 8) TILT_PAIR_CASES4(2, 16)
        TILT_PAIR_CASE(1, 32, 5) TILT_PAIR_CASE(1, 32, 6) TILT_PAIR_CASE(1, 32, 7) TILT_PAIR_CASE(1, 32, 8)
        TILT_PAIR_CASE(1, 64, 3) TILT_PAIR_CASE(1, 64, 4) TILT_PAIR_CASE(1, 64, 5) TILT_PAIR_CASE(1, 64, 6)
        TILT_PAIR_CASE(1, 64, 7) TILT_PAIR_CASE(1, 64, 8) TILT_PAIR_CASE(2, 64, 3) TILT_PAIR_CASE(2, 64, 4)
        default:
            break;
    }
    return 0;
}

__device__ int jacobi_pair_dispatch_warm(int cfg, float* B, float* Rm, int sb, int ld, float tol, bool inner,
                                         JacobiStats& js) {
    switch (cfg) {
        TILT_WPAIR_CASES4(1, 4) TILT_WPAIR_CASES4(1, 8) TILT_WPAIR_CASES4(1, 16)
        TILT_WPAIR_CASES4(2, 4) TILT_WPAIR_CASES4(2, 8) TILT_WPAIR_CASES4(2, 16)
        default:
            break;
    }
    return 0;
}
#undef TILT_WPAIR_CASES4
#undef TILT_WPAIR_CASE
#undef TILT_PAIR_CASES4
#undef TILT_PAIR_CASES8
#undef TILT_PAIR_CASE

// ---------------------------------------------------------------------------
// Tiled one-sided Jacobi for matrices that do not fit in LDS.
//
// The ncp rows (nc real rows, then zero rows) live in a device plane with
// stride ldg and are split into nsb super-blocks of sb rows.  A sweep runs
// the circle method over super-blocks; for each super-block pair both
// blocks are staged into LDS as one 2 sb-row matrix, every cross pair (one
// row from each block) is examined, and the blocks are written back if
// anything rotated.  In the first round of a sweep, where every super-block
// takes part once, the pairs inside both blocks are examined first.  So
// every pair of rows is examined exactly once per sweep; a sweep in which
// no pair rotates leaves every row unchanged, so all pairs were tested
// against the final rows, and the iteration stops.  Zero rows are never
// rotated (a.b = 0).
// ---------------------------------------------------------------------------

__device__ void clear_lds_padding(float* B, int nc, int ldg, int ld);

__device__ void load_block(const float* Bg, int r0, int cnt, int ldg, float* mini, int dst, int ld) {
    const int nr4 = ldg >> 2;
    for (int idx = threadIdx.x; idx < cnt * nr4; idx += NT) {
        const int row = idx / nr4, c = idx - row * nr4;
        *reinterpret_cast<float4*>(mini + (dst + row) * ld + 4 * c) =
            reinterpret_cast<const float4*>(Bg + (size_t)(r0 + row) * ldg)[c];
    }
}

__device__ void store_block(float* Bg, int r0, int cnt, int ldg, const float* mini, int src, int ld) {
    const int nr4 = ldg >> 2;
    for (int idx = threadIdx.x; idx < cnt * nr4; idx += NT) {
        const int row = idx / nr4, c = idx - row * nr4;
        reinterpret_cast<float4*>(Bg + (size_t)(r0 + row) * ldg)[c] =
            *reinterpret_cast<const float4*>(mini + (src + row) * ld + 4 * c);
    }
}

// Pair k of round r of the circle ordering over nsb super-blocks: the
// super-blocks I and J it joins.
__device__ inline void superblock_pair(int nsb, int r, int k, int& I, int& J) { CirclePairs{r, nsb - 1}(k, I, J); }

// One super-block pair: stage both blocks into LDS, examine their pairs
// (the cross pairs, and in round 0 the pairs inside each block first),
// write them back if anything rotated.  With Rg (the warm start) the
// matching rows of the rotation are staged after them and take the same
// rotations.  Returns 1 if a pair rotated (uniform over the workgroup).
__device__ int superblock_task(int cfg, float* Bg, float* Rg, int sb, int nsb, int ldg, int ld, float* mini,
                               float tol, int r, int k, JacobiStats& js) {
    int I, J;
    superblock_pair(nsb, r, k, I, J);
    float* rmini = mini + 2 * sb * ld;
    load_block(Bg, I * sb, sb, ldg, mini, 0, ld);
    load_block(Bg, J * sb, sb, ldg, mini, sb, ld);
    clear_lds_padding(mini, 2 * sb, ldg, ld);
    if (Rg) {
        load_block(Rg, I * sb, sb, ldg, rmini, 0, ld);
        load_block(Rg, J * sb, sb, ldg, rmini, sb, ld);
        clear_lds_padding(rmini, 2 * sb, ldg, ld);
    }
    __syncthreads();
    const int rot = Rg ? jacobi_pair_dispatch_warm(cfg, mini, rmini, sb, ld, tol, r == 0, js)
                       : jacobi_pair_dispatch(cfg, mini, sb, ld, tol, r == 0, js);
    if (rot) {
        store_block(Bg, I * sb, sb, ldg, mini, 0, ld);
        store_block(Bg, J * sb, sb, ldg, mini, sb, ld);
        if (Rg) {
            store_block(Rg, I * sb, sb, ldg, rmini, 0, ld);
            store_block(Rg, J * sb, sb, ldg, rmini, sb, ld);
        }
    }
    __syncthreads();
    return rot;
}

// ---------------------------------------------------------------------------
// Help for windows beyond LDS inside the fused kernel.
//
// A window whose SVT is tiled is solved by one workgroup, its leader, like
// every other window.  Once the work queue is empty, workgroups with nothing
// left to solve become helpers.  While helpers are idle, a leader publishes
// each round of its tiled Jacobi in its control block: the round's
// parameters, then one 64-bit word (round id, pairs, pairs claimed).  Any
// helper, and the leader itself, claims a pair by a compare-and-swap on the
// word and runs it; the leader then waits only for the pairs helpers have
// claimed.  A round never waits for a helper to arrive, nobody waits on a
// workgroup that has not claimed work, and the pairs of a round touch
// disjoint rows, so the result is the same whoever takes which pair.
// Members may sit on different XCDs (each with its own L2): data goes out
// with an agent-scope release before a round is published or a finished
// pair is counted, and comes in with an agent-scope acquire after a claim
// or the leader's wait.
// ---------------------------------------------------------------------------

__device__ inline int gang_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Polling loads are relaxed: an agent-scope acquire invalidates the
// non-coherent lines of the XCD's L2 (and its dirty lines go back to
// memory), which, repeated by every spinning workgroup, would evict the
// working sets of the workgroups still solving.  Data is acquired once,
// after the awaited value has been seen.
__device__ inline int poll_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void release_all_waves() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
}

__device__ inline void acquire_all_waves() {
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

constexpr unsigned long long kRoundIdShift = 32;

// Claim the next pair of the published round `w` of c (thread 0 only).
// Returns the pair index, or -1 if the round is fully claimed or moved on.
__device__ int gang_try_claim(GangCtl* c, unsigned long long w) {
    const int pairs = (int)((w >> 16) & 0xffffu), claimed = (int)(w & 0xffffu);
    if (claimed >= pairs) return -1;
    unsigned long long expect = w;
    if (__hip_atomic_compare_exchange_strong(&c->word, &expect, w + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
        return claimed;
    return -1;
}

// Leader: the tiled Jacobi of the ncp rows of Bg (with the rotation rows Rg
// when warm-started), publishing rounds while helpers are idle.  The
// helpers' pair counts are added to js at the end.
__device__ void jacobi_tiled_shared(GangCtl* c, int cfg, float* Bg, float* Rg, int sb, int nsb, int ldg, int ld,
                                    float* mini, float tol, int max_sweeps, JacobiStats& js) {
    __shared__ int sh_v;
    const int tid = threadIdx.x;
    const int Nb = nsb - 1, Pb = nsb >> 1;
    FusedCtl* fc = c->fc;
    const long long sweeps0 = js.sweeps;  // the staged sweeps of single pairs are not sweeps of the matrix
    int sweeps = 0;
    int helped = 0;  // pairs run by helpers so far in this decomposition
    int base_done = 0;
    if (tid == 0) sh_v = poll_load(&c->done);
    __syncthreads();
    base_done = sh_v;
    __syncthreads();
    for (int sw = 0; sw < max_sweeps; ++sw) {
        int any = 0;
        int first_id = 0;  // id of this sweep's first published round (0: none)
        for (int r = 0; r < Nb; ++r) {
            if (tid == 0) sh_v = (Pb > 1 && poll_load(&fc->idle) > 0) ? 1 : 0;
            __syncthreads();
            const int publish = sh_v;
            __syncthreads();
            if (!publish) {
                for (int k = 0; k < Pb; ++k) any |= superblock_task(cfg, Bg, Rg, sb, nsb, ldg, ld, mini, tol, r, k, js);
                continue;
            }
            release_all_waves();
            if (tid == 0) {
                if (c->slot < 0) {
                    // register where helpers look (once per request)
                    const int idx = (int)(c - fc->gangs);
                    for (int i = 0; i < HELP_SLOTS; ++i) {
                        const int sl = (idx + i) & (HELP_SLOTS - 1);
                        int zero = 0;
                        if (__hip_atomic_compare_exchange_strong(&fc->slots[sl], &zero, idx + 1, __ATOMIC_RELAXED,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            c->slot = sl;
                            break;
                        }
                    }
                }
                c->Bg = Bg;
                c->Rg = Rg;
                c->sb = sb;
                c->nsb = nsb;
                c->ldg = ldg;
                c->ld = ld;
                c->cfg = cfg;
                c->r = r;
                c->tol = tol;
                const unsigned id = (unsigned)(++c->rid);
                __hip_atomic_store(&c->word, ((unsigned long long)id << kRoundIdShift) | ((unsigned long long)Pb << 16),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                sh_v = (int)id;
            }
            __syncthreads();
            const int id = sh_v;
            if (!first_id) first_id = id;
            __syncthreads();
            int mine = 0;
            for (;;) {
                if (tid == 0) {
                    int k = -1;
                    for (;;) {
                        const unsigned long long w =
                            __hip_atomic_load(&c->word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if ((w & 0xffffu) >= ((w >> 16) & 0xffffu)) break;
                        k = gang_try_claim(c, w);
                        if (k >= 0) break;
                    }
                    sh_v = k;
                }
                __syncthreads();
                const int k = sh_v;
                __syncthreads();
                if (k < 0) break;
                any |= superblock_task(cfg, Bg, Rg, sb, nsb, ldg, ld, mini, tol, r, k, js);
                ++mine;
            }
            helped += Pb - mine;
            if (tid == 0)
                while (poll_load(&c->done) < base_done + helped) __builtin_amdgcn_s_sleep(1);
            acquire_all_waves();
        }
        ++sweeps;
        // a helper's pair that rotated raised `rot` to its round's id
        if (tid == 0) sh_v = any || (first_id > 0 && gang_load(&c->rot) >= first_id);
        __syncthreads();
        const int rotated = sh_v;
        __syncthreads();
        if (!rotated) break;
    }
    js.sweeps = sweeps0 + sweeps;
    if (tid == 0 && helped > 0) {
        // every helper added its counts before counting its pair done
        js.pairs += (long long)__hip_atomic_exchange(&c->pairs, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        js.rotations += (long long)__hip_atomic_exchange(&c->rotations, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Helper, first half (inlined into the kernel's idle loop, no call): wave
// 0 looks for a published round with an unclaimed pair among the
// registered leaders and thread 0 tries to claim it.  On success the
// round's parameters, id and pair are left in *job, *id and the return
// value is the leader's index; else -1.
__device__ __forceinline__ int help_find(FusedCtl* fc, GangCtl* job, unsigned* id, int* pair) {
    __shared__ int sh_g;
    const int tid = threadIdx.x;
    if (tid < 64) {
        // 64 slots at a time, from a start that differs between workgroups
        const int start = (int)((blockIdx.x * 97u) & (HELP_SLOTS - 1));
        int found = -1;
        for (int base = 0; base < HELP_SLOTS && found < 0; base += 64) {
            const int sl = (start + base + tid) & (HELP_SLOTS - 1);
            const int v = __hip_atomic_load(&fc->slots[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool open = false;
            if (v > 0) {
                const unsigned long long w =
                    __hip_atomic_load(&fc->gangs[v - 1].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                open = (w & 0xffffu) < ((w >> 16) & 0xffffu);
            }
            const unsigned long long bal = __ballot(open);
            if (bal) {
                const int lane = __ffsll((long long)bal) - 1;
                found = __shfl(v, lane) - 1;
            }
        }
        if (tid == 0) {
            sh_g = -1;
            if (found >= 0) {
                GangCtl* c = fc->gangs + found;
                const unsigned long long w = __hip_atomic_load(&c->word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // parameters of the round named by w: valid if the claim below
                // succeeds (a newer round is published only after every pair
                // of this one was claimed and finished; the claim acquires)
                job->Bg = c->Bg;
                job->Rg = c->Rg;
                job->sb = c->sb;
                job->nsb = c->nsb;
                job->ldg = c->ldg;
                job->ld = c->ld;
                job->cfg = c->cfg;
                job->r = c->r;
                job->tol = c->tol;
                *id = (unsigned)(w >> kRoundIdShift);
                *pair = gang_try_claim(c, w);
                if (*pair >= 0) sh_g = found;
            }
        }
    }
    __syncthreads();
    const int g = sh_g;
    __syncthreads();
    return g;
}

// Helper, second half (out of line; called only with a claimed pair): run
// pair k of the round described by *job of leader g and report it done.
__device__ __noinline__ void help_run(FusedCtl* fc, int g, const GangCtl* job, unsigned id, int k, float* mini) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    GangCtl* c = fc->gangs + g;
    JacobiStats jr{0, 0, 0};
    const int rot =
        superblock_task(job->cfg, job->Bg, job->Rg, job->sb, job->nsb, job->ldg, job->ld, mini, job->tol, job->r, k, jr);
    release_all_waves();
    if (threadIdx.x == 0) {
        if (rot) atomicMax(&c->rot, (int)id);
        if (jr.pairs) atomicAdd(&c->pairs, (unsigned long long)jr.pairs);
        if (jr.rotations) atomicAdd(&c->rotations, (unsigned long long)jr.rotations);
        __hip_atomic_fetch_add(&c->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// The tiled Jacobi of the ncp rows of Bg (with the rotation rows Rg when
// warm-started) on this workgroup, with helpers when `gang` is given.
__device__ void jacobi_tiled(int cfg, float* Bg, float* Rg, int sb, int nsb, int ldg, int ld, float* mini, float tol,
                             int max_sweeps, JacobiStats& js, GangCtl* gang = nullptr) {
    if (gang) {
        jacobi_tiled_shared(gang, cfg, Bg, Rg, sb, nsb, ldg, ld, mini, tol, max_sweeps, js);
        return;
    }
    const int Nb = nsb - 1, Pb = nsb >> 1;
    const long long sweeps0 = js.sweeps;
    int sweeps = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        int any = 0;
        for (int r = 0; r < Nb; ++r)
            for (int k = 0; k < Pb; ++k) any |= superblock_task(cfg, Bg, Rg, sb, nsb, ldg, ld, mini, tol, r, k, js);
        ++sweeps;
        if (!any) break;
    }
    js.sweeps = sweeps0 + sweeps;
}

// Squared norms of rows 0..nrows-1 of a device plane (stride ldg) into s2.
__device__ void row_norms_global(const float* X, int nrows, int ldg, float* s2) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nr4 = ldg >> 2;
    for (int j = wv; j < nrows; j += NWAVE) {
        const float4* pr = reinterpret_cast<const float4*>(X + (size_t)j * ldg);
        float acc = 0.f;
        for (int c = lane; c < nr4; c += 64) {
            const float4 v = pr[c];
            acc = dot4(v, v, acc);
        }
        acc = wave_sum_f(acc);
        if (lane == 0) s2[j] = acc;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Singular value shrinkage from the orthogonalised rows.
//
// With B = V^T X (rows b_j orthogonal, s_j = ||b_j||) the SVD of X is
// V diag(s) (B/s)^T rows, so S_eps(X) = sum_{s_j > eps} (1 - eps/s_j)/s_j^2
// (X b_j^T) b_j.  Computed in blocks of TB rows of X:
//   C = Xblk B_act^T,  Cw = C diag(w),  A_blk = Cw B_act.
// ---------------------------------------------------------------------------

__device__ void shrink_weights(const float* s2, int nc, float eps, float* w, int* act, int* k_out,
                               double* nuc_out) {
    // w_j = (1 - eps/s_j)/s_j^2 for s_j > eps (else 0); act lists the kept
    // rows in ascending order (ballot + prefix count per wavefront).
    __shared__ int wave_cnt[NWAVE];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double nuc[1] = {0.0};
    int base = 0;
    for (int j0 = 0; j0 < nc; j0 += NT) {
        const int j = j0 + tid;
        bool on = false;
        if (j < nc) {
            const float sg = sqrtf(s2[j]);
            on = sg > eps;
            w[j] = on ? (1.0f - eps / sg) / s2[j] : 0.f;
            if (on) nuc[0] += (double)sg - (double)eps;
        }
        const unsigned long long bal = __ballot(on);
        if (lane == 0) wave_cnt[wv] = __popcll(bal);
        __syncthreads();
        int off = base, tot = base;
        for (int u = 0; u < NWAVE; ++u) {
            if (u < wv) off += wave_cnt[u];
            tot += wave_cnt[u];
        }
        if (on) act[off + __popcll(bal & ((1ull << lane) - 1ull))] = j;
        __syncthreads();
        base = tot;
    }
    block_sum_d<1>(nuc);
    *k_out = base;
    *nuc_out = nuc[0];
}

// Returns this thread's partial sum of (A_new - A_old)^2 when track_diff.
__device__ float reconstruct(const float* B, int ld, const float* Xg, float* Ag, int nc, int nr4, int ldg,
                             const float* w, const int* act, int k, int TB, float* xblk, float* cwt,
                             bool track_diff) {
    const int tid = threadIdx.x;
    const int tb4 = TB >> 2;
    const int k4 = (k + 3) >> 2;
    float dsum = 0.f;
    for (int i0 = 0; i0 < nc; i0 += TB) {
        for (int idx = tid; idx < TB * nr4; idx += NT) {
            const int ii = idx / nr4, c = idx - ii * nr4;
            float4 v = f4(0.f);
            if (i0 + ii < nc) v = reinterpret_cast<const float4*>(Xg + (size_t)(i0 + ii) * ldg)[c];
            *reinterpret_cast<float4*>(xblk + ii * ld + 4 * c) = v;
        }
        __syncthreads();
        for (int tile = tid; tile < tb4 * k4; tile += NT) {
            const int ii4 = tile % tb4, jj4 = tile / tb4;
            int jr[4];
            float wj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jj = 4 * jj4 + u;
                if (jj < k) {
                    jr[u] = act[jj];
                    wj[u] = w[jr[u]];
                } else {
                    jr[u] = act[0];
                    wj[u] = 0.f;
                }
            }
            float acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[a][u] = 0.f;
            for (int c = 0; c < nr4; ++c) {
                float4 x[4], b[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) x[a] = *reinterpret_cast<const float4*>(xblk + (4 * ii4 + a) * ld + 4 * c);
#pragma unroll
                for (int u = 0; u < 4; ++u) b[u] = *reinterpret_cast<const float4*>(B + jr[u] * ld + 4 * c);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        float s = acc[a][u];
                        s = fmaf(x[a].x, b[u].x, s);
                        s = fmaf(x[a].y, b[u].y, s);
                        s = fmaf(x[a].z, b[u].z, s);
                        s = fmaf(x[a].w, b[u].w, s);
                        acc[a][u] = s;
                    }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int a = 0; a < 4; ++a) cwt[(4 * jj4 + u) * TB + 4 * ii4 + a] = acc[a][u] * wj[u];
        }
        __syncthreads();
        for (int tile = tid; tile < tb4 * nr4; tile += NT) {
            const int r4 = tile % nr4, ii4 = tile / nr4;
            float4 acc[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] = f4(0.f);
            for (int jj = 0; jj < k; ++jj) {
                const float4 cw = *reinterpret_cast<const float4*>(cwt + jj * TB + 4 * ii4);
                const float4 b = *reinterpret_cast<const float4*>(B + act[jj] * ld + 4 * r4);
                acc[0].x = fmaf(cw.x, b.x, acc[0].x); acc[0].y = fmaf(cw.x, b.y, acc[0].y);
                acc[0].z = fmaf(cw.x, b.z, acc[0].z); acc[0].w = fmaf(cw.x, b.w, acc[0].w);
                acc[1].x = fmaf(cw.y, b.x, acc[1].x); acc[1].y = fmaf(cw.y, b.y, acc[1].y);
                acc[1].z = fmaf(cw.y, b.z, acc[1].z); acc[1].w = fmaf(cw.y, b.w, acc[1].w);
                acc[2].x = fmaf(cw.z, b.x, acc[2].x); acc[2].y = fmaf(cw.z, b.y, acc[2].y);
                acc[2].z = fmaf(cw.z, b.z, acc[2].z); acc[2].w = fmaf(cw.z, b.w, acc[2].w);
                acc[3].x = fmaf(cw.w, b.x, acc[3].x); acc[3].y = fmaf(cw.w, b.y, acc[3].y);
                acc[3].z = fmaf(cw.w, b.z, acc[3].z); acc[3].w = fmaf(cw.w, b.w, acc[3].w);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int row = i0 + 4 * ii4 + a;
                if (row < nc) {
                    float4* p = reinterpret_cast<float4*>(Ag + (size_t)row * ldg) + r4;
                    if (track_diff) {
                        const float4 o = *p;
                        const float dx = acc[a].x - o.x, dy = acc[a].y - o.y;
                        const float dz = acc[a].z - o.z, dw = acc[a].w - o.w;
                        dsum = fmaf(dx, dx, dsum);
                        dsum = fmaf(dy, dy, dsum);
                        dsum = fmaf(dz, dz, dsum);
                        dsum = fmaf(dw, dw, dsum);
                    }
                    *p = acc[a];
                }
            }
        }
        __syncthreads();
    }
    return dsum;
}

// LDS carve-up shared by the setup and SVT steps.
struct SvtLds {
    float* B;
    float* xblk;
    float* cwt;
    float* s2;
    float* w;
    int* act;
};

__device__ inline SvtLds carve_lds(float* base, int nc, int ld, int tb) {
    SvtLds L;
    const int nc4 = (nc + 3) & ~3;
    L.B = base;
    L.xblk = L.B + nc4 * ld;
    L.cwt = L.xblk + tb * ld;
    L.s2 = L.cwt + nc4 * tb;
    L.w = L.s2 + nc4;
    L.act = reinterpret_cast<int*>(L.w + nc4);
    return L;
}

// Tiled SVT: the staged super-block pair (2 sb rows of stride ld, followed
// by their 2 sb rotation rows when warm-started) and the reconstruction
// blocks (tb rows of stride ldg, ncp x tb products) share the front of LDS;
// the per-row arrays follow.
__device__ inline SvtLds carve_lds_tiled(float* base, int sb, int ncp, int ld, int ldg, int tb, bool warm) {
    SvtLds L;
    L.B = base;
    L.xblk = base;
    L.cwt = L.xblk + tb * ldg;
    const int front = max((warm ? 4 : 2) * sb * ld, tb * ldg + ncp * tb);
    L.s2 = base + front;
    L.w = L.s2 + ncp;
    L.act = reinterpret_cast<int*>(L.w + ncp);
    return L;
}

// Singular values (squared, into L.s2, rows 0..nc-1) of the X-layout plane
// X: the Jacobi runs on LDS (rows in L.B) or, tiled, on the working plane
// Bg, which then holds the orthogonalised rows.
__device__ void svd_rows(const PatchDesc& d, const float* X, float* Bg, const SvtLds& L, float tol, int max_sweeps,
                         JacobiStats& js);


// Zero the LDS padding of the Jacobi matrix: columns [ldg, ld) of every
// row and the extra rows nc..nc4-1 (nc rounded up to a multiple of 4).
__device__ void clear_lds_padding(float* B, int nc, int ldg, int ld) {
    const int tid = threadIdx.x;
    const int padw4 = (ld - ldg) >> 2;
    for (int idx = tid; idx < nc * padw4; idx += NT) {
        const int row = idx / padw4, c = idx - row * padw4;
        *reinterpret_cast<float4*>(B + row * ld + ldg + 4 * c) = f4(0.f);
    }
    const int nc4 = (nc + 3) & ~3;
    const int ld4 = ld >> 2;
    for (int idx = tid; idx < (nc4 - nc) * ld4; idx += NT) {
        const int row = nc + idx / ld4, c = idx - (row - nc) * ld4;
        *reinterpret_cast<float4*>(B + row * ld + 4 * c) = f4(0.f);
    }
}

// Load an X-layout plane into the Jacobi matrix in LDS and clear padding.
__device__ void load_rows_lds(const float* Xg, int nc, int ldg, int ld, float* B) {
    const int tid = threadIdx.x;
    const int nr4 = ldg >> 2;
    for (int idx = tid; idx < nc * nr4; idx += NT) {
        const int row = idx / nr4, c = idx - row * nr4;
        *reinterpret_cast<float4*>(B + row * ld + 4 * c) = reinterpret_cast<const float4*>(Xg + (size_t)row * ldg)[c];
    }
    clear_lds_padding(B, nc, ldg, ld);
    __syncthreads();
}

__device__ void svd_rows(const PatchDesc& d, const float* X, float* Bg, const SvtLds& L, float tol, int max_sweeps,
                         JacobiStats& js) {
    if (d.sb > 0) {
        const int nr4 = d.ldg >> 2;
        for (int idx = threadIdx.x; idx < d.ncp * nr4; idx += NT) {
            const int row = idx / nr4, c = idx - row * nr4;
            float4 v = f4(0.f);
            if (row < d.nc) v = reinterpret_cast<const float4*>(X + (size_t)row * d.ldg)[c];
            reinterpret_cast<float4*>(Bg + (size_t)row * d.ldg)[c] = v;
        }
        __syncthreads();
        jacobi_tiled(d.svt_cfg, Bg, nullptr, d.sb, d.nsb, d.ldg, d.ld, L.B, tol, max_sweeps, js, d.gang);
        row_norms_global(Bg, d.nc, d.ldg, L.s2);
    } else {
        load_rows_lds(X, d.nc, d.ldg, d.ld, L.B);
        jacobi_dispatch(d.svt_cfg, L.B, d.nc, d.ld, tol, max_sweeps, js, L.s2);
    }
}

__device__ inline SvtLds carve_for(const PatchDesc& d, float* lds) {
    return d.sb > 0 ? carve_lds_tiled(lds, d.sb, d.ncp, d.ld, d.ldg, d.tb, d.warm != 0)
                    : carve_lds(lds, d.nc, d.ld, d.tb);
}

// ---------------------------------------------------------------------------
// Geometry (Alg. 1 Step 1): bilinear sample and the coordinate Jacobian.
// ---------------------------------------------------------------------------

__device__ inline void xlayout_to_ij(const PatchDesc& d, int row, int col, int& i, int& j) {
    if (d.colmajor) {
        j = row;
        i = col;
    } else {
        i = row;
        j = col;
    }
}

constexpr double kSnap = 1e-9;  // pixels

// Sample D o tau at grid point (i, j) and the raw Jacobian d(D o tau)/dtau.
// Bilinear interpolation written as two horizontal lerps and one vertical
// lerp; its partial derivatives are the exact ones of that interpolant.
__device__ inline float warp_pixel(const PatchDesc& d, const double* h, int i, int j, float* jraw) {
    const double s = d.s;
    const double ut = ((double)j - 0.5 * (double)(d.n - 1)) / s;
    const double vt = ((double)i - 0.5 * (double)(d.m - 1)) / s;
    const double X = h[0] * ut + h[1] * vt + h[2];
    const double Y = h[3] * ut + h[4] * vt + h[5];
    const double Wh = h[6] * ut + h[7] * vt + 1.0;
    const double iw = 1.0 / Wh;
    const double xt = X * iw, yt = Y * iw;
    const double x = s * xt + d.cx, y = s * yt + d.cy;
    const double xc = fmin(fmax(x, 0.0), (double)(d.W - 1));
    const double yc = fmin(fmax(y, 0.0), (double)(d.H - 1));
    // A sample within SNAP of a pixel line belongs to the cell right of /
    // below it, so rounding of the coordinate cannot flip the cell (and the
    // one-sided gradient) of samples that sit on the pixel grid.
    const int x0 = min((int)floor(xc + kSnap), d.W - 2);
    const int y0 = min((int)floor(yc + kSnap), d.H - 2);
    const float fx = (float)(xc - (double)x0);
    const float fy = (float)(yc - (double)y0);
    const float* r0 = d.image + (long long)y0 * d.stride + x0;
    const float* r1 = r0 + d.stride;
    const float v00 = r0[0], v01 = r0[1], v10 = r1[0], v11 = r1[1];
    const float dtop = v01 - v00, dbot = v11 - v10;
    const float top = fmaf(fx, dtop, v00);
    const float bot = fmaf(fx, dbot, v10);
    const float val = fmaf(fy, bot - top, top);
    const bool inx = (x >= 0.0) && (x <= (double)(d.W - 1));
    const bool iny = (y >= 0.0) && (y <= (double)(d.H - 1));
    const float dl = v10 - v00, dr = v11 - v01;
    const float gx = inx ? fmaf(fy, dbot - dtop, dtop) : 0.f;
    const float gy = iny ? fmaf(fx, dr - dl, dl) : 0.f;
    const double sw = s * iw;
    const double gxd = gx, gyd = gy;
    jraw[0] = (float)(gxd * sw * ut);
    jraw[1] = (float)(gxd * sw * vt);
    jraw[2] = (float)(gxd * sw);
    jraw[3] = (float)(gyd * sw * ut);
    jraw[4] = (float)(gyd * sw * vt);
    jraw[5] = (float)(gyd * sw);
    jraw[6] = (float)(-(gxd * xt + gyd * yt) * sw * ut);
    jraw[7] = (float)(-(gxd * xt + gyd * yt) * sw * vt);
    return val;
}

__device__ inline void tau_to_h(const PatchState* st, int model, double* h) {
    for (int k = 0; k < 6; ++k) h[k] = st->tau[k];
    h[6] = model == 8 ? st->tau[6] : 0.0;
    h[7] = model == 8 ? st->tau[7] : 0.0;
}

// Gradient of the area of the image of the rectified rectangle w.r.t. tau
// (normalised units), from the shoelace formula over the corners TL, TR, BR, BL.
__device__ void area_gradient(const PatchDesc& d, const double* h, double* g) {
    const double a = (double)(d.n - 1) / (2.0 * d.s);
    const double b = (double)(d.m - 1) / (2.0 * d.s);
    const double cu[4] = {-a, a, a, -a};
    const double cv[4] = {-b, -b, b, b};
    double xs[4], ys[4], dx[4][MAXP], dy[4][MAXP];
    for (int c = 0; c < 4; ++c) {
        const double u = cu[c], v = cv[c];
        const double X = h[0] * u + h[1] * v + h[2];
        const double Y = h[3] * u + h[4] * v + h[5];
        const double Wd = h[6] * u + h[7] * v + 1.0;
        const double xt = X / Wd, yt = Y / Wd;
        xs[c] = xt;
        ys[c] = yt;
        for (int k = 0; k < MAXP; ++k) dx[c][k] = dy[c][k] = 0.0;
        dx[c][0] = u / Wd;
        dx[c][1] = v / Wd;
        dx[c][2] = 1.0 / Wd;
        dy[c][3] = u / Wd;
        dy[c][4] = v / Wd;
        dy[c][5] = 1.0 / Wd;
        dx[c][6] = -xt * u / Wd;
        dx[c][7] = -xt * v / Wd;
        dy[c][6] = -yt * u / Wd;
        dy[c][7] = -yt * v / Wd;
    }
    for (int k = 0; k < MAXP; ++k) {
        double acc = 0.0;
        for (int c = 0; c < 4; ++c) {
            const int c2 = (c + 1) & 3;
            acc += dx[c][k] * ys[c2] + xs[c] * dy[c2][k] - dx[c2][k] * ys[c] - xs[c2] * dy[c][k];
        }
        g[k] = 0.5 * acc;
    }
    if (d.model != 8) g[6] = g[7] = 0.0;
}

// Orthonormal basis of null(Q) with Q = [e_h13; e_h23; grad area]: the
// translation entries are frozen and a Householder reflection of the area
// gradient restricted to the other entries spans its complement.
__device__ bool null_basis(const PatchDesc& d, const double* g, double* NQ) {
    const int p = d.model;
    int idx[MAXP];
    int f = 0;
    for (int k = 0; k < p; ++k)
        if (k != 2 && k != 5) idx[f++] = k;
    double v[MAXP];
    double nrm2 = 0.0;
    for (int a = 0; a < f; ++a) {
        v[a] = g[idx[a]];
        nrm2 += v[a] * v[a];
    }
    for (int k = 0; k < MAXP * MAXPP; ++k) NQ[k] = 0.0;
    if (!(nrm2 > 0.0)) return false;
    const double nrm = sqrt(nrm2);
    v[0] += (v[0] >= 0.0 ? nrm : -nrm);
    double vv = 0.0;
    for (int a = 0; a < f; ++a) vv += v[a] * v[a];
    // H = I - 2 v v^T / (v^T v); columns 1..f-1 span grad^perp.
    for (int col = 1; col < f; ++col) {
        for (int a = 0; a < f; ++a) {
            const double hv = (a == col ? 1.0 : 0.0) - 2.0 * v[a] * v[col] / vv;
            NQ[idx[a] * MAXPP + (col - 1)] = hv;
        }
    }
    return true;
}

// Packed upper-triangle index of (l, l2), l <= l2 < MAXPP (constant after
// unrolling, so the Gram accumulators stay in registers).
constexpr int NTRI = MAXPP * (MAXPP + 1) / 2;
__host__ __device__ constexpr int tri(int l, int l2) { return l * MAXPP - l * (l - 1) / 2 + (l2 - l); }

// Cholesky G = R^T R of a pp x pp SPD matrix (row-major, upper R).
__device__ bool cholesky_upper(const double* G, int pp, double* R) {
    for (int k = 0; k < MAXPP * MAXPP; ++k) R[k] = 0.0;
    #pragma unroll
    for (int i = 0; i < MAXPP; ++i) if (i < pp) {
        double s = G[i * MAXPP + i];
        for (int k = 0; k < i; ++k) s -= R[k * MAXPP + i] * R[k * MAXPP + i];
        if (!(s > 0.0)) return false;
        const double rii = sqrt(s);
        R[i * MAXPP + i] = rii;
        for (int j = i + 1; j < pp; ++j) {
            double t = G[i * MAXPP + j];
            for (int k = 0; k < i; ++k) t -= R[k * MAXPP + i] * R[k * MAXPP + j];
            R[i * MAXPP + j] = t / rii;
        }
    }
    return true;
}

// x = y R^{-1} for a row vector y (forward substitution on R^T); unrolled so
// that x and y stay in registers.
__device__ inline void solve_row_upper(const double* R, int pp, const double* y, double* x) {
#pragma unroll
    for (int l = 0; l < MAXPP; ++l) {
        if (l < pp) {
            double s = y[l];
#pragma unroll
            for (int k = 0; k < MAXPP; ++k)
                if (k < l) s -= x[k] * R[k * MAXPP + l];
            x[l] = s / R[l * MAXPP + l];
        } else {
            x[l] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Step 1 + constraints + warm start
// ---------------------------------------------------------------------------

__device__ void dev_factor(const PatchDesc& d, PatchState* st, const SolverParams& prm, float* lds,
                           const double* gram);

__device__ void dev_setup(const PatchDesc& d, PatchState* st, const SolverParams& prm, float* lds) {
    __shared__ double sh_sIJ[MAXP];
    __shared__ double sh_norm;
    __shared__ double sh_NQ[MAXP * MAXPP];
    __shared__ int sh_fail;

    const int tid = threadIdx.x;
    const int p = d.model, pp = d.pp;
    const int ldg = d.ldg, nr = d.nr, nc = d.nc;
    const size_t np = (size_t)nc * ldg;
    float* I = d.ws + PL_I * np;
    float* A = d.ws + PL_A * np;
    float* E = d.ws + PL_E * np;
    float* Y = d.ws + PL_Y * np;
    float* R = d.ws + PL_R * np;
    float* Qp = d.ws + PL_Q * np;
    const bool first = (st->outer == 0);

    double h[8];
    tau_to_h(st, p, h);

    // Pass A: warp, raw Jacobian, ||I||^2 and I^T J_raw.
    double acc[1 + MAXP];
#pragma unroll
    for (int k = 0; k <= MAXP; ++k) acc[k] = 0.0;
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) {
            I[e] = 0.f;
            #pragma unroll
            for (int k = 0; k < MAXP; ++k) if (k < p) Qp[k * np + e] = 0.f;
            continue;
        }
        int i, j;
        xlayout_to_ij(d, row, col, i, j);
        float jr[MAXP];
        const float val = warp_pixel(d, h, i, j, jr);
        I[e] = val;
        acc[0] += (double)val * (double)val;
        #pragma unroll
        for (int k = 0; k < MAXP; ++k) if (k < p) {
            Qp[k * np + e] = jr[k];
            acc[1 + k] += (double)val * (double)jr[k];
        }
    }
    block_sum_d<1 + MAXP>(acc);
    if (tid == 0) {
        sh_norm = sqrt(acc[0]);
        for (int k = 0; k < MAXP; ++k) sh_sIJ[k] = acc[1 + k];
        double g[MAXP];
        area_gradient(d, h, g);
        const bool ok = null_basis(d, g, sh_NQ) && (sh_norm > 0.0) && isfinite(sh_norm);
        sh_fail = ok ? 0 : 1;
        for (int k = 0; k < MAXP * MAXPP; ++k) st->NQ[k] = sh_NQ[k];
    }
    __syncthreads();
    if (sh_fail) {
        if (tid == 0) {
            st->status = (isfinite(sh_norm) ? -4 : -5);
            st->done_outer = 1;
            st->done_inner = 1;
        }
        __syncthreads();
        return;
    }
    const double inv_n = 1.0 / sh_norm;
    const double inv_n3 = inv_n * inv_n * inv_n;

    // Pass B: normalise, J = J_raw/|I| - I (I^T J_raw)/|I|^3, J~ = J N_Q, Gram.
    double gram[NTRI];
#pragma unroll
    for (int k = 0; k < NTRI; ++k) gram[k] = 0.0;
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) {
            if (first) A[e] = E[e] = Y[e] = 0.f;
            continue;
        }
        const double val = (double)I[e];
        double jt[MAXPP];
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) jt[l] = 0.0;
        #pragma unroll
        for (int k = 0; k < MAXP; ++k) if (k < p) {
            const double jk = (double)Qp[k * np + e] * inv_n - val * sh_sIJ[k] * inv_n3;
            #pragma unroll
            for (int l = 0; l < MAXPP; ++l) if (l < pp) jt[l] += jk * sh_NQ[k * MAXPP + l];
        }
        const float vn = (float)(val * inv_n);
        I[e] = vn;
        if (first) {
            A[e] = vn;
            E[e] = 0.f;
            Y[e] = 0.f;
        }
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            const float f = (float)jt[l];
            Qp[l * np + e] = f;
            jt[l] = (double)f;
        }
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l)
            #pragma unroll
            for (int l2 = 0; l2 < MAXPP; ++l2)
                if (l <= l2 && l2 < pp) gram[tri(l, l2)] += jt[l] * jt[l2];
    }
    block_sum_d<NTRI>(gram);
    dev_factor(d, st, prm, lds, gram);
}

// Passes C-E of the set-up, shared with the inner-loop-only entry: given
// the Gram sums of J~ (upper triangle, FP64), the Cholesky-QR2 basis Qb of
// J~ (stored over J~), the factor R (J~ = Qb R), the warm-start projection
// of Y, R_0 = J~perp(A + E - I), c = ||J~perp I||_F and mu_0.
__device__ void dev_factor(const PatchDesc& d, PatchState* st, const SolverParams& prm, float* lds,
                           const double* gram) {
    __shared__ double sh_R[MAXPP * MAXPP];
    __shared__ double sh_R1[MAXPP * MAXPP];
    __shared__ int sh_fail;
    const int tid = threadIdx.x;
    const int pp = d.pp;
    const int ldg = d.ldg, nr = d.nr, nc = d.nc;
    const size_t np = (size_t)nc * ldg;
    float* I = d.ws + PL_I * np;
    float* A = d.ws + PL_A * np;
    float* E = d.ws + PL_E * np;
    float* Y = d.ws + PL_Y * np;
    float* R = d.ws + PL_R * np;
    float* Qp = d.ws + PL_Q * np;
    if (tid == 0) {
        double G[MAXPP * MAXPP];
        for (int l = 0; l < MAXPP; ++l)
            for (int l2 = l; l2 < MAXPP; ++l2) {
                G[l * MAXPP + l2] = gram[tri(l, l2)];
                G[l2 * MAXPP + l] = gram[tri(l, l2)];
            }
        sh_fail = cholesky_upper(G, pp, sh_R1) ? 0 : 1;
    }
    __syncthreads();
    if (sh_fail) {
        if (tid == 0) {
            st->status = -4;
            st->done_outer = 1;
            st->done_inner = 1;
        }
        __syncthreads();
        return;
    }

    // Pass C: second Gram of J~ R1^{-1} (Cholesky-QR, second pass).
    double gram2[NTRI];
#pragma unroll
    for (int k = 0; k < NTRI; ++k) gram2[k] = 0.0;
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) continue;
        double y[MAXPP], x[MAXPP];
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) y[l] = (double)Qp[l * np + e];
        solve_row_upper(sh_R1, pp, y, x);
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l)
            #pragma unroll
            for (int l2 = 0; l2 < MAXPP; ++l2)
                if (l <= l2 && l2 < pp) gram2[tri(l, l2)] += x[l] * x[l2];
    }
    block_sum_d<NTRI>(gram2);
    if (tid == 0) {
        double G[MAXPP * MAXPP], R2[MAXPP * MAXPP];
        for (int l = 0; l < MAXPP; ++l)
            for (int l2 = l; l2 < MAXPP; ++l2) {
                G[l * MAXPP + l2] = gram2[tri(l, l2)];
                G[l2 * MAXPP + l] = gram2[tri(l, l2)];
            }
        const bool ok = cholesky_upper(G, pp, R2);
        sh_fail = ok ? 0 : 1;
        // R = R2 R1
        for (int i = 0; i < MAXPP; ++i)
            for (int j = 0; j < MAXPP; ++j) {
                double s = 0.0;
                for (int k = 0; k < MAXPP; ++k) s += R2[i * MAXPP + k] * sh_R1[k * MAXPP + j];
                sh_R[i * MAXPP + j] = s;
                st->R[i * MAXPP + j] = s;
            }
    }
    __syncthreads();
    if (sh_fail) {
        if (tid == 0) {
            st->status = -4;
            st->done_outer = 1;
            st->done_inner = 1;
        }
        __syncthreads();
        return;
    }

    // Pass D: Qb = J~ R^{-1} (stored), coefficients of Y, A + E - I and I.
    float co[3 * MAXPP];
#pragma unroll
    for (int k = 0; k < 3 * MAXPP; ++k) co[k] = 0.f;
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) continue;
        double y[MAXPP], x[MAXPP];
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) y[l] = (double)Qp[l * np + e];
        solve_row_upper(sh_R, pp, y, x);
        const float iv = I[e];
        const float yv = Y[e];
        const float sv = A[e] + E[e] - iv;
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            const float qb = (float)x[l];
            Qp[l * np + e] = qb;
            co[l] = fmaf(qb, yv, co[l]);
            co[MAXPP + l] = fmaf(qb, sv, co[MAXPP + l]);
            co[2 * MAXPP + l] = fmaf(qb, iv, co[2 * MAXPP + l]);
        }
    }
    block_sum_f<3 * MAXPP>(co);

    // Pass E: Y <- J~perp Y (Eq. warm_start_Y), R <- J~perp(A + E - I),
    // c^2 = ||J~perp I||^2.
    float c2[1] = {0.f};
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) {
            R[e] = 0.f;
            continue;
        }
        const float iv = I[e];
        float yv = Y[e];
        float sv = A[e] + E[e] - iv;
        float ci = iv;
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            const float qb = Qp[l * np + e];
            yv = fmaf(-qb, co[l], yv);
            sv = fmaf(-qb, co[MAXPP + l], sv);
            ci = fmaf(-qb, co[2 * MAXPP + l], ci);
        }
        Y[e] = yv;
        R[e] = sv;
        c2[0] = fmaf(ci, ci, c2[0]);
    }
    block_sum_f<1>(c2);

    // mu_0 = 1.25 / ||I||_2 from the Jacobi singular values of I.
    double mu0 = prm.mu0;
    if (!(mu0 > 0.0)) {
        const SvtLds L = carve_for(d, lds);
        JacobiStats js{0, 0, 0};
        svd_rows(d, I, d.ws + NPLANES * np, L, svt_tolerance_cap(prm.jacobi_tol, d.nr), prm.max_sweeps, js);
        __shared__ float sh_smax;
        if (tid == 0) {
            float mx = 0.f;
            for (int j = 0; j < nc; ++j) mx = fmaxf(mx, L.s2[j]);
            sh_smax = sqrtf(mx);
            st->svt_calls += 1;
            st->sweeps += js.sweeps;
            st->pairs += js.pairs;
            st->rotations += js.rotations;
        }
        __syncthreads();
        mu0 = 1.25 / (double)sh_smax;
    }
    if (tid == 0) {
        st->c = sqrt((double)c2[0]);
        st->mu = mu0;
        st->inner = 0;
        st->done_inner = 0;
        if (!(st->c > 0.0) || !isfinite(mu0)) {
            st->status = -5;
            st->done_outer = 1;
            st->done_inner = 1;
        }
    }
    __syncthreads();
}

// Inner loop alone (the setting of Table 1): I (row-major m x n) and the p
// columns of J (parameter-major, p x m x n) are given; no normalisation and
// no extra constraints (J~ = J, p <= 5); A = I, E = Y = 0; then the
// factorisation of the set-up.
__device__ void dev_setup_given(const PatchDesc& d, PatchState* st, const SolverParams& prm, float* lds,
                                const float* Iin, const float* Jin) {
    const int tid = threadIdx.x;
    const int pp = d.pp;
    const int ldg = d.ldg, nr = d.nr, nc = d.nc;
    const size_t np = (size_t)nc * ldg;
    const size_t mn = (size_t)d.m * d.n;
    float* I = d.ws + PL_I * np;
    float* A = d.ws + PL_A * np;
    float* E = d.ws + PL_E * np;
    float* Y = d.ws + PL_Y * np;
    float* Qp = d.ws + PL_Q * np;
    double gram[NTRI];
#pragma unroll
    for (int k = 0; k < NTRI; ++k) gram[k] = 0.0;
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) {
            I[e] = A[e] = E[e] = Y[e] = 0.f;
#pragma unroll
            for (int l = 0; l < MAXPP; ++l) if (l < pp) Qp[l * np + e] = 0.f;
            continue;
        }
        int i, j;
        xlayout_to_ij(d, row, col, i, j);
        const size_t src = (size_t)i * d.n + j;
        const float iv = Iin[src];
        I[e] = iv;
        A[e] = iv;
        E[e] = 0.f;
        Y[e] = 0.f;
        double jt[MAXPP];
#pragma unroll
        for (int l = 0; l < MAXPP; ++l)
            if (l < pp) {
                const float f = Jin[(size_t)l * mn + src];
                Qp[l * np + e] = f;
                jt[l] = (double)f;
            }
#pragma unroll
        for (int l = 0; l < MAXPP; ++l)
#pragma unroll
            for (int l2 = 0; l2 < MAXPP; ++l2)
                if (l <= l2 && l2 < pp) gram[tri(l, l2)] += jt[l] * jt[l2];
    }
    block_sum_d<NTRI>(gram);
    dev_factor(d, st, prm, lds, gram);
}

// ---------------------------------------------------------------------------
// Warm-started SVT.  The rows of R (nc x nc, orthonormal) are the product of
// all Jacobi rotations applied so far; the decomposition of the next
// iterate starts from B = R M, whose rows are already nearly orthogonal
// when M changed little, and the new rotations are accumulated into R.
// Rounding slowly erodes the orthonormality of R, so every few calls one
// Newton-Schulz step R <- 1.5 R - 0.5 (R R^T) R restores it.  The SVT
// result is built from B and M as in the cold case, so its accuracy rests
// on R being orthogonal to rounding level, not on the quality of the start.
// ---------------------------------------------------------------------------

// LDS: B (nc4 x ld) | R (nc4 x ld), with the reconstruction blocks reusing
// the R area after R has been saved | s2, w, act.
__device__ inline SvtLds carve_lds_warm(float* base, int nc, int ld, int tb, float** Rl) {
    SvtLds L;
    const int nc4 = (nc + 3) & ~3;
    L.B = base;
    *Rl = base + nc4 * ld;
    L.xblk = *Rl;
    L.cwt = L.xblk + tb * ld;
    L.s2 = *Rl + max(nc4 * ld, tb * ld + nc4 * tb);
    L.w = L.s2 + nc4;
    L.act = reinterpret_cast<int*>(L.w + nc4);
    return L;
}

typedef float tilt_floatx4 __attribute__((ext_vector_type(4)));

// C = A B on the matrix cores (FP32 in, FP32 accumulate): C is M x N, A is
// M x K (row stride lda), B is K x N with B[k][j] = Bm[k * ldb + j], or
// Bm[j * ldb + k] when BT.  16 x 16 output tiles, one wavefront per tile,
// v_mfma_f32_16x16x4f32 over k in steps of 4: lane l supplies
// A[i0 + l % 16][k0 + l / 16] and B[k0 + l / 16][j0 + l % 16] and receives
// rows i0 + 4 (l / 16) + r, r = 0..3, of column j0 + l % 16.  Operands
// outside M, N, K read as 0 and results outside M x N are not stored.
template <bool BT>
__device__ void mfma_gemm(const float* A, int lda, int M, const float* Bm, int ldb, int N, int K, float* C,
                          int ldc) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ti = (M + 15) >> 4, tj = (N + 15) >> 4;
    const int li = lane & 15, lk = lane >> 4;
    for (int t = wv; t < ti * tj; t += NWAVE) {
        const int tr = t / tj;
        const int i0 = tr * 16, j0 = (t - tr * tj) * 16;
        tilt_floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        const int i = i0 + li, j = j0 + li;
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + lk;
            const float a = (i < M && k < K) ? A[(size_t)i * lda + k] : 0.f;
            float b = 0.f;
            if (k < K && j < N) b = BT ? Bm[(size_t)j * ldb + k] : Bm[(size_t)k * ldb + j];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int oi = i0 + 4 * lk + r;
            if (oi < M && j < N) C[(size_t)oi * ldc + j] = acc[r];
        }
    }
}

typedef short tilt_short4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ inline short to_bf16(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// C = A B with A and B rounded to bfloat16 and FP32 accumulation on the
// matrix cores (v_mfma_f32_16x16x16bf16_1k: lane l supplies
// A[i0 + l % 16][k0 + 4 (l / 16) + u] and B[k0 + 4 (l / 16) + u][j0 + l % 16],
// u = 0..3; output layout as in mfma_gemm).  Same operand conventions and
// bounds as mfma_gemm<false>.
__device__ void mfma_gemm_bf16(const float* A, int lda, int M, const float* Bm, int ldb, int N, int K, float* C,
                               int ldc) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ti = (M + 15) >> 4, tj = (N + 15) >> 4;
    const int li = lane & 15, lk = lane >> 4;
    for (int t = wv; t < ti * tj; t += NWAVE) {
        const int tr = t / tj;
        const int i0 = tr * 16, j0 = (t - tr * tj) * 16;
        tilt_floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        const int i = i0 + li, j = j0 + li;
        for (int k0 = 0; k0 < K; k0 += 16) {
            tilt_short4 av, bv;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + 4 * lk + u;
                av[u] = (i < M && k < K) ? to_bf16(A[(size_t)i * lda + k]) : (short)0;
                bv[u] = (k < K && j < N) ? to_bf16(Bm[(size_t)k * ldb + j]) : (short)0;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int oi = i0 + 4 * lk + r;
            if (oi < M && j < N) C[(size_t)oi * ldc + j] = acc[r];
        }
    }
}

// R <- 1.5 R - 0.5 (R R^T) R on the nc x nc rotation in LDS (stride ld).
// G = R R^T goes to Gs (LDS, stride ld), T = G R to the device plane T
// (stride ldg).
__device__ void newton_schulz_rows(float* Rl, int ld, int nc, float* Gs, float* T, int ldg) {
    mfma_gemm<true>(Rl, ld, nc, Rl, ld, nc, nc, Gs, ld);
    __syncthreads();
    mfma_gemm<false>(Gs, ld, nc, Rl, ld, nc, nc, T, ldg);
    __syncthreads();
    for (int e = threadIdx.x; e < nc * nc; e += NT) {
        const int i = e / nc, j = e - i * nc;
        Rl[i * ld + j] = fmaf(-0.5f, T[(size_t)i * ldg + j], 1.5f * Rl[i * ld + j]);
    }
    __syncthreads();
}

// Load the saved rotation (or the identity) into the R area: rows and
// columns beyond nc are zero.
__device__ void load_rotation(float* Rl, int ld, int nc, const float* V, int ldg, bool saved) {
    const int nc4 = (nc + 3) & ~3;
    const int ld4 = ld >> 2;
    for (int e = threadIdx.x; e < nc4 * ld4; e += NT) {
        const int i = e / ld4, c = e - i * ld4;
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * c + u;
            v[u] = 0.f;
            if (i < nc && j < nc) v[u] = saved ? V[(size_t)i * ldg + j] : (i == j ? 1.f : 0.f);
        }
        *reinterpret_cast<float4*>(Rl + i * ld + 4 * c) = make_float4(v[0], v[1], v[2], v[3]);
    }
    __syncthreads();
}

__device__ void save_rotation(const float* Rl, int ld, int nc, float* V, int ldg) {
    for (int e = threadIdx.x; e < nc * nc; e += NT) {
        const int i = e / nc, j = e - i * nc;
        V[(size_t)i * ldg + j] = Rl[i * ld + j];
    }
    __syncthreads();
}

// Tiled matrices: the rotation is an ncp x ldg device plane whose first nc
// rows and columns hold R; everything else stays zero (padding rows of the
// Jacobi matrix are zero and never rotate, so their rotation rows never
// change).
__device__ void rotation_identity_global(float* Rg, int nc, int ncp, int ldg) {
    for (size_t e = threadIdx.x; e < (size_t)ncp * ldg; e += NT) {
        const int i = (int)(e / ldg), j = (int)(e - (size_t)i * ldg);
        Rg[e] = (i == j && i < nc) ? 1.f : 0.f;
    }
    __syncthreads();
}

// R <- 1.5 R - 0.5 (R R^T) R on the rotation plane: G = R R^T into the
// device plane G, T = G R into T (both nc x nc, stride ldg).
__device__ void newton_schulz_global(float* Rg, int nc, int ldg, float* G, float* T, float* unused) {
    (void)unused;
    mfma_gemm<true>(Rg, ldg, nc, Rg, ldg, nc, nc, G, ldg);
    __threadfence_block();
    __syncthreads();
    mfma_gemm<false>(G, ldg, nc, Rg, ldg, nc, nc, T, ldg);
    __threadfence_block();
    __syncthreads();
    for (int e = threadIdx.x; e < nc * nc; e += NT) {
        const int i = e / nc, j = e - i * nc;
        const size_t o = (size_t)i * ldg + j;
        Rg[o] = fmaf(-0.5f, T[o], 1.5f * Rg[o]);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// A-update: M = A - R - Y/mu, A <- S_{1/mu}(M)
// ---------------------------------------------------------------------------

// M_k = A_k - J~perp(A_k + E_k - I) - Y_k/mu_k (R = J~perp(A_k + E_k - I)),
// into the M plane and, when Bl is given, into the LDS Jacobi matrix.
__device__ void svt_form_m(const PatchDesc& d, const PatchState* st, float* Bl) {
    const int nc = d.nc, ldg = d.ldg, ld = d.ld;
    const int nr4 = ldg >> 2;
    const size_t np = (size_t)nc * ldg;
    const float* A = d.ws + PL_A * np;
    const float* R = d.ws + PL_R * np;
    const float* Y = d.ws + PL_Y * np;
    float* M = d.ws + PL_M * np;
    const float inv_mu = (float)(1.0 / st->mu);
    for (int idx = threadIdx.x; idx < nc * nr4; idx += NT) {
        const int row = idx / nr4, c = idx - row * nr4;
        const size_t o = (size_t)row * ldg + 4 * c;
        const float4 a = *reinterpret_cast<const float4*>(A + o);
        const float4 r = *reinterpret_cast<const float4*>(R + o);
        const float4 y = *reinterpret_cast<const float4*>(Y + o);
        float4 mm;
        mm.x = fmaf(-y.x, inv_mu, a.x - r.x);
        mm.y = fmaf(-y.y, inv_mu, a.y - r.y);
        mm.z = fmaf(-y.z, inv_mu, a.z - r.z);
        mm.w = fmaf(-y.w, inv_mu, a.w - r.w);
        *reinterpret_cast<float4*>(M + o) = mm;
        if (Bl) *reinterpret_cast<float4*>(Bl + row * ld + 4 * c) = mm;
    }
}

// Shrinkage and reconstruction from the orthogonalised rows (LDS rows L.B,
// or the working plane when tiled) whose squared norms are in L.s2; A and
// the SVT statistics of the state are updated.
__device__ void svt_finish(const PatchDesc& d, PatchState* st, const SvtLds& L, const JacobiStats& js) {
    const int tid = threadIdx.x;
    const int nc = d.nc, ldg = d.ldg, ld = d.ld;
    const int nr4 = ldg >> 2;
    const size_t np = (size_t)nc * ldg;
    float* A = d.ws + PL_A * np;
    const float* M = d.ws + PL_M * np;
    const float* Bg = d.ws + NPLANES * np;
    const double mu = st->mu;
    const float eps = (float)(1.0 / mu);
    int k;
    double nuc;
    shrink_weights(L.s2, nc, eps, L.w, L.act, &k, &nuc);
    float dA[1];
    dA[0] = d.sb > 0
                ? reconstruct(Bg, ldg, M, A, nc, nr4, ldg, L.w, L.act, k, d.tb, L.xblk, L.cwt, true)
                : reconstruct(L.B, ld, M, A, nc, nr4, ldg, L.w, L.act, k, d.tb, L.xblk, L.cwt, true);
    block_sum_f<1>(dA);
    if (tid == 0) {
        // numerical rank of the result: its singular values are s_j - eps
        // for the kept rows
        double top = 0.0;
        for (int j = 0; j < nc; ++j) top = fmax(top, (double)sqrtf(L.s2[j]) - (double)eps);
        int nr_rank = 0;
        for (int j = 0; j < nc; ++j) nr_rank += ((double)sqrtf(L.s2[j]) - (double)eps) > 1e-3 * top ? 1 : 0;
        st->num_rank = top > 0.0 ? nr_rank : 0;
        st->dA2 = (double)dA[0];
        st->nuc = nuc;
        st->svt_rank = k;
        st->svt_calls += 1;
        st->sweeps += js.sweeps;
        st->pairs += js.pairs;
        st->rotations += js.rotations;
        st->recon_rows += k;
    }
    __syncthreads();
}

// Warm-started SVT of a tiled window (rare: only windows beyond LDS with
// svt_mode 1), kept out of line so that dev_svt's common paths keep their
// registers.
__device__ __noinline__ void svt_tiled_warm(const PatchDesc& d, PatchState* st, const SolverParams& prm,
                                            const SvtLds& L, float tol, JacobiStats& js) {
    const int nc = d.nc, ldg = d.ldg, ld = d.ld;
    const size_t np = (size_t)nc * ldg;
    float* M = d.ws + PL_M * np;
    float* Bg = d.ws + NPLANES * np;
    // The rotation lives in its own working plane (ncp rows, so that it
    // is staged by super-blocks with the Jacobi rows).
    float* Rg = Bg + (size_t)d.ncp * ldg;
    const bool saved = st->warm_ok != 0;
    __syncthreads();
    if (!saved) rotation_identity_global(Rg, nc, d.ncp, ldg);
    else if (prm.ns_every > 0 && st->warm_count % prm.ns_every == 0)
        newton_schulz_global(Rg, nc, ldg, d.ws + (PL_Q + 6) * np, d.ws + (PL_Q + 7) * np, Bg);
    // B = R M into the Jacobi rows (rows nc.. of Bg stay zero)
    mfma_gemm<false>(Rg, ldg, nc, M, ldg, ldg, nc, Bg, ldg);
    for (int e = threadIdx.x; e < (d.ncp - nc) * ldg; e += NT) Bg[(size_t)nc * ldg + e] = 0.f;
    __syncthreads();
    jacobi_tiled(d.svt_cfg, Bg, Rg, d.sb, d.nsb, ldg, ld, L.B, tol, prm.max_sweeps, js, d.gang);
    row_norms_global(Bg, nc, ldg, L.s2);
    if (threadIdx.x == 0) {
        st->warm_ok = 1;
        st->warm_count += 1;
    }
}


// ---------------------------------------------------------------------------
// SVD with warm start inside the loop (svt_mode 4; Sec. 5, Alg. 2).  The
// row layout holds X = M (nc x nr); the step works on the m = nr by n = nc
// matrix X^T, whose SVD after a full decomposition by the warm-started
// Jacobi is U = the normalised Jacobi rows (transposed), Sigma = their
// norms and V = the accumulated rotation (transposed), since B = R X with
// orthogonal rows.
// ---------------------------------------------------------------------------

#include "tilt_svdws.inc"

// A window's region after its solver planes (layout of svdws_region_words).
struct SvdwsRegion {
    float *U, *Mp, *Mn, *Uo, *Ao, *V, *Vo, *S, *So, *W;
};

__device__ inline SvdwsRegion svdws_region(const PatchDesc& d) {
    const size_t mn = svdws_round64((size_t)d.nr * d.nc), nn = svdws_round64((size_t)d.nc * d.nc);
    const size_t sv = svdws_round64(d.nc);
    float* p = d.ws + NPLANES * (size_t)d.nc * d.ldg;
    SvdwsRegion r;
    r.U = p;
    r.Mp = r.U + mn;
    r.Mn = r.Mp + mn;
    r.Uo = r.Mn + mn;
    r.Ao = r.Uo + mn;
    r.V = r.Ao + mn;
    r.Vo = r.V + nn;
    r.S = r.Vo + nn;
    r.So = r.S + sv;
    r.W = r.So + sv;
    return r;
}

// Before the Jacobi: X^T into the region, then Alg. 2's choice.  With a
// previous decomposition, the Cayley step is taken when ||X - X_prev||_F <
// eps_svd ||X||_F (or, with svdws_every > 0, in every inner iteration not
// divisible by it); if it succeeds, A (row layout) = U(t) T_eps(Sigma(t))
// V(t)^T, the decomposition moves on and the state's SVT statistics are
// set.  Returns 1 (uniform) if A was formed this way, 0 if a full SVD is
// needed.
__device__ __noinline__ int svdws_try(const PatchDesc& d, PatchState* st, const SolverParams& prm) {
    const int m = d.nr, n = d.nc, ldg = d.ldg;
    const int mn = m * n;
    const size_t np = (size_t)d.nc * ldg;
    const float* M = d.ws + PL_M * np;
    float* A = d.ws + PL_A * np;
    const SvdwsRegion R = svdws_region(d);
    const int have = st->svdws_ok;
    __syncthreads();  // M was written by every thread of the workgroup (svt_form_m)
    double sums[2] = {0.0, 0.0};
    for (int e = threadIdx.x; e < mn; e += NT) {
        const int i = e / n, j = e - i * n;
        const float v = M[(size_t)j * ldg + i];
        R.Mn[e] = v;
        if (have) {
            const double dv = (double)v - (double)R.Mp[e];
            sums[0] += dv * dv;
            sums[1] += (double)v * (double)v;
        }
    }
    block_sum_d<2>(sums);
    int use = 0;
    if (have) use = prm.svdws_every > 0 ? (st->inner % prm.svdws_every) != 0 : sqrt(sums[0]) < prm.eps_svd * sqrt(sums[1]);
    if (!use) return 0;
    const float eps = (float)(1.0 / st->mu);
    double t, f0, ft;
    if (svdws_step(m, n, R.U, R.S, R.V, R.Mn, R.Uo, R.So, R.Vo, R.Ao, eps, R.W, t, f0, ft) != 0) return 0;
    float dA[1] = {0.f};
    for (int e = threadIdx.x; e < mn; e += NT) {
        const int i = e / n, j = e - i * n;
        const size_t o = (size_t)j * ldg + i;
        const float v = R.Ao[e];
        const float diff = v - A[o];
        dA[0] = fmaf(diff, diff, dA[0]);
        A[o] = v;
        R.U[e] = R.Uo[e];
        R.Mp[e] = R.Mn[e];
    }
    for (int e = threadIdx.x; e < n * n; e += NT) R.V[e] = R.Vo[e];
    for (int j = threadIdx.x; j < n; j += NT) R.S[j] = R.So[j];
    block_sum_f<1>(dA);
    if (threadIdx.x == 0) {
        // A's singular values are |Sigma_j(t)| - eps for the kept ones
        int k = 0;
        double nuc = 0.0, top = 0.0;
        for (int j = 0; j < n; ++j) {
            const double a = fabs((double)R.So[j]) - (double)eps;
            if (a > 0.0) {
                k += 1;
                nuc += a;
                top = fmax(top, a);
            }
        }
        int nr_rank = 0;
        for (int j = 0; j < n; ++j) nr_rank += (fabs((double)R.So[j]) - (double)eps) > 1e-3 * top ? 1 : 0;
        st->num_rank = top > 0.0 ? nr_rank : 0;
        st->dA2 = (double)dA[0];
        st->nuc = nuc;
        st->svt_rank = k;
        st->svt_calls += 1;
        st->recon_rows += k;
        st->svdws_steps += 1;
    }
    __syncthreads();
    return 1;
}

// After a full SVD by the warm-started Jacobi (rows B and rotation Rl in
// LDS, squared row norms s2): its decomposition of X^T and X^T itself into
// the region for the next step.
__device__ __noinline__ void svdws_save(const PatchDesc& d, PatchState* st, const float* B, const float* Rl,
                                        const float* s2) {
    const int m = d.nr, n = d.nc, ld = d.ld;
    const SvdwsRegion R = svdws_region(d);
    for (int j = threadIdx.x; j < n; j += NT) R.S[j] = sqrtf(s2[j]);
    __syncthreads();
    for (int e = threadIdx.x; e < m * n; e += NT) {
        const int i = e / n, j = e - i * n;
        const float sj = R.S[j];
        R.U[e] = sj > 0.f ? B[j * ld + i] / sj : 0.f;
        R.Mp[e] = R.Mn[e];
    }
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e - i * n;
        R.V[e] = Rl[j * ld + i];
    }
    if (threadIdx.x == 0) st->svdws_ok = 1;
    __syncthreads();
}

__device__ void dev_svt(const PatchDesc& d, PatchState* st, const SolverParams& prm, float* lds) {
    const int nc = d.nc, ldg = d.ldg, ld = d.ld;
    const size_t np = (size_t)nc * ldg;
    float* M = d.ws + PL_M * np;
    const bool tiled = d.sb > 0;
    const bool warm = d.warm != 0;
    float* Bg = d.ws + NPLANES * np;
    float* Rl = nullptr;
    const SvtLds L = (warm && !tiled) ? carve_lds_warm(lds, nc, ld, d.tb, &Rl) : carve_for(d, lds);

    svt_form_m(d, st, (!tiled && !warm) ? L.B : nullptr);
    const float tol = svt_tolerance(prm.jacobi_tol, prm.eps2, st->mu, d.nr);
    JacobiStats js{0, 0, 0};
    if (warm && tiled) {
        svt_tiled_warm(d, st, prm, L, tol, js);
    } else if (warm) {
        if (d.warm == 4 && svdws_try(d, st, prm)) return;  // A formed by the Cayley step
        float* V = d.ws + PL_V * np;
        const bool saved = st->warm_ok != 0;
        load_rotation(Rl, ld, nc, V, ldg, saved);
        if (saved && prm.ns_every > 0 && st->warm_count % prm.ns_every == 0)
            newton_schulz_rows(Rl, ld, nc, L.B, d.ws + (PL_Q + 6) * np, ldg);
        // B = R M (nc4 x ldg; rows of R beyond nc are zero).  warm = 1, 4:
        // FP32 products.  warm = 2, 3: the start is formed from bfloat16 operands
        // (FP32 accumulation); 2 then refines: B = R' M again in FP32 with
        // the accumulated rotation R' and the Jacobi continues from there,
        // so the result has FP32 accuracy; 3 keeps the bfloat16 start
        // (precision study).
        const int nc4 = (nc + 3) & ~3;
        if (d.warm == 1 || d.warm == 4)
            mfma_gemm<false>(Rl, ld, nc4, M, ldg, ldg, nc, L.B, ld);
        else
            mfma_gemm_bf16(Rl, ld, nc4, M, ldg, ldg, nc, L.B, ld);
        clear_lds_padding(L.B, nc, ldg, ld);
        __syncthreads();
        jacobi_dispatch_warm(d.svt_cfg, L.B, Rl, nc, ld, tol, prm.max_sweeps, js, L.s2);
        if (d.warm == 2) {
            mfma_gemm<false>(Rl, ld, nc4, M, ldg, ldg, nc, L.B, ld);
            clear_lds_padding(L.B, nc, ldg, ld);
            __syncthreads();
            jacobi_dispatch_warm(d.svt_cfg, L.B, Rl, nc, ld, tol, prm.max_sweeps, js, L.s2);
        }
        if (d.warm == 4) svdws_save(d, st, L.B, Rl, L.s2);
        save_rotation(Rl, ld, nc, V, ldg);
        if (threadIdx.x == 0) {
            st->warm_ok = 1;
            st->warm_count += 1;
        }
    } else if (tiled) {
        __syncthreads();
        svd_rows(d, M, Bg, L, tol, prm.max_sweeps, js);
    } else {
        clear_lds_padding(L.B, nc, ldg, ld);
        __syncthreads();
        jacobi_dispatch(d.svt_cfg, L.B, nc, ld, tol, prm.max_sweeps, js, L.s2);
    }
    svt_finish(d, st, L, js);
}

// ---------------------------------------------------------------------------
// E-, Y- and mu-updates with the two J~perp products of Sec. 4.2
// ---------------------------------------------------------------------------

// Cond1, Cond2 (Eqs. Cond1, Cond2), the penalty update (Eqs. mu, rho) and
// the inner stop, from ||J~perp(A + E - I)||^2 and ||E_{k+1} - E_k||^2
// (||A_{k+1} - A_k||^2 is in the state).  One thread.
__device__ void finish_inner_iteration(PatchState* st, const SolverParams& prm, double r2, double dE2) {
    const double mu = st->mu;
    const double c = st->c;
    const double dA = sqrt(st->dA2), dE = sqrt(dE2);
    const double cond1 = sqrt(r2) / c;
    const double cond2 = mu * fmax(dA, dE) / c;
    st->cond1 = cond1;
    st->cond2 = cond2;
    st->inner += 1;
    st->inner_total += 1;
    int stop = 0;
    if (!isfinite(cond1) || !isfinite(cond2)) {
        st->status = -5;
        st->done_outer = 1;
        stop = 1;
    } else {
        if (!prm.fixed_iters && cond1 < prm.eps1 && cond2 < prm.eps2) stop = 1;
        if (!stop && cond2 < prm.eps2) st->mu = fmin(prm.mu_max, prm.rho0 * mu);
        if (!stop && st->inner >= prm.max_inner) {
            stop = 1;
            if (!prm.fixed_iters) st->warn = 1;
        }
    }
    st->done_inner = stop;
}

__device__ void dev_update(const PatchDesc& d, PatchState* st, const SolverParams& prm) {
    const int tid = threadIdx.x;
    const int pp = d.pp;
    const size_t np = (size_t)d.nc * d.ldg;
    const int n4 = (int)(np >> 2);
    const float4* A = reinterpret_cast<const float4*>(d.ws + PL_A * np);
    float4* E = reinterpret_cast<float4*>(d.ws + PL_E * np);
    const float4* I = reinterpret_cast<const float4*>(d.ws + PL_I * np);
    float4* Y = reinterpret_cast<float4*>(d.ws + PL_Y * np);
    float4* R = reinterpret_cast<float4*>(d.ws + PL_R * np);
    const float* Qp = d.ws + PL_Q * np;
    const double mu = st->mu;
    const float muf = (float)mu;
    const float inv_mu = (float)(1.0 / mu);
    const float thr = (float)(d.lam / mu);

    // t1 = Qb^T (A_{k+1} + E_k - I)
    float t1[MAXPP];
#pragma unroll
    for (int l = 0; l < MAXPP; ++l) t1[l] = 0.f;
    for (int e = tid; e < n4; e += NT) {
        const float4 a = A[e], ev = E[e], iv = I[e];
        const float4 s = make_float4(a.x + ev.x - iv.x, a.y + ev.y - iv.y, a.z + ev.z - iv.z, a.w + ev.w - iv.w);
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            const float4 q = reinterpret_cast<const float4*>(Qp + l * np)[e];
            float acc = t1[l];
            acc = fmaf(q.x, s.x, acc);
            acc = fmaf(q.y, s.y, acc);
            acc = fmaf(q.z, s.z, acc);
            acc = fmaf(q.w, s.w, acc);
            t1[l] = acc;
        }
    }
    block_sum_f<MAXPP>(t1);

    // N_k = E_k - J~perp(A_{k+1} + E_k - I) - Y_k/mu; E_{k+1} = T_{lam/mu}(N_k);
    // t2 = Qb^T (A_{k+1} + E_{k+1} - I).
    float t2[MAXPP + 1];
#pragma unroll
    for (int l = 0; l <= MAXPP; ++l) t2[l] = 0.f;
    for (int e = tid; e < n4; e += NT) {
        const float4 a = A[e], ev = E[e], iv = I[e], yv = Y[e];
        float s[4] = {a.x + ev.x - iv.x, a.y + ev.y - iv.y, a.z + ev.z - iv.z, a.w + ev.w - iv.w};
        float4 q[MAXPP];
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            q[l] = reinterpret_cast<const float4*>(Qp + l * np)[e];
            s[0] = fmaf(-q[l].x, t1[l], s[0]);
            s[1] = fmaf(-q[l].y, t1[l], s[1]);
            s[2] = fmaf(-q[l].z, t1[l], s[2]);
            s[3] = fmaf(-q[l].w, t1[l], s[3]);
        }
        const float eo[4] = {ev.x, ev.y, ev.z, ev.w};
        const float yy[4] = {yv.x, yv.y, yv.z, yv.w};
        const float aa[4] = {a.x, a.y, a.z, a.w};
        const float ii[4] = {iv.x, iv.y, iv.z, iv.w};
        float en[4], s2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float nv = fmaf(-yy[u], inv_mu, eo[u] - s[u]);
            const float mag = fabsf(nv) - thr;
            en[u] = mag > 0.f ? copysignf(mag, nv) : 0.f;
            const float de = en[u] - eo[u];
            t2[MAXPP] = fmaf(de, de, t2[MAXPP]);
            s2[u] = aa[u] + en[u] - ii[u];
        }
        E[e] = make_float4(en[0], en[1], en[2], en[3]);
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            float acc = t2[l];
            acc = fmaf(q[l].x, s2[0], acc);
            acc = fmaf(q[l].y, s2[1], acc);
            acc = fmaf(q[l].z, s2[2], acc);
            acc = fmaf(q[l].w, s2[3], acc);
            t2[l] = acc;
        }
    }
    block_sum_f<MAXPP + 1>(t2);

    // R_{k+1} = J~perp(A_{k+1} + E_{k+1} - I); Y_{k+1} = Y_k + mu R_{k+1}.
    float r2[1] = {0.f};
    for (int e = tid; e < n4; e += NT) {
        const float4 a = A[e], ev = E[e], iv = I[e];
        float4 yv = Y[e];
        float s[4] = {a.x + ev.x - iv.x, a.y + ev.y - iv.y, a.z + ev.z - iv.z, a.w + ev.w - iv.w};
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) {
            const float4 q = reinterpret_cast<const float4*>(Qp + l * np)[e];
            s[0] = fmaf(-q.x, t2[l], s[0]);
            s[1] = fmaf(-q.y, t2[l], s[1]);
            s[2] = fmaf(-q.z, t2[l], s[2]);
            s[3] = fmaf(-q.w, t2[l], s[3]);
        }
        R[e] = make_float4(s[0], s[1], s[2], s[3]);
        yv.x = fmaf(muf, s[0], yv.x);
        yv.y = fmaf(muf, s[1], yv.y);
        yv.z = fmaf(muf, s[2], yv.z);
        yv.w = fmaf(muf, s[3], yv.w);
        Y[e] = yv;
        r2[0] = fmaf(s[0], s[0], r2[0]);
        r2[0] = fmaf(s[1], s[1], r2[0]);
        r2[0] = fmaf(s[2], s[2], r2[0]);
        r2[0] = fmaf(s[3], s[3], r2[0]);
    }
    block_sum_f<1>(r2);

    if (tid == 0) finish_inner_iteration(st, prm, (double)r2[0], (double)t2[MAXPP]);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Steps 3 and 4: Delta tau and the transform update
// ---------------------------------------------------------------------------

// Outer stop from ||Delta tau||^2 (one thread).
__device__ void finish_outer_iteration(PatchState* st, const SolverParams& prm, double nrm2, bool finite, double f) {
    st->dtau_norm = sqrt(nrm2);
    st->outer += 1;
    int stop = 0;
    if (!finite) {
        st->status = -5;
        stop = 1;
    }
    if (!prm.fixed_iters && st->dtau_norm < prm.eps_outer) stop = 1;
    // the objective no longer changes (from the second outer iteration of a level on)
    if (!prm.fixed_iters && prm.eps_obj > 0.0 && st->outer > 1 && fabs(f - st->f_prev) < prm.eps_obj * st->f_prev)
        stop = 1;
    st->f_prev = f;
    if (st->outer >= prm.max_outer) stop = 1;
    st->done_outer = stop;
}

__device__ void dev_dtau(const PatchDesc& d, PatchState* st, const SolverParams& prm) {
    const int tid = threadIdx.x;
    const int pp = d.pp, p = d.model;
    const size_t np = (size_t)d.nc * d.ldg;
    const float* A = d.ws + PL_A * np;
    const float* E = d.ws + PL_E * np;
    const float* I = d.ws + PL_I * np;
    const float* Qp = d.ws + PL_Q * np;
    // t = Qb^T (A + E - I); t[MAXPP] = ||E||_1 for the objective
    double t[MAXPP + 1];
#pragma unroll
    for (int l = 0; l <= MAXPP; ++l) t[l] = 0.0;
    for (size_t e = tid; e < np; e += NT) {
        const float s = A[e] + E[e] - I[e];
        #pragma unroll
        for (int l = 0; l < MAXPP; ++l) if (l < pp) t[l] += (double)Qp[l * np + e] * (double)s;
        t[MAXPP] += fabs((double)E[e]);
    }
    block_sum_d<MAXPP + 1>(t);
    if (tid == 0) {
        // y = R^{-1} t (back substitution), Delta tau = N_Q y.
        double y[MAXPP];
        for (int l = pp - 1; l >= 0; --l) {
            double s = t[l];
            for (int k = l + 1; k < pp; ++k) s -= st->R[l * MAXPP + k] * y[k];
            y[l] = s / st->R[l * MAXPP + l];
        }
        double nrm2 = 0.0;
        bool finite = true;
        #pragma unroll
        for (int k = 0; k < MAXP; ++k) if (k < p) {
            double dk = 0.0;
            #pragma unroll
            for (int l = 0; l < MAXPP; ++l) if (l < pp) dk += st->NQ[k * MAXPP + l] * y[l];
            st->tau[k] += dk;
            nrm2 += dk * dk;
            finite = finite && isfinite(st->tau[k]);
        }
        finish_outer_iteration(st, prm, nrm2, finite, st->nuc + d.lam * t[MAXPP]);
    }
    __syncthreads();
}

// Outputs in row-major m x n and the objective ||A||_* + lam ||E||_1.
__device__ void dev_finalize(const PatchDesc& d, PatchState* st) {
    const int tid = threadIdx.x;
    const size_t np = (size_t)d.nc * d.ldg;
    const float* A = d.ws + PL_A * np;
    const float* E = d.ws + PL_E * np;
    double l1[1] = {0.0};
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / d.ldg), col = (int)(e - (size_t)row * d.ldg);
        if (col >= d.nr) continue;
        int i, j;
        xlayout_to_ij(d, row, col, i, j);
        const float ev = E[e];
        l1[0] += fabs((double)ev);
        if (d.A_out) d.A_out[(size_t)i * d.n + j] = A[e];
        if (d.E_out) d.E_out[(size_t)i * d.n + j] = ev;
    }
    block_sum_d<1>(l1);
    if (tid == 0) {
        st->l1 = l1[0];
        st->objective = st->nuc + d.lam * l1[0];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

extern __shared__ float4 tilt_dyn_lds[];

// The kernels read the scaled coordinates of the level being solved from
// the state (the host sets them for the first level; level transitions
// move them on the device).
__device__ inline PatchDesc desc_at_level(const PatchDesc* dp, const PatchState* st) {
    PatchDesc d = *dp;
    d.cx = st->geo[0];
    d.cy = st->geo[1];
    d.s = st->geo[2];
    return d;
}

__device__ void solve_patch(const PatchDesc& d, PatchState* st, const SolverParams& prm, float* lds) {
    __shared__ int sh_flag;
    for (;;) {
        dev_setup(d, st, prm, lds);
        if (threadIdx.x == 0) sh_flag = st->status < 0;
        __syncthreads();
        if (sh_flag) break;
        for (;;) {
            dev_svt(d, st, prm, lds);
            dev_update(d, st, prm);
            if (threadIdx.x == 0) sh_flag = st->done_inner;
            __syncthreads();
            if (sh_flag) break;
        }
        if (threadIdx.x == 0) sh_flag = st->status < 0;
        __syncthreads();
        if (sh_flag) break;
        dev_dtau(d, st, prm);
        if (threadIdx.x == 0) sh_flag = st->done_outer;
        __syncthreads();
        if (sh_flag) break;
    }
    dev_finalize(d, st);
}

// ---------------------------------------------------------------------------
// Coarse-to-fine pyramid.  Level l+1 is level l blurred with the separable
// binomial kernel [1 4 6 4 1]/16 (indices clamped at the borders) at every
// second pixel; the window halves with it and transforms move between
// levels by conjugation with diag(1/2, 1/2, 1).  Each level is solved cold
// from the transform the coarser level returned.
// ---------------------------------------------------------------------------

__device__ void blur_decimate(const float* src, int Hs, int Ws, long long ss, float* dst, int Hd, int Wd) {
    const float w[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
    for (int e = threadIdx.x; e < Hd * Wd; e += NT) {
        const int i = e / Wd, j = e - i * Wd;
        int cols[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) cols[b] = min(max(2 * j + b - 2, 0), Ws - 1);
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const float* row = src + (long long)min(max(2 * i + a - 2, 0), Hs - 1) * ss;
            float r = 0.f;
#pragma unroll
            for (int b = 0; b < 5; ++b) r = fmaf(w[b], row[cols[b]], r);
            acc = fmaf(w[a], r, acc);
        }
        dst[e] = acc;
    }
}

// Build levels 1..levels-1 (dl[l].image points into the request workspace).
__device__ void build_pyramid(const PatchDesc* dl, int levels) {
    for (int l = 1; l < levels; ++l) {
        blur_decimate(dl[l - 1].image, dl[l - 1].H, dl[l - 1].W, dl[l - 1].stride, const_cast<float*>(dl[l].image),
                      dl[l].H, dl[l].W);
        __syncthreads();
    }
}

// Move the state from the solved coarser level to level `d` (thread 0).
__device__ void level_transition(const PatchDesc& d, PatchState* st) {
    if (threadIdx.x == 0) {
        double Hn[9] = {st->tau[0], st->tau[1], st->tau[2], st->tau[3], st->tau[4], st->tau[5], 0.0, 0.0, 1.0};
        if (d.model == 8) {
            Hn[6] = st->tau[6];
            Hn[7] = st->tau[7];
        }
        double H[9], geo[3], Hf[9];
        denormalise_h(Hn, st->geo, H);
        to_finer_h(H);
        if (normalise_h(H, d.m, d.n, geo, Hf)) {
            st->tau[0] = Hf[0];
            st->tau[1] = Hf[1];
            st->tau[2] = Hf[2];
            st->tau[3] = Hf[3];
            st->tau[4] = Hf[4];
            st->tau[5] = Hf[5];
            st->tau[6] = d.model == 8 ? Hf[6] : 0.0;
            st->tau[7] = d.model == 8 ? Hf[7] : 0.0;
            st->geo[0] = geo[0];
            st->geo[1] = geo[1];
            st->geo[2] = geo[2];
        } else {
            st->status = -5;
        }
        st->outer = 0;
        st->inner = 0;
        st->done_inner = 0;
        st->done_outer = 0;
        st->warm_ok = 0;
        st->warm_count = 0;
        st->svdws_ok = 0;
    }
    __syncthreads();
}

// One request: build its pyramid, then solve from the coarsest level to
// level 0.  dl[0..levels-1] are the level descriptors.
__device__ void solve_request(const PatchDesc* dl, int levels, PatchState* st, const SolverParams& prm, float* lds) {
    __shared__ int sh_fail;
    if (threadIdx.x == 0) st->t_begin = (long long)wall_clock64();
    if (levels > 1) build_pyramid(dl, levels);
    for (int l = levels - 1; l >= 0; --l) {
        if (l < levels - 1) {
            if (threadIdx.x == 0) sh_fail = st->status < 0;
            __syncthreads();
            if (sh_fail) break;
            level_transition(dl[l], st);
            if (threadIdx.x == 0) sh_fail = st->status < 0;
            __syncthreads();
            if (sh_fail) break;
        }
        const PatchDesc d = desc_at_level(dl + l, st);
        solve_patch(d, st, prm, lds);
    }
    if (threadIdx.x == 0) st->t_end = (long long)wall_clock64();
}

// Persistent solver: each workgroup takes the next request from the queue
// (in the order given by `order`, longest predicted solve first) until the
// queue is exhausted, then helps the leaders of windows beyond LDS with
// their Jacobi rounds until every request is finished.  Request i has its
// level descriptors at descs[i * levels ...].
__global__ void __launch_bounds__(NT) k_fused(const PatchDesc* __restrict__ descs, PatchState* states,
                                               SolverParams prm, int count, int levels,
                                               const int* __restrict__ order, FusedCtl* fc, int help) {
    __shared__ int sh_idx;
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    for (;;) {
        if (threadIdx.x == 0) {
            const int q = atomicAdd(&fc->queue, 1);
            sh_idx = q < count ? order[q] : count;
        }
        __syncthreads();
        const int idx = sh_idx;
        __syncthreads();
        if (idx >= count) break;
        const PatchDesc* dl = descs + (size_t)idx * levels;
        solve_request(dl, levels, states + idx, prm, lds);
        if (threadIdx.x == 0) {
            GangCtl* c = dl[0].gang;
            if (c && c->slot >= 0)
                __hip_atomic_store(&fc->slots[c->slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&fc->remaining, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (!help) return;  // no window of this launch is tiled
    __shared__ GangCtl sh_job;
    __shared__ unsigned sh_id;
    __shared__ int sh_pair;
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&fc->idle, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const int g = help_find(fc, &sh_job, &sh_id, &sh_pair);
        if (g >= 0) {
            help_run(fc, g, &sh_job, sh_id, sh_pair, lds);
            continue;
        }
        if (threadIdx.x == 0) sh_idx = poll_load(&fc->remaining);
        __syncthreads();
        const int left = sh_idx;
        __syncthreads();
        if (left <= 0) break;
        __builtin_amdgcn_s_sleep(32);
    }
}

// ---------------------------------------------------------------------------
// Serving kernel (continuous batching).  Each workgroup polls the ring for
// published requests, claims the next one with a compare-and-swap on the
// device counter `head`, copies its descriptors and initial state to device
// memory, solves it and writes the final state back to the slot before
// raising the slot's `done`.  The workgroups leave together: `ctr` holds
// the claim counter, the number of requests being solved, a closing latch
// and the device wall-clock time of the last finished request.  A
// workgroup that finds nothing to claim sets the latch when no request is
// in flight and neither it nor any other workgroup has worked for
// `idle_ticks`; every workgroup exits once the latch or the host's `stop`
// is set, so every wave reaches an exit and none leaves while others still
// solve.  The host clears the latch before each launch and relaunches the
// kernel when requests are outstanding and it has ended.
//
// Workspaces are recycled between requests that may run on different
// XCDs: an agent-scope fence at the start of a request drops stale cached
// lines, and a system-scope fence before `done` makes the results (state,
// A, E) visible to the host.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(NT) k_serve(ServeCtl* ctl, ServeSlot* slots, PatchDesc* ddesc, PatchState* dstates,
                                               unsigned long long* ctr, int ring, long long idle_ticks, FusedCtl* fc,
                                               int help) {
    __shared__ long long sh_seq;
    __shared__ GangCtl sh_job;
    __shared__ unsigned sh_id;
    __shared__ int sh_pair;
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const int tid = threadIdx.x;
    long long idle_since = (long long)wall_clock64();
    // counted in fc->idle while it has no request (help = 1): leaders of
    // tiled requests publish their rounds while idle workgroups exist
    bool counted_idle = false;
    for (;;) {
        if (tid == 0) {
            unsigned long long* head = ctr;
            unsigned long long* busy = ctr + 1;
            unsigned long long* closing = ctr + 2;
            unsigned long long* last_done = ctr + 3;
            long long seq = -1;
            // polls are relaxed (an acquire would invalidate the L2 lines the
            // solving workgroups of this XCD work from); a claimed request's
            // slot is acquired below
            const bool closed = __hip_atomic_load(closing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull;
            if (!closed) {
                const unsigned long long tail =
                    __hip_atomic_load(&ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                unsigned long long h = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < tail) {
                    // counted as busy before the claim, so that no workgroup
                    // closes the kernel between this claim and its solve
                    __hip_atomic_fetch_add(busy, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                    while (h < tail) {
                        if (__hip_atomic_compare_exchange_strong(head, &h, h + 1, __ATOMIC_ACQ_REL,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            seq = (long long)h;
                            break;
                        }
                    }
                    if (seq < 0) __hip_atomic_fetch_add(busy, ~0ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                    // pairs with the host's release of `tail`: the slot's
                    // contents are visible from here on
                    if (seq >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                }
            }
            if (seq < 0) {
                const int stop = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (stop || closed) {
                    seq = -2;
                } else {
                    const long long now = (long long)wall_clock64();
                    const long long last =
                        (long long)__hip_atomic_load(last_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const long long since = last > idle_since ? last : idle_since;
                    if (now - since > idle_ticks &&
                        __hip_atomic_load(busy, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0ull) {
                        __hip_atomic_store(closing, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        seq = -2;
                    }
                }
            }
            sh_seq = seq;
        }
        __syncthreads();
        const long long seq = sh_seq;
        __syncthreads();
        if (seq == -2) {
            if (counted_idle && tid == 0) __hip_atomic_fetch_add(&fc->idle, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        if (seq < 0) {
            if (help) {
                // between two polls of the ring (~30 us apart), help the
                // leaders of tiled requests (helpers as in the fused kernel)
                if (!counted_idle && tid == 0)
                    __hip_atomic_fetch_add(&fc->idle, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                counted_idle = true;
                for (int k = 0; k < 16; ++k) {
                    const int g = help_find(fc, &sh_job, &sh_id, &sh_pair);
                    if (g >= 0) {
                        help_run(fc, g, &sh_job, sh_id, sh_pair, lds);
                        k = 0;
                        continue;
                    }
                    __builtin_amdgcn_s_sleep(64);
                }
            } else {
                if (tid == 0) {
                    for (int k = 0; k < 8; ++k) __builtin_amdgcn_s_sleep(127);
                }
                __syncthreads();
            }
            continue;
        }
        if (counted_idle) {
            if (tid == 0) __hip_atomic_fetch_add(&fc->idle, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            counted_idle = false;
        }
        const int slot = (int)(seq % ring);
        ServeSlot* sl = slots + slot;
        PatchDesc* dl = ddesc + (size_t)slot * MAX_LEVELS;
        PatchState* st = dstates + slot;
        __threadfence();
        const int levels = sl->levels;
        {
            const unsigned long long* src = reinterpret_cast<const unsigned long long*>(sl->d);
            unsigned long long* dst = reinterpret_cast<unsigned long long*>(dl);
            const int nw = (int)(sizeof(PatchDesc) * MAX_LEVELS / 8);
            for (int k = tid; k < nw; k += NT) dst[k] = src[k];
            const unsigned long long* s0 = reinterpret_cast<const unsigned long long*>(&sl->init);
            unsigned long long* s1 = reinterpret_cast<unsigned long long*>(st);
            for (int k = tid; k < (int)(sizeof(PatchState) / 8); k += NT) s1[k] = s0[k];
        }
        __shared__ SolverParams sh_prm;
        if (tid == 0) sh_prm = sl->prm;
        __syncthreads();
        const SolverParams prm = sh_prm;
        solve_request(dl, levels, st, prm, lds);
        if (tid == 0) {
            // a tiled request's leader leaves the helpers' registry; the
            // slot's control block is reused by the next request in it
            // (its round ids and counters run on, so no stale claim of
            // this request can match a round of the next)
            GangCtl* c = dl[0].gang;
            if (c && c->slot >= 0) {
                __hip_atomic_store(&fc->slots[c->slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                c->slot = -1;
            }
        }
        __syncthreads();
        {
            const unsigned long long* s0 = reinterpret_cast<const unsigned long long*>(st);
            unsigned long long* s1 = reinterpret_cast<unsigned long long*>(&sl->result);
            for (int k = tid; k < (int)(sizeof(PatchState) / 8); k += NT) s1[k] = s0[k];
        }
        __threadfence_system();
        __syncthreads();
        idle_since = (long long)wall_clock64();
        if (tid == 0) {
            __hip_atomic_store(&sl->done, (unsigned long long)seq + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_fetch_max(ctr + 3, (unsigned long long)idle_since, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(ctr + 1, ~0ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Plain (step-by-step) kernels: one workgroup, one patch; `d` and `st`
// point at the level descriptor and the patch state.
__global__ void __launch_bounds__(NT) k_setup(const PatchDesc* dp, PatchState* st, SolverParams prm) {
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const PatchDesc d = desc_at_level(dp, st);
    dev_setup(d, st, prm, lds);
}

// The inner-iteration kernels do nothing once the inner loop has stopped,
// so a captured sequence of several iterations can be replayed past the
// stopping point without changing the result.
__global__ void __launch_bounds__(NT) k_svt(const PatchDesc* dp, PatchState* st, SolverParams prm) {
    if (st->done_inner) return;
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const PatchDesc d = desc_at_level(dp, st);
    dev_svt(d, st, prm, lds);
}

__global__ void __launch_bounds__(NT) k_update(const PatchDesc* dp, PatchState* st, SolverParams prm) {
    if (st->done_inner) return;
    const PatchDesc d = desc_at_level(dp, st);
    dev_update(d, st, prm);
}

__global__ void __launch_bounds__(NT) k_dtau(const PatchDesc* dp, PatchState* st, SolverParams prm) {
    const PatchDesc d = desc_at_level(dp, st);
    dev_dtau(d, st, prm);
}

__global__ void __launch_bounds__(NT) k_finalize(const PatchDesc* dp, PatchState* st, int last) {
    const PatchDesc d = desc_at_level(dp, st);
    dev_finalize(d, st);
    if (threadIdx.x == 0 && last) st->t_end = (long long)wall_clock64();
}

// Inner loop alone for `count` problems of one shape (one workgroup each).
__global__ void __launch_bounds__(NT) k_inner(const PatchDesc* descs, PatchState* states, SolverParams prm,
                                               const float* Iall, const float* Jall) {
    __shared__ int sh_flag;
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const int idx = blockIdx.x;
    PatchState* st = states + idx;
    const PatchDesc d = desc_at_level(descs + idx, st);
    const size_t mn = (size_t)d.m * d.n;
    if (threadIdx.x == 0) st->t_begin = (long long)wall_clock64();
    dev_setup_given(d, st, prm, lds, Iall + idx * mn, Jall + (size_t)idx * d.pp * mn);
    if (threadIdx.x == 0) sh_flag = st->status < 0;
    __syncthreads();
    if (!sh_flag) {
        for (;;) {
            dev_svt(d, st, prm, lds);
            dev_update(d, st, prm);
            if (threadIdx.x == 0) sh_flag = st->done_inner;
            __syncthreads();
            if (sh_flag) break;
        }
    }
    dev_finalize(d, st);
    if (threadIdx.x == 0) st->t_end = (long long)wall_clock64();
}

// ---------------------------------------------------------------------------
// Wide SVT for a few large problems of the inner-loop entry.  The
// super-block pairs of one round of the tiled Jacobi touch disjoint rows, so
// each runs on its own workgroup (one launch per round); the host ends a
// sweep by reading the per-problem rotation flags.  Every pair of a round
// sees the same rows in whatever order the workgroups run, so the result is
// the one the single-workgroup tiled Jacobi gives with the same super-blocks.
// ---------------------------------------------------------------------------

// Set-up of problem blockIdx.x (as the first part of k_inner).
__global__ void __launch_bounds__(NT) k_wide_setup(const PatchDesc* descs, PatchState* states, SolverParams prm,
                                                    const float* Iall, const float* Jall) {
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const int idx = blockIdx.x;
    PatchState* st = states + idx;
    const PatchDesc d = desc_at_level(descs + idx, st);
    const size_t mn = (size_t)d.m * d.n;
    if (threadIdx.x == 0) st->t_begin = (long long)wall_clock64();
    dev_setup_given(d, st, prm, lds, Iall + idx * mn, Jall + (size_t)idx * d.pp * mn);
}

// Stage the Jacobi rows of problem active[blockIdx.x] into its working
// plane (rows beyond nc zero): M_k, formed first, when form_m; else the
// normalised image I (whose largest singular value sets mu_0).  Clears the
// problem's rotation flag.
__global__ void __launch_bounds__(NT) k_wide_stage(const PatchDesc* descs, PatchState* states, const int* active,
                                                    int form_m, int* flags) {
    const int idx = active[blockIdx.x];
    PatchState* st = states + idx;
    const PatchDesc d = desc_at_level(descs + idx, st);
    const size_t np = (size_t)d.nc * d.ldg;
    if (form_m) {
        svt_form_m(d, st, nullptr);
        __syncthreads();
    }
    const float* X = d.ws + (form_m ? PL_M : PL_I) * np;
    float* Bg = d.ws + NPLANES * np;
    const int nr4 = d.ldg >> 2;
    for (int e = threadIdx.x; e < d.ncp * nr4; e += NT) {
        const int row = e / nr4, c = e - row * nr4;
        float4 v = f4(0.f);
        if (row < d.nc) v = reinterpret_cast<const float4*>(X + (size_t)row * d.ldg)[c];
        reinterpret_cast<float4*>(Bg + (size_t)row * d.ldg)[c] = v;
    }
    if (threadIdx.x == 0) flags[idx] = 0;
}

// One super-block pair of round r of the circle ordering over super-blocks:
// workgroup g takes problem active[g / pairs], pair g % pairs.
__global__ void __launch_bounds__(NT) k_wide_round(const PatchDesc* descs, PatchState* states, const int* active,
                                                    int pairs, int r, float tol_max, double eps2, int* flags) {
    float* mini = reinterpret_cast<float*>(tilt_dyn_lds);
    const int slot = blockIdx.x / pairs, k = blockIdx.x - slot * pairs;
    const int idx = active[slot];
    PatchState* st = states + idx;
    const PatchDesc& d = descs[idx];
    // inner-loop SVTs (eps2 > 0) follow mu as in dev_svt; the decomposition
    // of I for mu_0 uses tol_max
    const float tol = eps2 > 0.0 ? svt_tolerance(tol_max, eps2, st->mu, d.nr) : svt_tolerance_cap(tol_max, d.nr);
    const int sb = d.sb;
    int I, J;
    superblock_pair(d.nsb, r, k, I, J);
    float* Bg = d.ws + NPLANES * (size_t)d.nc * d.ldg;
    load_block(Bg, I * sb, sb, d.ldg, mini, 0, d.ld);
    load_block(Bg, J * sb, sb, d.ldg, mini, sb, d.ld);
    clear_lds_padding(mini, 2 * sb, d.ldg, d.ld);
    __syncthreads();
    JacobiStats js{0, 0, 0};
    const int rot = jacobi_pair_dispatch(d.svt_cfg, mini, sb, d.ld, tol, r == 0, js);
    if (rot) {
        store_block(Bg, I * sb, sb, d.ldg, mini, 0, d.ld);
        store_block(Bg, J * sb, sb, d.ldg, mini, sb, d.ld);
    }
    if (threadIdx.x == 0) {
        if (rot) atomicOr(flags + idx, 1);
        atomicAdd(reinterpret_cast<unsigned long long*>(&st->pairs), (unsigned long long)js.pairs);
        atomicAdd(reinterpret_cast<unsigned long long*>(&st->rotations), (unsigned long long)js.rotations);
    }
}

// After the sweeps of problem active[blockIdx.x]: row norms of the working
// plane, then (mode 0) shrinkage and reconstruction of A, or (mode 1)
// mu_0 = 1.25 / sigma_max(I) unless mu_0 is given.
__global__ void __launch_bounds__(NT) k_wide_finish(const PatchDesc* descs, PatchState* states, const int* active,
                                                     SolverParams prm, const int* sweeps, int mode) {
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const int idx = active[blockIdx.x];
    PatchState* st = states + idx;
    const PatchDesc d = desc_at_level(descs + idx, st);
    const SvtLds L = carve_for(d, lds);
    const float* Bg = d.ws + NPLANES * (size_t)d.nc * d.ldg;
    row_norms_global(Bg, d.nc, d.ldg, L.s2);
    if (mode == 0) {
        const JacobiStats js{sweeps[idx], 0, 0};
        svt_finish(d, st, L, js);
        return;
    }
    if (threadIdx.x == 0) {
        float mx = 0.f;
        for (int j = 0; j < d.nc; ++j) mx = fmaxf(mx, L.s2[j]);
        const double mu0 = prm.mu0 > 0.0 ? prm.mu0 : 1.25 / (double)sqrtf(mx);
        st->mu = mu0;
        st->svt_calls += 1;
        st->sweeps += sweeps[idx];
        if (!isfinite(mu0)) {
            st->status = -5;
            st->done_outer = 1;
            st->done_inner = 1;
        }
    }
}

__global__ void __launch_bounds__(NT) k_wide_update(const PatchDesc* descs, PatchState* states, const int* active,
                                                     SolverParams prm) {
    const int idx = active[blockIdx.x];
    PatchState* st = states + idx;
    const PatchDesc d = desc_at_level(descs + idx, st);
    dev_update(d, st, prm);
}

__global__ void __launch_bounds__(NT) k_wide_end(const PatchDesc* descs, PatchState* states) {
    const int idx = blockIdx.x;
    PatchState* st = states + idx;
    const PatchDesc d = desc_at_level(descs + idx, st);
    dev_finalize(d, st);
    if (threadIdx.x == 0) st->t_end = (long long)wall_clock64();
}

__global__ void __launch_bounds__(NT) k_mark_end(PatchState* st) {
    if (threadIdx.x == 0) st->t_end = (long long)wall_clock64();
}

// Plain path, pyramid: build the level images of one request (dl[0..levels-1]).
__global__ void __launch_bounds__(NT) k_pyramid_build(const PatchDesc* dl, int levels) {
    build_pyramid(dl, levels);
}

// Plain path: start a level (transition from the coarser level's result;
// for the first level only the start time is recorded).
__global__ void __launch_bounds__(NT) k_level_begin(const PatchDesc* dp, PatchState* st, int first) {
    if (first) {
        if (threadIdx.x == 0) st->t_begin = (long long)wall_clock64();
    } else {
        level_transition(*dp, st);
    }
}

// Component kernel: pyramid levels 1..levels-1 of one image, stored one
// after the other (level l is ceil(H/2^l) x ceil(W/2^l), row-major).
__global__ void __launch_bounds__(NT) k_pyramid_jobs(const float* image, int H, int W, long long stride, float* out,
                                                     int levels) {
    const float* src = image;
    int Hs = H, Ws = W;
    long long ss = stride;
    float* dst = out;
    for (int l = 1; l < levels; ++l) {
        const int Hd = (Hs + 1) / 2, Wd = (Ws + 1) / 2;
        blur_decimate(src, Hs, Ws, ss, dst, Hd, Wd);
        __syncthreads();
        src = dst;
        Hs = Hd;
        Ws = Wd;
        ss = Wd;
        dst += (size_t)Hd * Wd;
    }
}

// Component kernel: normalised warp and Jacobian (Alg. 1 Step 1); one
// workgroup per patch, outputs in row-major m x n (I) and p planes of m x n
// (J, parameter-major).
// Component kernels: Step 1 (warp, Jacobian of the normalised warp) for a
// batch of windows, each window split over STEP1_SLICES workgroups so that
// every SIMD holds several waves.  The first kernel writes each slice's
// partial sums (||I||^2 and I^T J_raw); the second combines the partials of
// its window in a fixed order, samples its slice again and writes I and J.

__device__ inline void step1_slice(const PatchDesc& d, int slice, size_t* e0, size_t* e1) {
    const size_t mn = (size_t)d.m * d.n;
    const size_t per = (mn + STEP1_SLICES - 1) / STEP1_SLICES;
    *e0 = min(mn, per * (size_t)slice);
    *e1 = min(mn, *e0 + per);
}

__global__ void __launch_bounds__(NT) k_step1_sums(const PatchDesc* descs, const PatchState* states,
                                                   double* partial) {
    const int w = blockIdx.x / STEP1_SLICES, slice = blockIdx.x - w * STEP1_SLICES;
    const PatchDesc d = descs[w];
    const int p = d.model;
    double h[8];
    tau_to_h(states + w, p, h);
    size_t e0, e1;
    step1_slice(d, slice, &e0, &e1);
    double acc[1 + MAXP];
#pragma unroll
    for (int k = 0; k <= MAXP; ++k) acc[k] = 0.0;
    for (size_t e = e0 + threadIdx.x; e < e1; e += NT) {
        const int i = (int)(e / d.n), j = (int)(e - (size_t)i * d.n);
        float jr[MAXP];
        const float val = warp_pixel(d, h, i, j, jr);
        acc[0] += (double)val * val;
        #pragma unroll
        for (int k = 0; k < MAXP; ++k) if (k < p) acc[1 + k] += (double)val * (double)jr[k];
    }
    block_sum_d<1 + MAXP>(acc);
    if (threadIdx.x <= MAXP) partial[(size_t)blockIdx.x * (1 + MAXP) + threadIdx.x] = acc[threadIdx.x];
}

__global__ void __launch_bounds__(NT) k_step1_out(const PatchDesc* descs, const PatchState* states,
                                                  const double* partial, float* I_out, float* J_out) {
    const int w = blockIdx.x / STEP1_SLICES, slice = blockIdx.x - w * STEP1_SLICES;
    const PatchDesc d = descs[w];
    const int p = d.model;
    const size_t mn = (size_t)d.m * d.n;
    float* Io = I_out + (size_t)w * mn;
    float* Jo = J_out + (size_t)w * mn * p;
    double h[8];
    tau_to_h(states + w, p, h);
    double acc[1 + MAXP];
#pragma unroll
    for (int k = 0; k <= MAXP; ++k) {
        double s = 0.0;
        for (int q = 0; q < STEP1_SLICES; ++q) s += partial[((size_t)w * STEP1_SLICES + q) * (1 + MAXP) + k];
        acc[k] = s;
    }
    const double inv_n = 1.0 / sqrt(acc[0]);
    const double inv_n3 = inv_n * inv_n * inv_n;
    size_t e0, e1;
    step1_slice(d, slice, &e0, &e1);
    for (size_t e = e0 + threadIdx.x; e < e1; e += NT) {
        const int i = (int)(e / d.n), j = (int)(e - (size_t)i * d.n);
        float jr[MAXP];
        const double val = warp_pixel(d, h, i, j, jr);
        Io[e] = (float)(val * inv_n);
        #pragma unroll
        for (int k = 0; k < MAXP; ++k) if (k < p) Jo[k * mn + e] = (float)((double)jr[k] * inv_n - val * acc[1 + k] * inv_n3);
    }
}

// Component kernel: batched singular value shrinkage of independent
// matrices (the A-update of Eq. A_1 on its own).
__global__ void __launch_bounds__(NT) k_svt_jobs(const SvtJob* jobs, SvtShape shape, float tol, int max_sweeps,
                                                 long long* counters, float* scratch) {
    const SvtJob jb = jobs[blockIdx.x];
    float* lds = reinterpret_cast<float*>(tilt_dyn_lds);
    const int tid = threadIdx.x;
    const int m = jb.m, n = jb.n;
    const bool colmajor = m >= n;
    const int nc = colmajor ? n : m, nr = colmajor ? m : n;
    const int ldg = (nr + 3) & ~3;
    const int nr4 = ldg >> 2;
    const size_t np = (size_t)nc * ldg;
    const size_t per_job = 2 * np + (shape.sb > 0 ? (size_t)shape.ncp * ldg : 0);
    float* X = scratch + (size_t)blockIdx.x * per_job;
    float* AX = X + np;
    float* Bg = AX + np;
    PatchDesc d{};
    d.nc = nc;
    d.nr = nr;
    d.ldg = ldg;
    d.ld = shape.ld;
    d.svt_cfg = shape.cfg;
    d.tb = shape.tb;
    d.sb = shape.sb;
    d.nsb = shape.nsb;
    d.ncp = shape.ncp;
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        float v = 0.f;
        if (col < nr) v = colmajor ? jb.M[(size_t)col * n + row] : jb.M[(size_t)row * n + col];
        X[e] = v;
        AX[e] = 0.f;
    }
    __syncthreads();
    const SvtLds L = carve_for(d, lds);
    JacobiStats js{0, 0, 0};
    svd_rows(d, X, Bg, L, tol, max_sweeps, js);
    int k;
    double nuc;
    shrink_weights(L.s2, nc, jb.eps, L.w, L.act, &k, &nuc);
    if (jb.sigma) {
        for (int j = tid; j < nc; j += NT) jb.sigma[j] = sqrtf(L.s2[j]);
    }
    if (d.sb > 0)
        reconstruct(Bg, ldg, X, AX, nc, nr4, ldg, L.w, L.act, k, d.tb, L.xblk, L.cwt, false);
    else
        reconstruct(L.B, d.ld, X, AX, nc, nr4, ldg, L.w, L.act, k, d.tb, L.xblk, L.cwt, false);
    __syncthreads();
    for (size_t e = tid; e < np; e += NT) {
        const int row = (int)(e / ldg), col = (int)(e - (size_t)row * ldg);
        if (col >= nr) continue;
        if (colmajor)
            jb.A[(size_t)col * n + row] = AX[e];
        else
            jb.A[(size_t)row * n + col] = AX[e];
    }
    if (tid == 0 && counters) {
        long long* c = counters + 4 * blockIdx.x;
        c[0] = js.sweeps;
        c[1] = js.pairs;
        c[2] = js.rotations;
        c[3] = k;
    }
}

#include "tilt_rasl.inc"

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// Allow `lds` bytes of dynamic LDS; fails (hipErrorInvalidValue) when the
// kernel's static LDS plus `lds` exceeds the 160 KiB of a CU.
static hipError_t set_lds(const void* fn, size_t lds) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes + lds > (size_t)LDS_LIMIT) return hipErrorInvalidValue;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_fused(const PatchDesc* d, PatchState* st, const SolverParams& prm, int count, int levels,
                        const int* order, FusedCtl* fc, int help, int grid, size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_fused, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fused, dim3(grid), dim3(NT), lds, s, d, st, prm, count, levels, order, fc, help);
    return hipGetLastError();
}

hipError_t launch_serve(ServeCtl* ctl, ServeSlot* slots, PatchDesc* ddesc, PatchState* dstates,
                        unsigned long long* ctr, int ring, long long idle_ticks, FusedCtl* fc, int help, int grid,
                        size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_serve, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_serve, dim3(grid), dim3(NT), lds, s, ctl, slots, ddesc, dstates, ctr, ring, idle_ticks, fc,
                       help);
    return hipGetLastError();
}

hipError_t launch_setup(const PatchDesc* d, PatchState* st, const SolverParams& prm, size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_setup, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(NT), lds, s, d, st, prm);
    return hipGetLastError();
}

hipError_t launch_svt(const PatchDesc* d, PatchState* st, const SolverParams& prm, size_t lds, hipStream_t s,
                      bool configure) {
    if (configure) {
        hipError_t e = set_lds((const void*)k_svt, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_svt, dim3(1), dim3(NT), lds, s, d, st, prm);
    return hipGetLastError();
}

hipError_t launch_update(const PatchDesc* d, PatchState* st, const SolverParams& prm, hipStream_t s) {
    hipLaunchKernelGGL(k_update, dim3(1), dim3(NT), 0, s, d, st, prm);
    return hipGetLastError();
}

hipError_t launch_dtau(const PatchDesc* d, PatchState* st, const SolverParams& prm, hipStream_t s) {
    hipLaunchKernelGGL(k_dtau, dim3(1), dim3(NT), 0, s, d, st, prm);
    return hipGetLastError();
}

hipError_t launch_finalize(const PatchDesc* d, PatchState* st, int last, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(NT), 0, s, d, st, last);
    return hipGetLastError();
}

hipError_t launch_inner(const PatchDesc* d, PatchState* st, const SolverParams& prm, const float* I, const float* J,
                        int count, size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_inner, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inner, dim3(count), dim3(NT), lds, s, d, st, prm, I, J);
    return hipGetLastError();
}

hipError_t launch_wide_setup(const PatchDesc* d, PatchState* st, const SolverParams& prm, const float* I,
                             const float* J, int count, size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_wide_setup, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wide_setup, dim3(count), dim3(NT), lds, s, d, st, prm, I, J);
    return hipGetLastError();
}

hipError_t launch_wide_stage(const PatchDesc* d, PatchState* st, const int* active, int nactive, int form_m,
                             int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_wide_stage, dim3(nactive), dim3(NT), 0, s, d, st, active, form_m, flags);
    return hipGetLastError();
}

hipError_t launch_wide_round(const PatchDesc* d, PatchState* st, const int* active, int nactive, int pairs, int r,
                             float tol, double eps2, int* flags, size_t lds, bool configure, hipStream_t s) {
    if (configure) {
        hipError_t e = set_lds((const void*)k_wide_round, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_wide_round, dim3(nactive * pairs), dim3(NT), lds, s, d, st, active, pairs, r, tol, eps2,
                       flags);
    return hipGetLastError();
}

hipError_t launch_wide_finish(const PatchDesc* d, PatchState* st, const int* active, int nactive,
                              const SolverParams& prm, const int* sweeps, int mode, size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_wide_finish, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wide_finish, dim3(nactive), dim3(NT), lds, s, d, st, active, prm, sweeps, mode);
    return hipGetLastError();
}

hipError_t launch_wide_update(const PatchDesc* d, PatchState* st, const int* active, int nactive,
                              const SolverParams& prm, hipStream_t s) {
    hipLaunchKernelGGL(k_wide_update, dim3(nactive), dim3(NT), 0, s, d, st, active, prm);
    return hipGetLastError();
}

hipError_t launch_wide_end(const PatchDesc* d, PatchState* st, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_wide_end, dim3(count), dim3(NT), 0, s, d, st);
    return hipGetLastError();
}

hipError_t launch_mark_end(PatchState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_mark_end, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_pyramid_build(const PatchDesc* d, int levels, hipStream_t s) {
    hipLaunchKernelGGL(k_pyramid_build, dim3(1), dim3(NT), 0, s, d, levels);
    return hipGetLastError();
}

hipError_t launch_level_begin(const PatchDesc* d, PatchState* st, int first, hipStream_t s) {
    hipLaunchKernelGGL(k_level_begin, dim3(1), dim3(NT), 0, s, d, st, first);
    return hipGetLastError();
}

hipError_t launch_pyramid_jobs(const float* image, int H, int W, long long stride, float* out, int levels,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_pyramid_jobs, dim3(1), dim3(NT), 0, s, image, H, W, stride, out, levels);
    return hipGetLastError();
}

hipError_t launch_step1(const PatchDesc* d, PatchState* st, int count, double* partial, float* I_out, float* J_out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_step1_sums, dim3(count * STEP1_SLICES), dim3(NT), 0, s, d, st, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_step1_out, dim3(count * STEP1_SLICES), dim3(NT), 0, s, d, st, partial, I_out, J_out);
    return hipGetLastError();
}

hipError_t launch_svt_jobs(const SvtJob* jobs, int count, const SvtShape& shape, float tol, int max_sweeps,
                           long long* counters, float* scratch, size_t lds, hipStream_t s) {
    hipError_t e = set_lds((const void*)k_svt_jobs, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_svt_jobs, dim3(count), dim3(NT), lds, s, jobs, shape, tol, max_sweeps, counters,
                       scratch);
    return hipGetLastError();
}

}  // namespace tilt
