// Internal declarations shared by the HIP kernels and the host interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tilt {

constexpr int NT = 256;          // threads per workgroup, every kernel
constexpr int NWAVE = NT / 64;   // wavefronts per workgroup
constexpr int MAXP = 8;          // transform parameters (projective)
constexpr int MAXPP = 5;         // free parameters after the 3 constraints
constexpr int NPLANES = 7 + MAXP;
constexpr int LDS_LIMIT = 160 * 1024;
constexpr int MAX_LEVELS = 4;    // pyramid levels per request
constexpr int STEP1_SLICES = 4;  // workgroups per window in the batched Step-1 component kernels

// Per-patch device planes, each nc * ldg floats in "X layout": the matrix
// is stored with its shorter side as the outer index, so the vectors the
// one-sided Jacobi orthogonalises (length nr = max(m, n)) are contiguous.
// PL_V holds the accumulated Jacobi rotation of the warm-started SVT
// (nc x nc in the first nc columns); it persists across inner iterations.
enum Plane { PL_I = 0, PL_A = 1, PL_E = 2, PL_Y = 3, PL_R = 4, PL_M = 5, PL_Q = 6, PL_V = 6 + MAXP };

// Jacobi variants: BS rows per block (1 or 2), LPP lanes per block pair
// (4, 8, 16; 32 and 64 for rows longer than 512) and NCH float4 chunks of
// each row held per lane (1..8 for BS = 1, 1..4 for BS = 2: at most 64
// floats of rows per lane); encoded by svt_make_cfg.
constexpr int SVT_MAX_NCH = 8;
constexpr int SVT_MAX_ROWS = 256;  // rows of the Jacobi matrix held in LDS at once
// Tiled SVT (matrices larger than LDS): the rows live in a device plane and
// are processed in pairs of super-blocks of sb rows staged through LDS.
constexpr int SVT_MAX_TILED_ROWS = 1024;  // rows of the working plane (min(m, n) rounded up to whole super-blocks)
constexpr int SVT_MAX_COLS = 2048;       // max(m, n): 64 lanes x 8 chunks x 4 floats

// Helpers for windows whose SVT is tiled through device memory (fused
// kernel only): the window's leader publishes the rounds of its tiled
// Jacobi in its GangCtl while workgroups that ran out of work are idle, and
// those claim super-block pairs of it.  Both blocks live in device memory,
// zeroed (slot = -1) before the launch.
constexpr int HELP_SLOTS = 1024;  // registered leaders at once (power of 2, >= workgroups of a launch)

struct GangCtl;

struct FusedCtl {
    int queue;          // next entry of the order to claim
    int remaining;      // requests not finished yet
    int idle;           // workgroups that have left the queue and help
    int pad0;
    GangCtl* gangs;     // one control block per request
    int pad[26];
    int slots[HELP_SLOTS];  // request index + 1 of leaders that publish rounds, 0 = free
};

struct alignas(128) GangCtl {
    unsigned long long word;  // published round: (id << 32) | (pairs << 16) | pairs claimed
    int done;                 // pairs finished by helpers (only grows)
    int rot;                  // largest round id in which a helper's pair rotated
    float* Bg;                // round: working plane (ncp x ldg Jacobi rows)
    float* Rg;                // round: rotation rows of a warm-started decomposition, or null
    int sb, nsb, ldg, ld, cfg, r;
    float tol;
    int rid;                  // leader: rounds published so far
    int slot;                 // leader: its entry in FusedCtl::slots (-1: none yet)
    int pad0;
    unsigned long long pairs, rotations;  // helpers' work counts, taken by the leader
    FusedCtl* fc;
    int pad[8];
};
static_assert(sizeof(GangCtl) == 128, "one control block per 128-byte line");

struct PatchDesc {
    const float* image;
    long long stride;
    int H, W;
    int m, n, model, pp;      // pp = number of free parameters = model - 3
    int nc, nr, ldg, colmajor;
    int ld;                   // LDS row stride of the Jacobi matrix
    int svt_cfg;
    int tb;                   // rows per reconstruction block
    int sb;                   // tiled SVT: rows per super-block (0: whole matrix in LDS)
    int nsb;                  // tiled SVT: super-blocks (even)
    int ncp;                  // tiled SVT: rows of the working plane (nsb * sb >= nc)
    int warm;                 // SVT warm-started from the previous rotation: 1 FP32 start,
                              // 2 bfloat16 start + FP32 refinement, 3 bfloat16 start
    int pad1;
    double cx, cy, s;         // scaled coordinates of the level being solved (the
                              // kernels take them from PatchState::geo)
    double lam;
    float* ws;                // NPLANES planes (+ two ncp x ldg working planes when tiled:
                              // the Jacobi rows, then the rotation rows of the warm start)
    float* A_out;             // m x n row-major (may be null)
    float* E_out;
    GangCtl* gang;            // fused kernel, tiled windows: where helpers find its rounds (else null)
};

struct PatchState {
    double tau[MAXP];
    double NQ[MAXP * MAXPP];  // orthonormal basis of null(Q), p x pp
    double R[MAXPP * MAXPP];  // J~ = Qb R (upper triangular)
    double mu, c, dtau_norm, cond1, cond2, nuc, l1, objective;
    double dA2, dE2;
    int outer, inner, inner_total, done_inner, done_outer, status, svt_rank, warn;
    int num_rank;              // #{sigma_i(A) > 1e-3 sigma_1(A)} of the last SVT's result A
    int pad_rank;
    double f_prev;             // ||A||_* + lam ||E||_1 after the previous outer iteration of this level
    long long svt_calls, sweeps, pairs, rotations, recon_rows;
    long long t_begin, t_end;  // device wall clock at the start / end of the solve
    double geo[3];             // cx, cy, s of the level being solved
    int warm_ok;               // PL_V holds a rotation for this level's shape
    int warm_count;            // warm-started SVTs since the rotation was reset
    int svdws_ok;              // svt_mode 4: the region holds the previous decomposition
    int pad_svdws;
    long long svdws_steps;     // svt_mode 4: SVTs taken by a Cayley step
};

struct SolverParams {
    double eps1, eps2, eps_outer, mu0, rho0, mu_max;
    double eps_obj;  // outer stop when the objective changes by less than eps_obj times itself (0: off)
    int max_inner, max_outer, fixed_iters, max_sweeps;
    float jacobi_tol;
    int ns_every;  // warm SVT: Newton-Schulz re-orthonormalisation of the rotation every ns_every SVTs
    double eps_svd;   // svt_mode 4: Cayley step when ||M_k - M_prev||_F < eps_svd ||M_k||_F
    int svdws_every;  // svt_mode 4: > 0 replaces that rule by a fixed one (full SVD when inner % svdws_every == 0)
};

// SVD with warm start (svt_mode 4): words of the Cayley step's scratch for
// an m x n matrix (m >= n), and of the per-window region that follows the
// solver planes: the decomposition (U m x n, V n x n, Sigma n), the previous
// and the current matrix, the step's outputs and scratch, each rounded up
// to 64 words.
__host__ __device__ inline size_t svdws_scratch_words(int m, int n) {
    return (size_t)8 * m * n + (size_t)12 * n * n + (size_t)2 * n;
}
__host__ __device__ inline size_t svdws_round64(size_t w) { return (w + 63) & ~(size_t)63; }
__host__ __device__ inline size_t svdws_region_words(int m, int n) {
    const size_t mn = svdws_round64((size_t)m * n), nn = svdws_round64((size_t)n * n), s = svdws_round64(n);
    return 5 * mn + 2 * nn + 2 * s + svdws_round64(svdws_scratch_words(m, n));
}

// Jacobi tolerance of an inner-loop SVT.  The SVT's rounding (of the order
// of the tolerance, relative to ||M|| ~ 1 for the normalised window) enters
// the Cond2 quantity multiplied by mu, so the tolerance follows a tenth of
// the resolution Cond2 needs, eps2 / (10 mu), between the FP32 floor 1e-7
// and the cap.  The cap is tol_max for rows of up to 256 floats and
// tol_max sqrt(256 / len) for longer rows (len: the row length, the larger
// side), as the FP32 rounding of a row inner product grows like the
// square root of its length.
__host__ __device__ inline float svt_tolerance_cap(float tol_max, int len) {
    return len > 256 ? (float)((double)tol_max * sqrt(256.0 / (double)len)) : tol_max;
}
__host__ __device__ inline float svt_tolerance(float tol_max, double eps2, double mu, int len) {
    const double cap = (double)svt_tolerance_cap(tol_max, len);
    double t = 0.1 * eps2 / mu;
    if (!(t >= 1e-7)) t = 1e-7;
    if (t > cap) t = cap;
    return (float)t;
}

// Scaled coordinates of an m x n window (shared by host and device, FP64).
// Hn = T^{-1} H diag(s, s, 1) with T = [[s, 0, cx], [0, s, cy], [0, 0, 1]],
// (cx, cy) the image of the grid centre, s = max(m, n)/2, h33 = 1.
// Returns false for a non-finite or singular H.
__host__ __device__ inline bool normalise_h(const double* Hpx, int m, int n, double* geo, double* Hn) {
    for (int k = 0; k < 9; ++k)
        if (!(Hpx[k] == Hpx[k]) || Hpx[k] - Hpx[k] != 0.0) return false;
    if (Hpx[8] == 0.0) return false;
    double H[9];
    for (int k = 0; k < 9; ++k) H[k] = Hpx[k] / Hpx[8];
    const double s = (m > n ? m : n) / 2.0;
    const double cx = H[2], cy = H[5];
    for (int j = 0; j < 3; ++j) {
        const double sc = (j < 2) ? s : 1.0;
        Hn[0 * 3 + j] = (H[0 * 3 + j] - cx * H[2 * 3 + j]) / s * sc;
        Hn[1 * 3 + j] = (H[1 * 3 + j] - cy * H[2 * 3 + j]) / s * sc;
        Hn[2 * 3 + j] = H[2 * 3 + j] * sc;
    }
    const double h22 = Hn[8];
    if (h22 == 0.0) return false;
    for (int k = 0; k < 9; ++k) Hn[k] /= h22;
    const double det = Hn[0] * (Hn[4] * Hn[8] - Hn[5] * Hn[7]) - Hn[1] * (Hn[3] * Hn[8] - Hn[5] * Hn[6]) +
                       Hn[2] * (Hn[3] * Hn[7] - Hn[4] * Hn[6]);
    if (!(det > 1e-12 || det < -1e-12)) return false;
    geo[0] = cx;
    geo[1] = cy;
    geo[2] = s;
    return true;
}

// Inverse of normalise_h: H = T Hn diag(1/s, 1/s, 1), scaled to h33 = 1.
__host__ __device__ inline void denormalise_h(const double* Hn, const double* geo, double* Hpx) {
    const double cx = geo[0], cy = geo[1], s = geo[2];
    double H[9];
    for (int j = 0; j < 3; ++j) {
        const double sc = (j < 2) ? 1.0 / s : 1.0;
        H[0 * 3 + j] = (s * Hn[0 * 3 + j] + cx * Hn[2 * 3 + j]) * sc;
        H[1 * 3 + j] = (s * Hn[1 * 3 + j] + cy * Hn[2 * 3 + j]) * sc;
        H[2 * 3 + j] = Hn[2 * 3 + j] * sc;
    }
    for (int k = 0; k < 9; ++k) Hpx[k] = H[k] / H[8];
}

// Pixel and centred grid coordinates halve from one pyramid level to the
// next: H_coarse = S H_fine S^{-1} with S = diag(1/2, 1/2, 1).
__host__ __device__ inline void to_coarser_h(double* H) {
    H[2] *= 0.5;
    H[5] *= 0.5;
    H[6] *= 2.0;
    H[7] *= 2.0;
}
__host__ __device__ inline void to_finer_h(double* H) {
    H[2] *= 2.0;
    H[5] *= 2.0;
    H[6] *= 0.5;
    H[7] *= 0.5;
}

// RASL problem: the data matrix holds one window per image.  In the X
// layout of `d` the images are the rows (nc = count, nr = m n, colmajor =
// 0), so the one-sided Jacobi orthogonalises whole windows and the
// per-image projections run along contiguous rows.  d.image, d.stride, d.H
// and d.W describe image 0; image k starts img_stride floats further.
// d.s is the common scale; every image has its own window centre in geo and
// transform in tau, both in the workspace after the planes.
struct RaslDesc {
    PatchDesc d;
    long long img_stride;
    double* tau;   // count x MAXP scaled transforms (updated in place)
    double* geo;   // count x 2 window centres (cx, cy)
    double* Rf;    // count x MAXP x MAXP: J_k = Q_k R_k, R_k upper triangular
    int count;
    int pad[3];
};

// Launch shape of the SVT for one matrix shape.
struct SvtShape {
    int cfg, ld, tb;
    int sb, nsb, ncp;
};

// Standalone SVT job (component entry point).
struct SvtJob {
    const float* M;   // m x n row-major
    float* A;         // m x n row-major
    float* sigma;     // min(m, n) singular values (unsorted), may be null
    int m, n;
    float eps;
    int pad;
};

// One step of the SVD with warm start (component entry point): the
// previous decomposition (U m x n, S n, V n x n), the next matrix M (m x n,
// m >= n), the outputs, the threshold of the optional shrinkage A_out, and
// the step size, f(0), f(t) and status written back.
struct SvdwsJob {
    const float* U;
    const float* S;
    const float* V;
    const float* M;
    float* U_out;
    float* S_out;
    float* V_out;
    float* A_out;
    float eps;
    int status;
    double t, f0, ft;
};
size_t svdws_scratch_bytes(int m, int n);
hipError_t launch_svdws(SvdwsJob* jobs, int count, int m, int n, float* scratch, hipStream_t s);

// LDS layout helpers (host and device).
// cfg = TL * 256 + (BS - 1) * 128 + log2(LPP / 4) * 16 + (NCH - 1): blocks of
// BS rows, LPP lanes per block pair, NCH float4 chunks per lane and row,
// then TL (0, 1 or 2) single floats per lane, so a lane group covers
// LPP * (4 NCH + TL) floats of a row.
__host__ __device__ constexpr int svt_make_cfg(int bs, int lpp, int nch, int tl = 0) {
    return tl * 256 + (bs - 1) * 128 + (lpp == 4 ? 0 : lpp == 8 ? 1 : lpp == 16 ? 2 : lpp == 32 ? 3 : 4) * 16 +
           (nch - 1);
}
__host__ __device__ inline int svt_bs(int cfg) { return ((cfg >> 7) & 1) + 1; }
__host__ __device__ inline int svt_lpp(int cfg) { return 4 << ((cfg >> 4) & 7); }
__host__ __device__ inline int svt_nch(int cfg) { return (cfg & 15) + 1; }
__host__ __device__ inline int svt_tl(int cfg) { return (cfg >> 8) & 3; }
// Floats of a row covered by one lane group.
__host__ __device__ inline int svt_span(int cfg) { return svt_lpp(cfg) * (4 * svt_nch(cfg) + svt_tl(cfg)); }

// Serving ring: request slots and the control word live in pinned
// (coherent) host memory; the host publishes requests by raising `tail`,
// workgroups of the serving kernel claim them through a device counter and
// set `done` = sequence number + 1 when the result is in place.
struct ServeSlot {
    PatchDesc d[MAX_LEVELS];  // level 0 (the window as given) .. levels-1
    SolverParams prm;
    PatchState init;          // tau, geo of the coarsest level
    PatchState result;
    int levels;
    int pad[3];
    unsigned long long done;
};

struct ServeCtl {
    unsigned long long tail;  // requests published
    int stop;                 // host: finish the current requests and exit
    int pad;
};

// Kernel launchers (tilt_kernels.hip).
// help = 1: workgroups that run out of requests help the leaders of tiled
// windows until every request is done (else they exit).
hipError_t launch_fused(const PatchDesc* d, PatchState* st, const SolverParams& prm, int count, int levels,
                        const int* order, FusedCtl* fc, int help, int grid, size_t lds, hipStream_t s);
hipError_t launch_wide_setup(const PatchDesc* d, PatchState* st, const SolverParams& prm, const float* I,
                             const float* J, int count, size_t lds, hipStream_t s);
hipError_t launch_wide_stage(const PatchDesc* d, PatchState* st, const int* active, int nactive, int form_m,
                             int* flags, hipStream_t s);
hipError_t launch_wide_round(const PatchDesc* d, PatchState* st, const int* active, int nactive, int pairs, int r,
                             float tol, double eps2, int* flags, size_t lds, bool configure, hipStream_t s);
hipError_t launch_wide_finish(const PatchDesc* d, PatchState* st, const int* active, int nactive,
                              const SolverParams& prm, const int* sweeps, int mode, size_t lds, hipStream_t s);
hipError_t launch_wide_update(const PatchDesc* d, PatchState* st, const int* active, int nactive,
                              const SolverParams& prm, hipStream_t s);
hipError_t launch_wide_end(const PatchDesc* d, PatchState* st, int count, hipStream_t s);
hipError_t launch_rasl(const RaslDesc* d, PatchState* st, const SolverParams& prm, int count, int* queue, int grid,
                       size_t lds, hipStream_t s);
// fc, help: the helpers' control block (FusedCtl with a GangCtl per ring
// slot) and whether idle workgroups help the leaders of tiled requests.
hipError_t launch_serve(ServeCtl* ctl, ServeSlot* slots, PatchDesc* ddesc, PatchState* dstates,
                        unsigned long long* ctr, int ring, long long idle_ticks, FusedCtl* fc, int help, int grid,
                        size_t lds, hipStream_t s);
hipError_t launch_pyramid_build(const PatchDesc* d, int levels, hipStream_t s);
hipError_t launch_level_begin(const PatchDesc* d, PatchState* st, int first, hipStream_t s);
hipError_t launch_pyramid_jobs(const float* image, int H, int W, long long stride, float* out, int levels,
                               hipStream_t s);
hipError_t launch_setup(const PatchDesc* d, PatchState* st, const SolverParams& prm, size_t lds, hipStream_t s);
hipError_t launch_svt(const PatchDesc* d, PatchState* st, const SolverParams& prm, size_t lds, hipStream_t s,
                      bool configure = true);
hipError_t launch_update(const PatchDesc* d, PatchState* st, const SolverParams& prm, hipStream_t s);
hipError_t launch_dtau(const PatchDesc* d, PatchState* st, const SolverParams& prm, hipStream_t s);
hipError_t launch_finalize(const PatchDesc* d, PatchState* st, int last, hipStream_t s);
hipError_t launch_mark_end(PatchState* st, hipStream_t s);
hipError_t launch_inner(const PatchDesc* d, PatchState* st, const SolverParams& prm, const float* I, const float* J,
                        int count, size_t lds, hipStream_t s);
hipError_t launch_step1(const PatchDesc* d, PatchState* st, int count, double* partial, float* I_out, float* J_out,
                        hipStream_t s);
hipError_t launch_svt_jobs(const SvtJob* jobs, int count, const SvtShape& shape, float tol,
                           int max_sweeps, long long* counters, float* scratch, size_t lds, hipStream_t s);

}  // namespace tilt
