// Host side of the C interface declared in include/tilt.h: argument
// validation, transform normalisation (FP64), device workspace, and the
// plain (step-by-step) and batched (fused persistent) drivers.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "tilt.h"
#include "tilt_internal.h"

using namespace tilt;

namespace {

constexpr int kStaticLdsMargin = 8 * 1024;  // static __shared__ use of the kernels (checked at launch)

// ---------------------------------------------------------------------------
// Device buffer that grows on demand.
// ---------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = need;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// Shape-dependent launch configuration of the SVT for one patch.
struct ShapeCfg {
    int nc, nr, ldg, colmajor, cfg, ld, tb;
    int sb, nsb, ncp;  // tiled SVT (sb = 0: the whole matrix is held in LDS)
    size_t lds;
    size_t ws_floats;
};

// Jacobi layout for a matrix of nc rows of nr4 float4 chunks: rows per
// block (BS), lanes per block pair (LPP) and chunks per lane (NCH).  The
// model counts, per sweep, rounds x block pairs per lane group x the
// instructions of a round (BS^2 rotations of NCH chunks plus a fixed cost
// for the reduction and rotation parameters that grows with the reduction
// width, plus the row loads/stores), and divides by the number of
// concurrent groups' worth of issue slots when fewer groups than slots are
// busy.  The cheapest layout wins.
int pick_svt_cfg(int nc, int nr4) {
    const int nc4 = (nc + 3) & ~3;
    int best = -1;
    double best_cost = 1e300;
    const int lpps[3] = {4, 8, 16};
    for (int bs = 1; bs <= 2; ++bs) {
        for (int li = 0; li < 3; ++li) {
            const int lpp = lpps[li];
            const int nch = (nr4 + lpp - 1) / lpp;
            if (nch > (bs == 1 ? SVT_MAX_NCH : 4)) continue;
            const int groups = NT / lpp;
            const int nb = nc4 / bs;
            const int pairs = nb / 2;
            const int per_group = (pairs + groups - 1) / groups;
            const int active = std::min(pairs, groups);
            const double rot = 20.0 * nch + 30.0 + 4.0 * li;
            const double round_instr = per_group * (bs * bs * rot + 4.0 * bs * nch) + 40.0;
            // waves with work per SIMD: issue-bound when >= 2, latency-bound below
            const double waves = std::max(1.0, active * (double)lpp / 64.0 / 4.0);
            const double round_cycles = round_instr * 4.0 * std::max(waves, 2.0) / (bs == 2 ? 1.5 : 1.0);
            // layouts whose rows exceed the register budget spill to scratch
            const bool spills = NT > 256 && ((bs == 2 && nch > 2) || (bs == 1 && lpp == 16 && nch > 5));
            const double cost = (nb - 1) * round_cycles * (spills ? 4.0 : 1.0);
            if (cost < best_cost) {
                best_cost = cost;
                best = svt_make_cfg(bs, lpp, nch);
            }
        }
    }
    return best;
}

// LDS row stride: at least 4*LPP*NCH floats (every lane reads NCH chunks)
// and chosen so that the lane groups served by one 256-byte LDS pass
// (consecutive groups start BS rows apart) hit disjoint banks.
int pick_ld(int cfg) {
    const int bs = svt_bs(cfg), lpp = svt_lpp(cfg), nch = svt_nch(cfg);
    const int min_ld = 4 * lpp * nch;
    const int group_bytes = 16 * lpp;
    const int per_pass = std::max(1, 256 / group_bytes);
    for (int ld = min_ld; ld < min_ld + 256; ld += 4) {
        bool ok = true;
        unsigned used = 0;
        for (int gi = 0; gi < per_pass && ok; ++gi) {
            const int off = (gi * bs * ld * 4) % 256;
            if (off % group_bytes != 0) {
                ok = false;
                break;
            }
            const unsigned bit = 1u << (off / group_bytes);
            if (used & bit) ok = false;
            used |= bit;
        }
        if (ok) return ld;
    }
    return min_ld;
}

size_t lds_bytes(int nc, int ld, int tb) {
    const int nc4 = (nc + 3) & ~3;
    return sizeof(float) * ((size_t)nc4 * ld + (size_t)tb * ld + (size_t)nc4 * tb + 3 * (size_t)nc4);
}

size_t lds_bytes_tiled(int sb, int ncp, int ld, int ldg, int tb) {
    const size_t front = std::max((size_t)2 * sb * ld, (size_t)tb * ldg + (size_t)ncp * tb);
    return sizeof(float) * (front + 3 * (size_t)ncp);
}

// The whole matrix in LDS when it fits; otherwise the tiled Jacobi with the
// largest super-blocks whose staged pair fits (fewest block loads, most
// lane groups busy per round; the pairs examined per sweep, about ncp^2,
// do not depend on the block size).
int shape_config(int m, int n, ShapeCfg* out) {
    ShapeCfg c;
    c.colmajor = m >= n ? 1 : 0;
    c.nc = std::min(m, n);
    c.nr = std::max(m, n);
    c.ldg = (c.nr + 3) & ~3;
    c.sb = c.nsb = c.ncp = 0;
    const int nc4 = (c.nc + 3) & ~3;
    const size_t budget = (size_t)LDS_LIMIT - kStaticLdsMargin;
    if (nc4 <= SVT_MAX_ROWS) {
        c.cfg = pick_svt_cfg(c.nc, c.ldg / 4);
        if (c.cfg >= 0) {
            c.ld = pick_ld(c.cfg);
            for (int tb = 32; tb >= 16; tb -= 16) {
                c.tb = tb;
                c.lds = lds_bytes(c.nc, c.ld, c.tb);
                if (c.lds <= budget) {
                    c.ws_floats = (size_t)NPLANES * c.nc * c.ldg;
                    *out = c;
                    return TILT_OK;
                }
            }
        }
    }
    if (c.nr > SVT_MAX_COLS) return TILT_ERR_TOO_LARGE;
    for (int nsb = 2; nsb <= SVT_MAX_TILED_ROWS / 4; nsb += 2) {
        const int sb = (((nc4 + nsb - 1) / nsb) + 3) & ~3;
        if (2 * sb > SVT_MAX_ROWS) continue;
        const int ncp = nsb * sb;
        if (ncp > SVT_MAX_TILED_ROWS) break;
        const int cfg = pick_svt_cfg(2 * sb, c.ldg / 4);
        if (cfg < 0) return TILT_ERR_TOO_LARGE;
        const int ld = pick_ld(cfg);
        for (int tb = 32; tb >= 16; tb -= 16) {
            const size_t lds = lds_bytes_tiled(sb, ncp, ld, c.ldg, tb);
            if (lds <= budget) {
                c.cfg = cfg;
                c.ld = ld;
                c.tb = tb;
                c.sb = sb;
                c.nsb = nsb;
                c.ncp = ncp;
                c.lds = lds;
                c.ws_floats = (size_t)NPLANES * c.nc * c.ldg + (size_t)ncp * c.ldg;
                *out = c;
                return TILT_OK;
            }
        }
    }
    return TILT_ERR_TOO_LARGE;
}

// Predicted relative cost of a solve (one-sided Jacobi work per iteration).
double predicted_cost(const PatchDesc& d) { return (double)d.nc * d.nc * d.nr; }

// ---------------------------------------------------------------------------
// Transform normalisation (FP64).
// ---------------------------------------------------------------------------
struct Norm {
    double cx, cy, s;
    double tau[MAXP];
};

bool finite9(const double* h) {
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(h[k])) return false;
    return true;
}

int normalise(const double* Hpx, int m, int n, int model, Norm* out) {
    if (!finite9(Hpx) || Hpx[8] == 0.0) return TILT_ERR_ARG;
    double H[9];
    for (int k = 0; k < 9; ++k) H[k] = Hpx[k] / Hpx[8];
    const double scale = std::fabs(H[0]) + std::fabs(H[1]) + std::fabs(H[3]) + std::fabs(H[4]);
    if (model == TILT_AFFINE && (std::fabs(H[6]) > 1e-12 * (1.0 + scale) || std::fabs(H[7]) > 1e-12 * (1.0 + scale)))
        return TILT_ERR_ARG;
    const double s = std::max(m, n) / 2.0;
    const double cx = H[2], cy = H[5];
    // Hn = Timg^{-1} H diag(s, s, 1), Timg = [[s, 0, cx], [0, s, cy], [0, 0, 1]]
    double Hn[9];
    for (int j = 0; j < 3; ++j) {
        const double sc = (j < 2) ? s : 1.0;
        Hn[0 * 3 + j] = (H[0 * 3 + j] - cx * H[2 * 3 + j]) / s * sc;
        Hn[1 * 3 + j] = (H[1 * 3 + j] - cy * H[2 * 3 + j]) / s * sc;
        Hn[2 * 3 + j] = H[2 * 3 + j] * sc;
    }
    const double h22n = Hn[8];
    for (int k = 0; k < 9; ++k) Hn[k] /= h22n;
    out->cx = cx;
    out->cy = cy;
    out->s = s;
    out->tau[0] = Hn[0];
    out->tau[1] = Hn[1];
    out->tau[2] = Hn[2];
    out->tau[3] = Hn[3];
    out->tau[4] = Hn[4];
    out->tau[5] = Hn[5];
    out->tau[6] = model == TILT_PROJECTIVE ? Hn[6] : 0.0;
    out->tau[7] = model == TILT_PROJECTIVE ? Hn[7] : 0.0;
    const double det = Hn[0] * (Hn[4] * Hn[8] - Hn[5] * Hn[7]) - Hn[1] * (Hn[3] * Hn[8] - Hn[5] * Hn[6]) +
                       Hn[2] * (Hn[3] * Hn[7] - Hn[4] * Hn[6]);
    if (!(std::fabs(det) > 1e-12)) return TILT_ERR_ARG;
    return TILT_OK;
}

void denormalise(const double* tau, int model, double cx, double cy, double s, double* Hpx) {
    double Hn[9] = {tau[0], tau[1], tau[2], tau[3], tau[4], tau[5], 0.0, 0.0, 1.0};
    if (model == TILT_PROJECTIVE) {
        Hn[6] = tau[6];
        Hn[7] = tau[7];
    }
    // H = Timg Hn diag(1/s, 1/s, 1)
    double H[9];
    for (int j = 0; j < 3; ++j) {
        const double sc = (j < 2) ? 1.0 / s : 1.0;
        H[0 * 3 + j] = (s * Hn[0 * 3 + j] + cx * Hn[2 * 3 + j]) * sc;
        H[1 * 3 + j] = (s * Hn[1 * 3 + j] + cy * Hn[2 * 3 + j]) * sc;
        H[2 * 3 + j] = Hn[2 * 3 + j] * sc;
    }
    const double h22 = H[8];
    for (int k = 0; k < 9; ++k) Hpx[k] = H[k] / h22;
}

int validate_params(const tilt_params* p) {
    if (!p) return TILT_ERR_ARG;
    if (!(p->eps1 > 0) || !(p->eps2 > 0) || !(p->eps_outer >= 0)) return TILT_ERR_ARG;
    if (!(p->rho0 >= 1.0) || !(p->mu_max > 0)) return TILT_ERR_ARG;
    if (p->max_inner < 1 || p->max_outer < 1 || p->max_sweeps < 1) return TILT_ERR_ARG;
    if (!(p->jacobi_tol > 0.f) || !(p->jacobi_tol < 1.f)) return TILT_ERR_ARG;
    if (p->svt_mode != 0) return TILT_ERR_ARG;
    if (!std::isfinite(p->lambda) || !std::isfinite(p->mu0)) return TILT_ERR_ARG;
    return TILT_OK;
}

int validate_problem(const tilt_problem* pr) {
    if (!pr || !pr->image) return TILT_ERR_ARG;
    if (pr->height < 2 || pr->width < 2 || pr->row_stride < pr->width) return TILT_ERR_ARG;
    if (pr->m < 2 || pr->n < 2) return TILT_ERR_ARG;
    if (pr->model != TILT_AFFINE && pr->model != TILT_PROJECTIVE) return TILT_ERR_ARG;
    if (!finite9(pr->tau0)) return TILT_ERR_ARG;
    return TILT_OK;
}

SolverParams to_solver(const tilt_params* p) {
    SolverParams s;
    s.eps1 = p->eps1;
    s.eps2 = p->eps2;
    s.eps_outer = p->eps_outer;
    s.mu0 = p->mu0;
    s.rho0 = p->rho0;
    s.mu_max = p->mu_max;
    s.max_inner = p->max_inner;
    s.max_outer = p->max_outer;
    s.fixed_iters = p->fixed_iters ? 1 : 0;
    s.max_sweeps = p->max_sweeps;
    s.jacobi_tol = p->jacobi_tol;
    s.pad = 0;
    return s;
}

thread_local char g_last_error[512] = "";

int record_hip_error(hipError_t e, const char* what, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%s) at tilt_api.cpp:%d: %s", hipGetErrorName(e),
                  hipGetErrorString(e), line, what);
    return TILT_ERR_DEVICE;
}

int worse(int a, int b) {
    // errors (negative) dominate warnings (positive) dominate OK
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct tilt_ctx {
    int device = 0;
    size_t budget = 0;
    DevBuf descs, states, ws, queue, order, scratch, jobs, counters, img;
    double wall_rate_khz = 100000.0;  // device wall clock
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_kernel_ms = 0.0;
};

namespace {

struct Prepared {
    std::vector<PatchDesc> descs;
    std::vector<PatchState> states;
    std::vector<Norm> norms;
    std::vector<int> status;  // per-patch preparation status
    size_t max_lds = 0;
    size_t ws_floats = 0;
};

// Build descriptors; images are device pointers; A/E outputs device pointers.
int prepare(const tilt_problem* probs, int count, const tilt_params* prm, tilt_result* results, Prepared* P,
            bool device_outputs) {
    P->descs.resize(count);
    P->states.assign(count, PatchState{});
    P->norms.resize(count);
    P->status.assign(count, TILT_OK);
    size_t off = 0;
    int worst = TILT_OK;
    for (int i = 0; i < count; ++i) {
        const tilt_problem& pr = probs[i];
        int st = validate_problem(&pr);
        ShapeCfg sc{};
        if (st == TILT_OK) st = shape_config(pr.m, pr.n, &sc);
        Norm nm{};
        if (st == TILT_OK) st = normalise(pr.tau0, pr.m, pr.n, pr.model, &nm);
        P->status[i] = st;
        worst = worse(worst, st);
        PatchDesc& d = P->descs[i];
        std::memset(&d, 0, sizeof(d));
        if (st != TILT_OK) continue;
        d.image = pr.image;
        d.stride = pr.row_stride;
        d.H = pr.height;
        d.W = pr.width;
        d.m = pr.m;
        d.n = pr.n;
        d.model = pr.model;
        d.pp = pr.model - 3;
        d.nc = sc.nc;
        d.nr = sc.nr;
        d.ldg = sc.ldg;
        d.colmajor = sc.colmajor;
        d.ld = sc.ld;
        d.svt_cfg = sc.cfg;
        d.tb = sc.tb;
        d.sb = sc.sb;
        d.nsb = sc.nsb;
        d.ncp = sc.ncp;
        d.cx = nm.cx;
        d.cy = nm.cy;
        d.s = nm.s;
        d.lam = prm->lambda > 0 ? prm->lambda : 1.0 / std::sqrt((double)std::max(pr.m, pr.n));
        d.ws = reinterpret_cast<float*>(off);  // offset, rebased after allocation
        off += sc.ws_floats;
        d.A_out = device_outputs && results ? results[i].A : nullptr;
        d.E_out = device_outputs && results ? results[i].E : nullptr;
        PatchState& s = P->states[i];
        for (int k = 0; k < MAXP; ++k) s.tau[k] = nm.tau[k];
        P->norms[i] = nm;
        P->max_lds = std::max(P->max_lds, sc.lds);
    }
    P->ws_floats = off;
    return worst;
}

void fill_result(const PatchDesc& d, const PatchState& s, const Norm& nm, int prep_status, tilt_result* r,
                 double rate_khz, long long t0) {
    if (prep_status != TILT_OK) {
        r->status = prep_status;
        return;
    }
    r->solve_ms = (double)(s.t_end - s.t_begin) / rate_khz;
    r->done_ms = (double)(s.t_end - t0) / rate_khz;
    denormalise(s.tau, d.model, nm.cx, nm.cy, nm.s, r->tau);
    r->outer_iters = s.outer;
    r->inner_iters_total = s.inner_total;
    r->svt_rank = s.svt_rank;
    r->status = s.status < 0 ? s.status : (s.warn ? TILT_WARN_MAXITER : TILT_OK);
    r->objective = s.objective;
    r->mu = s.mu;
    r->cond1 = s.cond1;
    r->cond2 = s.cond2;
    r->dtau_norm = s.dtau_norm;
    r->counters.inner_iters = s.inner_total;
    r->counters.svt_calls = s.svt_calls;
    r->counters.jacobi_sweeps = s.sweeps;
    r->counters.jacobi_pairs = s.pairs;
    r->counters.jacobi_rotations = s.rotations;
    r->counters.recon_rows = s.recon_rows;
}

#define HIP_TRY(x)                                                  \
    do {                                                            \
        hipError_t _e = (x);                                        \
        if (_e != hipSuccess) return record_hip_error(_e, #x, __LINE__); \
    } while (0)

int upload(tilt_ctx* ctx, Prepared& P, hipStream_t stream) {
    const int count = (int)P.descs.size();
    if (P.ws_floats * sizeof(float) > ctx->budget) return TILT_ERR_NOMEM;
    if (ctx->ws.reserve(std::max<size_t>(P.ws_floats * sizeof(float), 256)) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->descs.reserve(sizeof(PatchDesc) * count) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->states.reserve(sizeof(PatchState) * count) != hipSuccess) return TILT_ERR_NOMEM;
    float* base = reinterpret_cast<float*>(ctx->ws.p);
    for (auto& d : P.descs) d.ws = base + reinterpret_cast<size_t>(d.ws);
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, P.descs.data(), sizeof(PatchDesc) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, P.states.data(), sizeof(PatchState) * count, hipMemcpyHostToDevice,
                           stream));
    return TILT_OK;
}

// Host-driven loop over the step kernels for patch idx (mirrors solve_patch).
int run_plain_patch(tilt_ctx* ctx, const Prepared& P, const SolverParams& sp, int idx, hipStream_t stream) {
    const PatchDesc* dd = reinterpret_cast<const PatchDesc*>(ctx->descs.p);
    PatchState* ds = reinterpret_cast<PatchState*>(ctx->states.p);
    const size_t lds = P.max_lds;
    PatchState hs;
    auto fetch = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(&hs, ds + idx, sizeof(PatchState), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return TILT_OK;
    };
    for (;;) {
        HIP_TRY(launch_setup(dd, ds, sp, idx, lds, stream));
        if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
        if (hs.status < 0) break;
        for (;;) {
            HIP_TRY(launch_svt(dd, ds, sp, idx, lds, stream));
            HIP_TRY(launch_update(dd, ds, sp, idx, stream));
            if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            if (hs.done_inner) break;
        }
        if (hs.status < 0) break;
        HIP_TRY(launch_dtau(dd, ds, sp, idx, stream));
        if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
        if (hs.done_outer) break;
    }
    HIP_TRY(launch_finalize(dd, ds, idx, stream));
    return TILT_OK;
}

int solve_batch_impl(tilt_ctx* ctx, const tilt_problem* probs, int count, const tilt_params* prm,
                     tilt_result* results, void* hip_stream, bool plain) {
    if (!ctx || !probs || count < 0 || !prm || !results) return TILT_ERR_ARG;
    int st = validate_params(prm);
    if (st != TILT_OK) return st;
    if (count == 0) return TILT_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Prepared P;
    int worst = prepare(probs, count, prm, results, &P, true);
    // Only valid patches are sent to the device.
    std::vector<int> live;
    for (int i = 0; i < count; ++i)
        if (P.status[i] == TILT_OK) live.push_back(i);
    if (!live.empty()) {
        Prepared Q;
        Q.max_lds = P.max_lds;
        Q.ws_floats = P.ws_floats;
        for (int i : live) {
            Q.descs.push_back(P.descs[i]);
            Q.states.push_back(P.states[i]);
        }
        int u = upload(ctx, Q, stream);
        if (u != TILT_OK) return u;
        const SolverParams sp = to_solver(prm);
        const int nlive = (int)live.size();
        if (plain) {
            for (int k = 0; k < nlive; ++k) {
                int r = run_plain_patch(ctx, Q, sp, k, stream);
                if (r != TILT_OK) return r;
            }
        } else {
            if (ctx->queue.reserve(256) != hipSuccess) return TILT_ERR_NOMEM;
            if (ctx->order.reserve(sizeof(int) * nlive) != hipSuccess) return TILT_ERR_NOMEM;
            // longest predicted solve first (stable: equal shapes keep their order)
            std::vector<int> order(nlive);
            for (int k = 0; k < nlive; ++k) order[k] = k;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                return predicted_cost(Q.descs[a]) > predicted_cost(Q.descs[b]);
            });
            HIP_TRY(hipMemcpyAsync(ctx->order.p, order.data(), sizeof(int) * nlive, hipMemcpyHostToDevice, stream));
            HIP_TRY(hipMemsetAsync(ctx->queue.p, 0, sizeof(int), stream));
            int ncu = 256;
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
                ncu = prop.multiProcessorCount;
            const int per_cu = std::max<int>(1, (int)(LDS_LIMIT / (Q.max_lds + kStaticLdsMargin)));
            const int grid = std::max(1, std::min(nlive, ncu * std::min(per_cu, 2)));
            HIP_TRY(hipEventRecord(ctx->ev0, stream));
            HIP_TRY(launch_fused(reinterpret_cast<const PatchDesc*>(ctx->descs.p),
                                 reinterpret_cast<PatchState*>(ctx->states.p), sp, nlive,
                                 reinterpret_cast<const int*>(ctx->order.p), reinterpret_cast<int*>(ctx->queue.p),
                                 grid, Q.max_lds, stream));
            HIP_TRY(hipEventRecord(ctx->ev1, stream));
        }
        std::vector<PatchState> out(nlive);
        HIP_TRY(hipMemcpyAsync(out.data(), ctx->states.p, sizeof(PatchState) * nlive, hipMemcpyDeviceToHost,
                               stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (!plain) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            ctx->last_kernel_ms = ms;
        }
        long long t0 = out[0].t_begin;
        for (int k = 1; k < nlive; ++k) t0 = std::min(t0, out[k].t_begin);
        for (int k = 0; k < nlive; ++k) {
            const int i = live[k];
            fill_result(P.descs[i], out[k], P.norms[i], TILT_OK, &results[i], ctx->wall_rate_khz, t0);
            worst = worse(worst, results[i].status);
        }
    }
    for (int i = 0; i < count; ++i)
        if (P.status[i] != TILT_OK) results[i].status = P.status[i];
    return worst;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------
extern "C" {

void tilt_default_params(tilt_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->lambda = -1.0;
    p->eps1 = 1e-5;
    p->eps2 = 1e-3;
    p->eps_outer = 1e-5;
    p->mu0 = -1.0;
    p->rho0 = 1.5;
    p->mu_max = 1e10;
    p->max_inner = 2000;
    p->max_outer = 50;
    p->fixed_iters = 0;
    p->svt_mode = 0;
    p->jacobi_tol = 1e-6f;
    p->max_sweeps = 40;
}

const char* tilt_status_string(int s) {
    switch (s) {
        case TILT_OK: return "ok";
        case TILT_WARN_MAXITER: return "inner loop reached max_inner";
        case TILT_PENDING: return "pending";
        case TILT_ERR_ARG: return "invalid argument";
        case TILT_ERR_NOMEM: return "out of device memory or over budget";
        case TILT_ERR_DEVICE: return "HIP runtime error";
        case TILT_ERR_SINGULAR: return "J^T J is singular";
        case TILT_ERR_NONFINITE: return "non-finite value in the iteration";
        case TILT_ERR_TOO_LARGE: return "patch too large for the on-chip SVT";
        case TILT_ERR_NOT_FOUND: return "unknown ticket";
        default: return "unknown status";
    }
}

const char* tilt_version(void) { return "tilt-mi355x 0.1 (gfx950)"; }

const char* tilt_last_error(void) { return g_last_error; }

int tilt_tau_from_quad(const double quad[8], int m, int n, int model, double tau_out[9]) {
    if (!quad || !tau_out || m < 2 || n < 2) return TILT_ERR_ARG;
    for (int k = 0; k < 8; ++k)
        if (!std::isfinite(quad[k])) return TILT_ERR_ARG;
    const double a = (n - 1) / 2.0, b = (m - 1) / 2.0;
    const double U[4] = {-a, a, a, -a}, V[4] = {-b, -b, b, b};
    if (model == TILT_AFFINE) {
        const double tlx = quad[0], tly = quad[1], trx = quad[2], try_ = quad[3];
        const double brx = quad[4], bry = quad[5], blx = quad[6], bly = quad[7];
        const double ex = trx - tlx, ey = try_ - tly, fx = blx - tlx, fy = bly - tly;
        const double scale = std::fabs(ex) + std::fabs(ey) + std::fabs(fx) + std::fabs(fy);
        if (std::fabs(brx - (trx + blx - tlx)) > 1e-9 * (1 + scale) ||
            std::fabs(bry - (try_ + bly - tly)) > 1e-9 * (1 + scale))
            return TILT_ERR_ARG;
        const double h00 = ex / (2 * a), h10 = ey / (2 * a), h01 = fx / (2 * b), h11 = fy / (2 * b);
        const double cx = tlx + 0.5 * ex + 0.5 * fx, cy = tly + 0.5 * ey + 0.5 * fy;
        const double det = h00 * h11 - h01 * h10;
        if (!(std::fabs(det) > 1e-12)) return TILT_ERR_ARG;
        const double H[9] = {h00, h01, cx, h10, h11, cy, 0, 0, 1};
        std::memcpy(tau_out, H, sizeof(H));
        return TILT_OK;
    }
    if (model != TILT_PROJECTIVE) return TILT_ERR_ARG;
    // 8x8 linear system for h11..h32 with h33 = 1.
    double Mx[8][9];
    for (int c = 0; c < 4; ++c) {
        const double u = U[c], v = V[c], x = quad[2 * c], y = quad[2 * c + 1];
        double r1[9] = {u, v, 1, 0, 0, 0, -u * x, -v * x, x};
        double r2[9] = {0, 0, 0, u, v, 1, -u * y, -v * y, y};
        std::memcpy(Mx[2 * c], r1, sizeof(r1));
        std::memcpy(Mx[2 * c + 1], r2, sizeof(r2));
    }
    for (int col = 0; col < 8; ++col) {
        int piv = col;
        for (int r = col + 1; r < 8; ++r)
            if (std::fabs(Mx[r][col]) > std::fabs(Mx[piv][col])) piv = r;
        if (!(std::fabs(Mx[piv][col]) > 1e-12)) return TILT_ERR_ARG;
        if (piv != col)
            for (int k = 0; k < 9; ++k) std::swap(Mx[piv][k], Mx[col][k]);
        for (int r = 0; r < 8; ++r) {
            if (r == col) continue;
            const double f = Mx[r][col] / Mx[col][col];
            for (int k = col; k < 9; ++k) Mx[r][k] -= f * Mx[col][k];
        }
    }
    for (int k = 0; k < 8; ++k) tau_out[k] = Mx[k][8] / Mx[k][k];
    tau_out[8] = 1.0;
    return TILT_OK;
}

int tilt_ctx_create(tilt_ctx** ctx, int device, size_t hbm_budget_bytes) {
    if (!ctx) return TILT_ERR_ARG;
    *ctx = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (ndev <= 0) return TILT_ERR_DEVICE;
    if (device < 0 || device >= ndev) return TILT_ERR_ARG;
    HIP_TRY(hipSetDevice(device));
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    tilt_ctx* c = new (std::nothrow) tilt_ctx();
    if (!c) return TILT_ERR_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : free_b / 2;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0)
        c->wall_rate_khz = (double)rate;
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return TILT_ERR_DEVICE;
    }
    *ctx = c;
    return TILT_OK;
}

int tilt_ctx_destroy(tilt_ctx* ctx) {
    if (!ctx) return TILT_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->descs.release();
    ctx->states.release();
    ctx->ws.release();
    ctx->queue.release();
    ctx->order.release();
    ctx->scratch.release();
    ctx->jobs.release();
    ctx->counters.release();
    ctx->img.release();
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return TILT_OK;
}

int tilt_ctx_last_kernel_ms(tilt_ctx* ctx, double* ms) {
    if (!ctx || !ms) return TILT_ERR_ARG;
    *ms = ctx->last_kernel_ms;
    return TILT_OK;
}

size_t tilt_workspace_bytes(const tilt_problem* prob) {
    if (!prob) return 0;
    ShapeCfg sc{};
    if (shape_config(prob->m, prob->n, &sc) != TILT_OK) return 0;
    return sc.ws_floats * sizeof(float) + sizeof(PatchDesc) + sizeof(PatchState);
}

int tilt_solve_batch(tilt_ctx* ctx, const tilt_problem* probs, int count, const tilt_params* prm,
                     tilt_result* results, void* hip_stream) {
    return solve_batch_impl(ctx, probs, count, prm, results, hip_stream, false);
}

int tilt_solve_batch_plain(tilt_ctx* ctx, const tilt_problem* probs, int count, const tilt_params* prm,
                           tilt_result* results, void* hip_stream) {
    return solve_batch_impl(ctx, probs, count, prm, results, hip_stream, true);
}

int tilt_solve(const tilt_problem* prob, const tilt_params* prm, tilt_result* res) {
    if (!prob || !prm || !res) return TILT_ERR_ARG;
    int st = validate_params(prm);
    if (st != TILT_OK) return st;
    st = validate_problem(prob);
    if (st != TILT_OK) {
        res->status = st;
        return st;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    tilt_ctx* ctx = nullptr;
    st = tilt_ctx_create(&ctx, dev, 0);
    if (st != TILT_OK) return st;
    const size_t mn = (size_t)prob->m * prob->n;
    const size_t img_elems = (size_t)(prob->height - 1) * prob->row_stride + prob->width;
    int rc = TILT_OK;
    hipStream_t stream = nullptr;
    float* dA = nullptr;
    float* dE = nullptr;
    do {
        if (hipStreamCreate(&stream) != hipSuccess) {
            rc = TILT_ERR_DEVICE;
            break;
        }
        if (ctx->img.reserve(img_elems * sizeof(float)) != hipSuccess ||
            ctx->scratch.reserve(2 * mn * sizeof(float)) != hipSuccess) {
            rc = TILT_ERR_NOMEM;
            break;
        }
        if (hipMemcpyAsync(ctx->img.p, prob->image, img_elems * sizeof(float), hipMemcpyHostToDevice, stream) !=
            hipSuccess) {
            rc = TILT_ERR_DEVICE;
            break;
        }
        dA = reinterpret_cast<float*>(ctx->scratch.p);
        dE = dA + mn;
        tilt_problem dp = *prob;
        dp.image = reinterpret_cast<const float*>(ctx->img.p);
        tilt_result r = *res;
        r.A = dA;
        r.E = dE;
        rc = tilt_solve_batch_plain(ctx, &dp, 1, prm, &r, stream);
        if (rc < 0 && r.status == 0) r.status = rc;
        float* hA = res->A;
        float* hE = res->E;
        *res = r;
        res->A = hA;
        res->E = hE;
        if (rc == TILT_ERR_DEVICE) break;
        if (hA && hipMemcpyAsync(hA, dA, mn * sizeof(float), hipMemcpyDeviceToHost, stream) != hipSuccess) {
            rc = TILT_ERR_DEVICE;
            break;
        }
        if (hE && hipMemcpyAsync(hE, dE, mn * sizeof(float), hipMemcpyDeviceToHost, stream) != hipSuccess) {
            rc = TILT_ERR_DEVICE;
            break;
        }
        if (hipStreamSynchronize(stream) != hipSuccess) rc = TILT_ERR_DEVICE;
    } while (0);
    if (stream) (void)hipStreamDestroy(stream);
    tilt_ctx_destroy(ctx);
    return rc;
}

int tilt_svt_batch(tilt_ctx* ctx, const float* M, float* A, float* sigma, int count, int m, int n,
                   const float* eps, const tilt_params* prm, int* ranks, tilt_counters* counters,
                   void* hip_stream) {
    if (!ctx || !M || !A || !eps || !prm || count < 0 || m < 1 || n < 1) return TILT_ERR_ARG;
    int st = validate_params(prm);
    if (st != TILT_OK) return st;
    if (count == 0) return TILT_OK;
    ShapeCfg sc{};
    st = shape_config(m, n, &sc);
    if (st != TILT_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t mn = (size_t)m * n;
    const int k = std::min(m, n);
    std::vector<SvtJob> jobs(count);
    for (int i = 0; i < count; ++i) {
        if (!std::isfinite(eps[i]) || eps[i] < 0.f) return TILT_ERR_ARG;
        jobs[i].M = M + (size_t)i * mn;
        jobs[i].A = A + (size_t)i * mn;
        jobs[i].sigma = sigma ? sigma + (size_t)i * k : nullptr;
        jobs[i].m = m;
        jobs[i].n = n;
        jobs[i].eps = eps[i];
        jobs[i].pad = 0;
    }
    const size_t np = (size_t)sc.nc * sc.ldg;
    const size_t per_job = 2 * np + (sc.sb > 0 ? (size_t)sc.ncp * sc.ldg : 0);
    if (ctx->jobs.reserve(sizeof(SvtJob) * count) != hipSuccess ||
        ctx->counters.reserve(sizeof(long long) * 4 * count) != hipSuccess ||
        ctx->scratch.reserve(sizeof(float) * per_job * count) != hipSuccess)
        return TILT_ERR_NOMEM;
    HIP_TRY(hipMemcpyAsync(ctx->jobs.p, jobs.data(), sizeof(SvtJob) * count, hipMemcpyHostToDevice, stream));
    const SvtShape shape{sc.cfg, sc.ld, sc.tb, sc.sb, sc.nsb, sc.ncp};
    HIP_TRY(launch_svt_jobs(reinterpret_cast<const SvtJob*>(ctx->jobs.p), count, shape, prm->jacobi_tol,
                            prm->max_sweeps, reinterpret_cast<long long*>(ctx->counters.p),
                            reinterpret_cast<float*>(ctx->scratch.p), sc.lds, stream));
    std::vector<long long> cnt(4 * (size_t)count);
    HIP_TRY(hipMemcpyAsync(cnt.data(), ctx->counters.p, sizeof(long long) * 4 * count, hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (counters) std::memset(counters, 0, sizeof(*counters));
    for (int i = 0; i < count; ++i) {
        if (ranks) ranks[i] = (int)cnt[4 * i + 3];
        if (counters) {
            counters->svt_calls += 1;
            counters->jacobi_sweeps += cnt[4 * i + 0];
            counters->jacobi_pairs += cnt[4 * i + 1];
            counters->jacobi_rotations += cnt[4 * i + 2];
            counters->recon_rows += cnt[4 * i + 3];
        }
    }
    return TILT_OK;
}

int tilt_warp_jacobian(tilt_ctx* ctx, const tilt_problem* probs, const double* taus, int count, float* I_out,
                       float* J_out, void* hip_stream) {
    if (!ctx || !probs || !taus || !I_out || !J_out || count < 0) return TILT_ERR_ARG;
    if (count == 0) return TILT_OK;
    const int m = probs[0].m, n = probs[0].n, model = probs[0].model;
    std::vector<PatchDesc> descs(count);
    std::vector<PatchState> states(count);
    for (int i = 0; i < count; ++i) {
        const tilt_problem& pr = probs[i];
        int st = validate_problem(&pr);
        if (st != TILT_OK) return st;
        if (pr.m != m || pr.n != n || pr.model != model) return TILT_ERR_ARG;
        Norm ref{}, cur{};
        st = normalise(pr.tau0, m, n, model, &ref);
        if (st != TILT_OK) return st;
        // The transform being evaluated, expressed in the window's scaled
        // coordinates (centre = image of the grid centre under tau0).
        double H[9];
        for (int k = 0; k < 9; ++k) H[k] = taus[9 * i + k];
        if (!finite9(H) || H[8] == 0.0) return TILT_ERR_ARG;
        for (int k = 0; k < 9; ++k) H[k] /= taus[9 * i + 8];
        const double s = ref.s;
        double Hn[9];
        for (int j = 0; j < 3; ++j) {
            const double sc = (j < 2) ? s : 1.0;
            Hn[0 * 3 + j] = (H[0 * 3 + j] - ref.cx * H[2 * 3 + j]) / s * sc;
            Hn[1 * 3 + j] = (H[1 * 3 + j] - ref.cy * H[2 * 3 + j]) / s * sc;
            Hn[2 * 3 + j] = H[2 * 3 + j] * sc;
        }
        const double h22n = Hn[8];
        for (int k = 0; k < 9; ++k) Hn[k] /= h22n;
        (void)cur;
        PatchDesc& d = descs[i];
        std::memset(&d, 0, sizeof(d));
        d.image = pr.image;
        d.stride = pr.row_stride;
        d.H = pr.height;
        d.W = pr.width;
        d.m = m;
        d.n = n;
        d.model = model;
        d.pp = model - 3;
        d.cx = ref.cx;
        d.cy = ref.cy;
        d.s = s;
        PatchState& ps = states[i];
        std::memset(&ps, 0, sizeof(ps));
        for (int k = 0; k < 6; ++k) ps.tau[k] = Hn[k];
        ps.tau[6] = model == TILT_PROJECTIVE ? Hn[6] : 0.0;
        ps.tau[7] = model == TILT_PROJECTIVE ? Hn[7] : 0.0;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (ctx->descs.reserve(sizeof(PatchDesc) * count) != hipSuccess ||
        ctx->states.reserve(sizeof(PatchState) * count) != hipSuccess)
        return TILT_ERR_NOMEM;
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(PatchDesc) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, states.data(), sizeof(PatchState) * count, hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(launch_step1(reinterpret_cast<const PatchDesc*>(ctx->descs.p),
                         reinterpret_cast<PatchState*>(ctx->states.p), count, I_out, J_out, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return TILT_OK;
}

}  // extern "C"
