// Host side of the RASL variant: validation, workspace layout, one fused
// launch per batch (k_rasl), results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"

using namespace tilt;
using namespace tilt::host;

namespace {

// Per-image arrays after the planes: tau (MAXP), window centre (2) and the
// factor R_k (MAXP x MAXP), all FP64.
constexpr size_t kPerImageDoubles = MAXP + 2 + MAXP * MAXP;

struct RaslPlan {
    RaslDesc rd;
    size_t ws_floats = 0;
    size_t planes_floats = 0;
    size_t lds = 0;
    std::vector<double> tau, geo;  // count x MAXP, count x 2 (host copies of the initial values)
};

int plan_rasl(const tilt_rasl_problem& pr, const tilt_params* prm, const tilt_rasl_result& res, RaslPlan* out) {
    if (!pr.images || !pr.tau0) return TILT_ERR_ARG;
    if (pr.model != TILT_AFFINE && pr.model != TILT_PROJECTIVE) return TILT_ERR_ARG;
    if (pr.height < 2 || pr.width < 2 || pr.row_stride < pr.width) return TILT_ERR_ARG;
    if (pr.m < 2 || pr.n < 2 || pr.count < 2) return TILT_ERR_ARG;
    if (pr.image_stride < (long long)(pr.height - 1) * pr.row_stride + pr.width) return TILT_ERR_ARG;
    const long long L = (long long)pr.m * pr.n;
    if (L > SVT_MAX_COLS) return TILT_ERR_TOO_LARGE;
    if (pr.count >= L) return TILT_ERR_ARG;  // images are the shorter side of the data matrix
    ShapeCfg sc;
    int st = shape_config(pr.count, (int)L, &sc);
    if (st != TILT_OK) return st;
    if (sc.colmajor != 0 || sc.nc != pr.count || sc.nr != (int)L) return TILT_ERR_ARG;
    RaslPlan& P = *out;
    std::memset(&P.rd, 0, sizeof(P.rd));
    P.tau.assign((size_t)pr.count * MAXP, 0.0);
    P.geo.assign((size_t)pr.count * 2, 0.0);
    double s = 0.0;
    for (int k = 0; k < pr.count; ++k) {
        double geo[3], tau[MAXP];
        st = normalise_window(pr.tau0 + 9 * k, pr.m, pr.n, pr.model, geo, tau);
        if (st != TILT_OK) return st;
        for (int q = 0; q < MAXP; ++q) P.tau[(size_t)k * MAXP + q] = tau[q];
        P.geo[2 * k] = geo[0];
        P.geo[2 * k + 1] = geo[1];
        s = geo[2];
    }
    PatchDesc& d = P.rd.d;
    d.image = pr.images;
    d.stride = pr.row_stride;
    d.H = pr.height;
    d.W = pr.width;
    d.m = pr.m;
    d.n = pr.n;
    d.model = pr.model;
    d.pp = pr.model;
    d.nc = sc.nc;
    d.nr = sc.nr;
    d.ldg = sc.ldg;
    d.colmajor = 0;
    d.ld = sc.ld;
    d.svt_cfg = sc.cfg;
    d.warm = 0;
    d.tb = sc.tb;
    d.sb = sc.sb;
    d.nsb = sc.nsb;
    d.ncp = sc.ncp;
    d.s = s;
    d.lam = prm->lambda > 0 ? prm->lambda : 1.0 / std::sqrt((double)std::max<long long>(L, pr.count));
    d.A_out = res.A;
    d.E_out = res.E;
    P.rd.img_stride = pr.image_stride;
    P.rd.count = pr.count;
    P.planes_floats = (sc.ws_floats + 63) & ~(size_t)63;
    P.ws_floats = P.planes_floats + ((2 * kPerImageDoubles * (size_t)pr.count + 63) & ~(size_t)63);
    P.lds = sc.lds;
    return TILT_OK;
}

}  // namespace

extern "C" int tilt_rasl_solve_batch(tilt_ctx* ctx, const tilt_rasl_problem* probs, int count, const tilt_params* prm,
                                     tilt_rasl_result* res, void* hip_stream) {
    if (!ctx || !probs || count < 0 || !prm || !res) return TILT_ERR_ARG;
    int st = validate_params(prm);
    if (st != TILT_OK) return st;
    if (prm->svt_mode != 0 || prm->pyramid_levels > 1) return TILT_ERR_ARG;
    if (count == 0) return TILT_OK;
    for (int i = 0; i < count; ++i)
        if (!res[i].tau) return TILT_ERR_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);

    std::vector<RaslPlan> plans(count);
    std::vector<int> live;
    int worst = TILT_OK;
    size_t total = 0, max_lds = 0;
    std::vector<size_t> off(count, 0);
    for (int i = 0; i < count; ++i) {
        const int s = plan_rasl(probs[i], prm, res[i], &plans[i]);
        res[i].status = s;
        if (s != TILT_OK) {
            worst = worse(worst, s);
            continue;
        }
        off[i] = total;
        total += plans[i].ws_floats;
        max_lds = std::max(max_lds, plans[i].lds);
        live.push_back(i);
    }
    if (live.empty()) return worst;
    if (total * sizeof(float) > ctx->budget) return TILT_ERR_NOMEM;
    const int nlive = (int)live.size();
    if (ctx->ws.reserve(std::max<size_t>(total * sizeof(float), 256)) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->descs.reserve(sizeof(RaslDesc) * nlive) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->states.reserve(sizeof(PatchState) * nlive) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->queue.reserve(256) != hipSuccess) return TILT_ERR_NOMEM;
    float* base = reinterpret_cast<float*>(ctx->ws.p);
    std::vector<RaslDesc> descs(nlive);
    std::vector<PatchState> states(nlive);
    for (int k = 0; k < nlive; ++k) {
        RaslPlan& P = plans[live[k]];
        float* ws = base + off[live[k]];
        RaslDesc rd = P.rd;
        rd.d.ws = ws;
        double* extra = reinterpret_cast<double*>(ws + P.planes_floats);
        const int N = rd.count;
        rd.tau = extra;
        rd.geo = extra + (size_t)N * MAXP;
        rd.Rf = extra + (size_t)N * (MAXP + 2);
        descs[k] = rd;
        std::memset(&states[k], 0, sizeof(PatchState));
        HIP_TRY(hipMemcpyAsync(rd.tau, P.tau.data(), sizeof(double) * P.tau.size(), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(rd.geo, P.geo.data(), sizeof(double) * P.geo.size(), hipMemcpyHostToDevice, stream));
    }
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(RaslDesc) * nlive, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, states.data(), sizeof(PatchState) * nlive, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemsetAsync(ctx->queue.p, 0, sizeof(int), stream));
    const int grid = std::max(1, std::min(nlive, ctx->num_cus));
    const SolverParams sp = to_solver(prm);
    HIP_TRY(hipEventRecord(ctx->ev0, stream));
    HIP_TRY(launch_rasl(reinterpret_cast<const RaslDesc*>(ctx->descs.p), reinterpret_cast<PatchState*>(ctx->states.p),
                        sp, nlive, reinterpret_cast<int*>(ctx->queue.p), grid, max_lds, stream));
    HIP_TRY(hipEventRecord(ctx->ev1, stream));
    std::vector<PatchState> out(nlive);
    HIP_TRY(hipMemcpyAsync(out.data(), ctx->states.p, sizeof(PatchState) * nlive, hipMemcpyDeviceToHost, stream));
    std::vector<std::vector<double>> taus(nlive);
    for (int k = 0; k < nlive; ++k) {
        taus[k].resize((size_t)descs[k].count * MAXP);
        HIP_TRY(hipMemcpyAsync(taus[k].data(), descs[k].tau, sizeof(double) * taus[k].size(), hipMemcpyDeviceToHost,
                               stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_kernel_ms = ms;
    for (int k = 0; k < nlive; ++k) {
        const int i = live[k];
        const RaslPlan& P = plans[i];
        const PatchState& s = out[k];
        tilt_rasl_result& r = res[i];
        const int N = P.rd.count;
        for (int j = 0; j < N; ++j) {
            const double* t = taus[k].data() + (size_t)j * MAXP;
            double Hn[9] = {t[0], t[1], t[2], t[3], t[4], t[5], 0.0, 0.0, 1.0};
            if (P.rd.d.model == TILT_PROJECTIVE) {
                Hn[6] = t[6];
                Hn[7] = t[7];
            }
            const double geo[3] = {P.geo[2 * j], P.geo[2 * j + 1], P.rd.d.s};
            denormalise_h(Hn, geo, r.tau + 9 * j);
        }
        r.objective = s.objective;
        r.outer_iters = s.outer;
        r.inner_iters_total = s.inner_total;
        r.svt_rank = s.svt_rank;
        r.status = s.status < 0 ? s.status : (s.warn ? TILT_WARN_MAXITER : TILT_OK);
        r.solve_ms = (double)(s.t_end - s.t_begin) / ctx->wall_rate_khz;
        r.counters.inner_iters = s.inner_total;
        r.counters.svt_calls = s.svt_calls;
        r.counters.jacobi_sweeps = s.sweeps;
        r.counters.jacobi_pairs = s.pairs;
        r.counters.jacobi_rotations = s.rotations;
        r.counters.recon_rows = s.recon_rows;
        worst = worse(worst, r.status);
    }
    return worst;
}
