// Host side of the C interface declared in include/tilt.h: argument
// validation, transform normalisation (FP64), request planning (pyramid
// levels, shapes, workspace layout), and the plain (step-by-step) and
// batched (fused persistent) drivers.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"

using namespace tilt;

namespace tilt {
namespace host {

hipError_t DevBuf::reserve(size_t need) {
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

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// Chunks per lane (and single floats after them) for rows of nr4 float4
// chunks in groups of lpp lanes.  With tails allowed, a two-row-block layout
// of 8 or 16 lanes whose last chunk would hold at most 2 real floats per lane
// keeps those as single floats instead (100 floats in 8 lanes: 3 chunks + 1
// float, 104 floats, instead of 4 chunks, 128).  The device instantiates
// these layouts for 1-3 chunks.
void split_row(int nr4, int bs, int lpp, bool tails, int* nch, int* tl) {
    *nch = (nr4 + lpp - 1) / lpp;
    *tl = 0;
    if (!tails || bs != 2 || (lpp != 8 && lpp != 16)) return;
    const int full = nr4 / lpp;
    const int rem = 4 * (nr4 - full * lpp);  // floats beyond the full chunks
    if (full < 1 || full > 3 || rem == 0) return;
    const int t = (rem + lpp - 1) / lpp;
    if (t <= 2) {
        *nch = full;
        *tl = t;
    }
}

// Jacobi layout for a matrix of nc rows of nr4 float4 chunks: rows per
// block (BS), lanes per block pair (LPP), chunks per lane (NCH) and single
// floats per lane (TL, only with tails: the one-workgroup SVT).  The
// model counts, per sweep, rounds x block pairs per lane group x the
// instructions of a round (BS^2 rotations of NCH chunks plus a fixed cost
// for the reduction and rotation parameters that grows with the reduction
// width, plus the row loads/stores), and divides by the number of
// concurrent groups' worth of issue slots when fewer groups than slots are
// busy.  The cheapest layout wins.
int pick_svt_cfg(int nc, int nr4, bool tails, double* cost_out = nullptr) {
    const int nc4 = (nc + 3) & ~3;
    int best = -1;
    double best_cost = 1e300;
    // Rows longer than 512 floats need groups of 32 or 64 lanes (the device
    // instantiates those layouts for exactly these chunk counts).
    const bool long_rows = nr4 > 16 * SVT_MAX_NCH;
    const int lpps[5] = {4, 8, 16, 32, 64};
    for (int bs = 1; bs <= 2; ++bs) {
        for (int li = long_rows ? 3 : 0; li < (long_rows ? 5 : 3); ++li) {
            if (long_rows && lpps[li] == 32 && bs == 2) continue;
            const int lpp = lpps[li];
            int nch, tl;
            split_row(nr4, bs, lpp, tails, &nch, &tl);
            if (nch > (bs == 1 ? SVT_MAX_NCH : 4)) continue;
            const int fl = 4 * nch + tl;  // floats per lane and row
            const int groups = NT / lpp;
            const int nb = nc4 / bs;
            const int pairs = nb / 2;
            const int per_group = (pairs + groups - 1) / groups;
            const int active = std::min(pairs, groups);
            const double rot = 5.0 * fl + 30.0 + 4.0 * li;
            const double round_instr = per_group * (bs * bs * rot + 1.0 * bs * fl) + 40.0;
            // waves with work per SIMD: issue-bound when >= 2, latency-bound below
            const double waves = std::max(1.0, active * (double)lpp / 64.0 / 4.0);
            const double round_cycles = round_instr * 4.0 * std::max(waves, 2.0) / (bs == 2 ? 1.5 : 1.0);
            // layouts whose rows exceed the register budget spill to scratch
            const bool spills = NT > 256 && ((bs == 2 && nch > 2) || (bs == 1 && lpp == 16 && nch > 5));
            const double cost = (nb - 1) * round_cycles * (spills ? 4.0 : 1.0);
            if (cost < best_cost) {
                best_cost = cost;
                best = svt_make_cfg(bs, lpp, nch, tl);
            }
        }
    }
    if (cost_out) *cost_out = best_cost;
    return best;
}

// LDS row stride: at least LPP*(4*NCH + TL) floats (every lane reads NCH
// chunks and TL single floats) and chosen so that the lane groups served by
// one 256-byte LDS pass (consecutive groups start BS rows apart) hit
// disjoint banks.
int pick_ld(int cfg) {
    const int bs = svt_bs(cfg), lpp = svt_lpp(cfg);
    const int min_ld = svt_span(cfg);
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

size_t lds_bytes_tiled(int sb, int ncp, int ld, int ldg, int tb, bool warm = false) {
    const size_t front = std::max((size_t)(warm ? 4 : 2) * sb * ld, (size_t)tb * ldg + (size_t)ncp * tb);
    return sizeof(float) * (front + 3 * (size_t)ncp);
}

// The whole matrix in LDS when it fits; otherwise the tiled Jacobi with the
// largest super-blocks whose staged pair fits (fewest block loads, most
// lane groups busy per round; the pairs examined per sweep, about ncp^2,
// do not depend on the block size).
// Measured layouts (autotuner): (nc, nr) -> (rows per block, lanes per
// pair).  A query uses the entry nearest in log(nc), log(nr) within a factor
// of 1.5 per axis, with the chunk count recomputed for its own row length;
// otherwise, or when that layout is not valid there, the cost model.
struct TuneEntry {
    int nc, nr, bs, lpp;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int tuned_cfg(int nc, int nr4, bool tails) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const TuneEntry* best = nullptr;
    double bd = 1e300;
    const double lc = std::log((double)nc), lr = std::log(4.0 * nr4);
    for (const auto& e : g_tune) {
        const double dc = std::log((double)e.nc) - lc, dr = std::log((double)e.nr) - lr;
        if (std::fabs(dc) > std::log(1.5) || std::fabs(dr) > std::log(1.5)) continue;
        const double d = dc * dc + dr * dr;
        if (d < bd) {
            bd = d;
            best = &e;
        }
    }
    if (!best) return -1;
    int nch, tl;
    split_row(nr4, best->bs, best->lpp, tails, &nch, &tl);
    if (nch > (best->bs == 1 ? SVT_MAX_NCH : 4)) return -1;
    return svt_make_cfg(best->bs, best->lpp, nch, tl);
}

// Layout of the one-workgroup SVT (single floats allowed).
int choose_svt_cfg(int nc, int nr4) {
    const int t = tuned_cfg(nc, nr4, true);
    return t >= 0 ? t : pick_svt_cfg(nc, nr4, true);
}

// Workgroups the tiled super-block size is planned for: kHelpPlan, or
// TILT_HELP_PLAN (1..16) from the environment, read once.
int help_plan() {
    static const int v = [] {
        const char* e = std::getenv("TILT_HELP_PLAN");
        const int k = e ? std::atoi(e) : 0;
        return k >= 1 && k <= 16 ? k : kHelpPlan;
    }();
    return v;
}

int shape_config(int m, int n, ShapeCfg* out, bool warm) {
    ShapeCfg c;
    c.colmajor = m >= n ? 1 : 0;
    c.nc = std::min(m, n);
    c.nr = std::max(m, n);
    c.ldg = (c.nr + 3) & ~3;
    c.sb = c.nsb = c.ncp = 0;
    c.warm_tb = 0;
    c.warm_lds = 0;
    const int nc4 = (c.nc + 3) & ~3;
    const size_t budget = (size_t)LDS_LIMIT - kStaticLdsMargin;
    if (nc4 <= SVT_MAX_ROWS) {
        c.cfg = choose_svt_cfg(c.nc, c.ldg / 4);
        if (c.cfg >= 0) {
            c.ld = pick_ld(c.cfg);
            for (int tb = 32; tb >= 16; tb -= 16) {
                c.tb = tb;
                c.lds = lds_bytes(c.nc, c.ld, c.tb);
                if (c.lds <= budget) {
                    c.ws_floats = (size_t)NPLANES * c.nc * c.ldg;
                    // warm start: the rotation rows share the layout of the
                    // Jacobi rows and need their own nc4 x ld LDS area
                    if (svt_nch(c.cfg) <= 4 && svt_lpp(c.cfg) <= 16) {
                        for (int wtb = 32; wtb >= 16; wtb -= 16) {
                            const size_t front = std::max((size_t)nc4 * c.ld, (size_t)wtb * c.ld + (size_t)nc4 * wtb);
                            const size_t wl = sizeof(float) * ((size_t)nc4 * c.ld + front + 3 * (size_t)nc4);
                            if (wl <= budget) {
                                c.warm_tb = wtb;
                                c.warm_lds = wl;
                                break;
                            }
                        }
                    }
                    *out = c;
                    // a warm-started solve whose rotation does not fit
                    // beside the rows takes the tiled layout when that one
                    // can carry the rotation (fewer sweeps per SVT than
                    // the cold SVT in LDS, and idle workgroups can help)
                    if (!warm || c.warm_lds > 0) return TILT_OK;
                    ShapeCfg t;
                    if (tiled_config(c, &t, true) == TILT_OK) *out = t;
                    return TILT_OK;
                }
            }
        }
    }
    return tiled_config(c, out);
}

// Tiled layout of a window (the fields set from the window's sides in c);
// need_warm: only layouts that can carry the rotation of the warm start.
int tiled_config(const ShapeCfg& c, ShapeCfg* out, bool need_warm) {
    const int nc4 = (c.nc + 3) & ~3;
    const size_t budget = (size_t)LDS_LIMIT - kStaticLdsMargin;
    if (c.nr > SVT_MAX_COLS) return TILT_ERR_TOO_LARGE;
    // Tiled: the super-block size is chosen for up to help_plan()
    // workgroups on one window (the fused kernel lets idle workgroups take
    // pairs of a round): the modelled time of a sweep is (rounds) x (pairs
    // per workgroup) x (one staged sweep over 2 sb rows, plus staging the
    // rows through LDS).  Ties within 10 % go to fewer super-blocks (fewer
    // rounds).  The choice fixes the arithmetic, so every path uses it.
    ShapeCfg best;
    double best_t = 1e300;
    bool found = false;
    for (int nsb = 2; nsb <= SVT_MAX_TILED_ROWS / 4; nsb += 2) {
        const int sb = (((nc4 + nsb - 1) / nsb) + 3) & ~3;
        if (2 * sb > SVT_MAX_ROWS) continue;
        if (sb < 4 || (nsb > 2 && ((nc4 + nsb - 3) / (nsb - 2) + 3 & ~3) == sb)) continue;  // same blocks, more rounds
        const int ncp = nsb * sb;
        if (ncp > SVT_MAX_TILED_ROWS) continue;  // rounding sb up to 4 rows: ncp is not monotonic in nsb
        double task = 0.0;
        const int cfg = pick_svt_cfg(2 * sb, c.ldg / 4, false, &task);
        if (cfg < 0) return TILT_ERR_TOO_LARGE;
        const int ld = pick_ld(cfg);
        task += 8.0 * (2.0 * sb) * (c.ldg / 4);  // staging both blocks in and out
        const int pairs = nsb / 2;
        const int members = std::min(pairs, help_plan());
        const double t = (nsb - 1) * (double)((pairs + members - 1) / members) * task;
        // warm start: the staged rotation rows double the staged pair
        // (chunks per lane up to 4, as in LDS)
        int wtb_fit = 0;
        size_t wl_fit = 0;
        if (svt_nch(cfg) <= 4 && svt_lpp(cfg) <= 16)
            for (int wtb = 32; wtb >= 16; wtb -= 16) {
                const size_t wl = lds_bytes_tiled(sb, ncp, ld, c.ldg, wtb, true);
                if (wl <= budget) {
                    wtb_fit = wtb;
                    wl_fit = wl;
                    break;
                }
            }
        if (need_warm && !wtb_fit) continue;
        for (int tb = 32; tb >= 16; tb -= 16) {
            const size_t lds = lds_bytes_tiled(sb, ncp, ld, c.ldg, tb);
            if (lds <= budget) {
                if (!found || t < 0.9 * best_t) {
                    best = c;
                    best.cfg = cfg;
                    best.ld = ld;
                    best.tb = tb;
                    best.sb = sb;
                    best.nsb = nsb;
                    best.ncp = ncp;
                    best.lds = lds;
                    best.ws_floats = (size_t)NPLANES * c.nc * c.ldg + 2 * (size_t)ncp * c.ldg;
                    best_t = t;
                    found = true;
                    best.warm_tb = wtb_fit;
                    best.warm_lds = wl_fit;
                }
                break;
            }
        }
    }
    if (!found) return TILT_ERR_TOO_LARGE;
    *out = best;
    return TILT_OK;
}

// Predicted relative cost of a solve (one-sided Jacobi work per iteration).
double predicted_cost(const PatchDesc& d) { return (double)d.nc * d.nc * d.nr; }

namespace {

bool finite9(const double* h) {
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(h[k])) return false;
    return true;
}

}  // namespace

// Pixel homography -> scaled coordinates of the window and the p entries of
// tau.  Affine transforms must have the last row (0, 0, 1).
int normalise_window(const double* Hpx, int m, int n, int model, double* geo, double* tau) {
    if (!finite9(Hpx) || Hpx[8] == 0.0) return TILT_ERR_ARG;
    double H[9];
    for (int k = 0; k < 9; ++k) H[k] = Hpx[k] / Hpx[8];
    const double scale = std::fabs(H[0]) + std::fabs(H[1]) + std::fabs(H[3]) + std::fabs(H[4]);
    if (model == TILT_AFFINE && (std::fabs(H[6]) > 1e-12 * (1.0 + scale) || std::fabs(H[7]) > 1e-12 * (1.0 + scale)))
        return TILT_ERR_ARG;
    double Hn[9];
    if (!normalise_h(H, m, n, geo, Hn)) return TILT_ERR_ARG;
    for (int k = 0; k < 6; ++k) tau[k] = Hn[k];
    tau[6] = model == TILT_PROJECTIVE ? Hn[6] : 0.0;
    tau[7] = model == TILT_PROJECTIVE ? Hn[7] : 0.0;
    return TILT_OK;
}

namespace {
thread_local char g_last_error[512] = "";
}  // namespace

int validate_params(const tilt_params* p) {
    if (!p) return TILT_ERR_ARG;
    if (!(p->eps1 > 0) || !(p->eps2 > 0) || !(p->eps_outer >= 0) || !(p->eps_obj >= 0)) return TILT_ERR_ARG;
    if (!(p->rho0 >= 1.0) || !(p->mu_max > 0)) return TILT_ERR_ARG;
    if (p->max_inner < 1 || p->max_outer < 1 || p->max_sweeps < 1) return TILT_ERR_ARG;
    if (!(p->jacobi_tol > 0.f) || !(p->jacobi_tol < 1.f)) return TILT_ERR_ARG;
    if (p->svt_mode < 0 || p->svt_mode > 4) return TILT_ERR_ARG;
    if (!(p->eps_svd >= 0) || !std::isfinite(p->eps_svd) || p->svdws_every < 0) return TILT_ERR_ARG;
    if (p->pyramid_levels < 0 || p->pyramid_levels > MAX_LEVELS) return TILT_ERR_ARG;
    if (p->graph_inner < 0 || p->graph_inner > 256) return TILT_ERR_ARG;
    if (!std::isfinite(p->lambda) || !std::isfinite(p->mu0)) return TILT_ERR_ARG;
    return TILT_OK;
}

int validate_problem(const tilt_problem* pr) {
    if (!pr || !pr->image) return TILT_ERR_ARG;
    if (pr->height < 2 || pr->width < 2 || pr->row_stride < pr->width) return TILT_ERR_ARG;
    if (pr->m < 2 || pr->n < 2) return TILT_ERR_ARG;
    if (pr->model != TILT_AFFINE && pr->model != TILT_PROJECTIVE) return TILT_ERR_ARG;
    double H[9];
    return initial_transform(*pr, H);
}

// The problem's initial pixel homography: tau0, or the map of the grid
// onto quad (init = 1).
int initial_transform(const tilt_problem& pr, double* H) {
    if (pr.init == 1) return tilt_tau_from_quad(pr.quad, pr.m, pr.n, pr.model, H);
    if (pr.init != 0 || !finite9(pr.tau0)) return TILT_ERR_ARG;
    for (int k = 0; k < 9; ++k) H[k] = pr.tau0[k];
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
    s.eps_obj = p->eps_obj;
    s.max_inner = p->max_inner;
    s.max_outer = p->max_outer;
    s.fixed_iters = p->fixed_iters ? 1 : 0;
    s.max_sweeps = p->max_sweeps;
    s.jacobi_tol = p->jacobi_tol;
    s.ns_every = 4;
    s.eps_svd = p->eps_svd;
    s.svdws_every = p->svdws_every;
    return s;
}

int record_hip_error(hipError_t e, const char* what, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%s) at line %d: %s", hipGetErrorName(e),
                  hipGetErrorString(e), line, what);
    return TILT_ERR_DEVICE;
}

const char* last_error_text() { return g_last_error; }

int worse(int a, int b) {
    // errors (negative) dominate warnings (positive) dominate OK
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

// Whether a window's SVT is warm-started: svt_mode >= 1 where the rotation
// fits beside the Jacobi rows (in LDS, or staged with them when tiled; the
// tiled warm start takes its start product in FP32 only).
bool warm_level(const tilt_params* prm, const ShapeCfg& sc) {
    return prm->svt_mode >= 1 && sc.warm_lds > 0 && (sc.sb == 0 || prm->svt_mode == 1);
}

// Workspace floats of one window: the solver planes (and the tiled working
// planes), plus the region of the SVD with warm start (svt_mode 4 on a
// window whose SVT is warm-started in LDS).
size_t level_ws_floats(const tilt_params* prm, const ShapeCfg& sc) {
    if (prm->svt_mode == 4 && warm_level(prm, sc) && sc.sb == 0)
        return (size_t)NPLANES * sc.nc * sc.ldg + svdws_region_words(sc.nr, sc.nc);
    return sc.ws_floats;
}

// Level l of a request: window ceil(m/2^l) x ceil(n/2^l) in an image of
// ceil(H/2^l) x ceil(W/2^l) pixels.  The workspace holds the solver planes
// (sized for the largest level) followed by the images of levels 1.. .
int plan_request(const tilt_problem& pr, const tilt_params* prm, float* A_out, float* E_out, RequestPlan* out) {
    int st = validate_problem(&pr);
    if (st != TILT_OK) return st;
    const int levels = std::max(1, prm->pyramid_levels);
    RequestPlan& P = *out;
    std::memset(&P, 0, sizeof(P));
    P.levels = levels;
    ShapeCfg sc[MAX_LEVELS];
    int hl[MAX_LEVELS], wl[MAX_LEVELS], ml[MAX_LEVELS], nl[MAX_LEVELS];
    size_t planes = 0;
    for (int l = 0; l < levels; ++l) {
        const int f = 1 << l;
        ml[l] = (pr.m + f - 1) / f;
        nl[l] = (pr.n + f - 1) / f;
        hl[l] = l == 0 ? pr.height : (hl[l - 1] + 1) / 2;
        wl[l] = l == 0 ? pr.width : (wl[l - 1] + 1) / 2;
        if (ml[l] < 2 || nl[l] < 2 || hl[l] < 2 || wl[l] < 2) return TILT_ERR_ARG;
        st = shape_config(ml[l], nl[l], &sc[l], prm->svt_mode == 1);
        if (st != TILT_OK) return st;
        planes = std::max(planes, level_ws_floats(prm, sc[l]));
        P.lds = std::max(P.lds, warm_level(prm, sc[l]) ? sc[l].warm_lds : sc[l].lds);
    }
    size_t off = (planes + 63) & ~(size_t)63;
    size_t img_off[MAX_LEVELS] = {0};
    for (int l = 1; l < levels; ++l) {
        img_off[l] = off;
        off += ((size_t)hl[l] * wl[l] + 63) & ~(size_t)63;
    }
    P.ws_floats = off;
    // initial transform at the coarsest level
    double H[9];
    st = initial_transform(pr, H);
    if (st != TILT_OK) return st;
    for (int l = 1; l < levels; ++l) to_coarser_h(H);
    PatchState& s0 = P.init;
    st = normalise_window(H, ml[levels - 1], nl[levels - 1], pr.model, s0.geo, s0.tau);
    if (st != TILT_OK) return st;
    for (int l = 0; l < levels; ++l) {
        PatchDesc& d = P.d[l];
        d.image = l == 0 ? pr.image : reinterpret_cast<const float*>(img_off[l] * sizeof(float));
        d.stride = l == 0 ? pr.row_stride : wl[l];
        d.H = hl[l];
        d.W = wl[l];
        d.m = ml[l];
        d.n = nl[l];
        d.model = pr.model;
        d.pp = pr.model - 3;
        d.nc = sc[l].nc;
        d.nr = sc[l].nr;
        d.ldg = sc[l].ldg;
        d.colmajor = sc[l].colmajor;
        d.ld = sc[l].ld;
        d.svt_cfg = sc[l].cfg;
        d.warm = warm_level(prm, sc[l]) ? prm->svt_mode : 0;
        d.tb = d.warm ? sc[l].warm_tb : sc[l].tb;
        d.sb = sc[l].sb;
        d.nsb = sc[l].nsb;
        d.ncp = sc[l].ncp;
        d.cx = s0.geo[0];
        d.cy = s0.geo[1];
        d.s = s0.geo[2];
        d.lam = prm->lambda > 0 ? prm->lambda : 1.0 / std::sqrt((double)std::max(ml[l], nl[l]));
        d.ws = nullptr;
        d.A_out = l == 0 ? A_out : nullptr;
        d.E_out = l == 0 ? E_out : nullptr;
    }
    return TILT_OK;
}

void rebase_plan(RequestPlan* plan, float* ws) {
    for (int l = 0; l < plan->levels; ++l) {
        PatchDesc& d = plan->d[l];
        d.ws = ws;
        if (l > 0) d.image = ws + reinterpret_cast<size_t>(d.image) / sizeof(float);
    }
}

void fill_result(const PatchDesc& d0, const PatchState& s, tilt_result* r, double rate_khz, long long t0) {
    r->solve_ms = (double)(s.t_end - s.t_begin) / rate_khz;
    r->done_ms = (double)(s.t_end - t0) / rate_khz;
    double Hn[9] = {s.tau[0], s.tau[1], s.tau[2], s.tau[3], s.tau[4], s.tau[5], 0.0, 0.0, 1.0};
    if (d0.model == TILT_PROJECTIVE) {
        Hn[6] = s.tau[6];
        Hn[7] = s.tau[7];
    }
    denormalise_h(Hn, s.geo, r->tau);
    r->outer_iters = s.outer;
    r->inner_iters_total = s.inner_total;
    r->svt_rank = s.svt_rank;
    r->rank = s.num_rank;
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
    r->counters.svdws_steps = s.svdws_steps;
}

// Whether idle workgroups of the fused and serving kernels help windows
// beyond LDS with their Jacobi rounds: on unless TILT_HELPERS=0 in the
// environment.  Only who runs which super-block pair depends on it, not the
// results.
bool helpers_enabled() {
    const char* e = std::getenv("TILT_HELPERS");
    return !(e && e[0] == '0');
}

}  // namespace host
}  // namespace tilt

using namespace tilt::host;

namespace {

struct Prepared {
    int levels = 1;
    std::vector<RequestPlan> plans;
    std::vector<int> status;  // per-problem preparation status
    size_t max_lds = 0;
    size_t ws_floats = 0;
};

// Plan every problem; images and A/E outputs are device pointers.
int prepare(const tilt_problem* probs, int count, const tilt_params* prm, tilt_result* results, Prepared* P) {
    P->levels = std::max(1, prm->pyramid_levels);
    P->plans.resize(count);
    P->status.assign(count, TILT_OK);
    int worst = TILT_OK;
    for (int i = 0; i < count; ++i) {
        const int st = plan_request(probs[i], prm, results ? results[i].A : nullptr, results ? results[i].E : nullptr,
                                    &P->plans[i]);
        P->status[i] = st;
        worst = worse(worst, st);
    }
    return worst;
}

// Device descriptors (levels per request, request-major), states and
// workspace for the live requests.
int upload(tilt_ctx* ctx, const Prepared& P, const std::vector<int>& live, std::vector<RequestPlan>* plans,
           hipStream_t stream) {
    const int count = (int)live.size();
    const int L = P.levels;
    size_t total = 0;
    std::vector<size_t> off(count);
    for (int k = 0; k < count; ++k) {
        off[k] = total;
        total += (P.plans[live[k]].ws_floats + 63) & ~(size_t)63;
    }
    if (total * sizeof(float) > ctx->budget) return TILT_ERR_NOMEM;
    if (ctx->ws.reserve(std::max<size_t>(total * sizeof(float), 256)) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->descs.reserve(sizeof(PatchDesc) * L * count) != hipSuccess) return TILT_ERR_NOMEM;
    if (ctx->states.reserve(sizeof(PatchState) * count) != hipSuccess) return TILT_ERR_NOMEM;
    float* base = reinterpret_cast<float*>(ctx->ws.p);
    std::vector<PatchDesc> descs((size_t)L * count);
    std::vector<PatchState> states(count);
    plans->resize(count);
    for (int k = 0; k < count; ++k) {
        RequestPlan pl = P.plans[live[k]];
        rebase_plan(&pl, base + off[k]);
        for (int l = 0; l < L; ++l) descs[(size_t)k * L + l] = pl.d[l];
        states[k] = pl.init;
        (*plans)[k] = pl;
    }
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(PatchDesc) * L * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, states.data(), sizeof(PatchState) * count, hipMemcpyHostToDevice, stream));
    return TILT_OK;
}

// Captured inner iterations: graph_k x (SVT, update) of one level.
struct InnerGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    ~InnerGraph() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
    }
};

int capture_inner(InnerGraph* G, const PatchDesc* d, PatchState* ds, const SolverParams& sp, size_t lds, int graph_k,
                  hipStream_t stream) {
    // One eager iteration first: it configures the kernel's LDS attribute
    // outside the capture and is an ordinary inner iteration.
    HIP_TRY(launch_svt(d, ds, sp, lds, stream));
    HIP_TRY(launch_update(d, ds, sp, stream));
    HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < graph_k; ++i) {
        hipError_t e = launch_svt(d, ds, sp, lds, stream, false);
        if (e == hipSuccess) e = launch_update(d, ds, sp, stream);
        if (e != hipSuccess) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            return record_hip_error(e, "capture of inner iterations", __LINE__);
        }
    }
    HIP_TRY(hipStreamEndCapture(stream, &G->g));
    HIP_TRY(hipGraphInstantiate(&G->ge, G->g, nullptr, nullptr, 0));
    return TILT_OK;
}

// Host-driven loop over the step kernels for request k (mirrors
// solve_request on the device: pyramid, then levels coarse to fine).  With
// graph_k > 0 the inner iterations run as replays of a captured graph of
// graph_k iterations (one stop-flag read per replay); the first inner
// iteration of each inner loop is launched eagerly.
// A level whose SVT does not fit LDS runs each Jacobi round's super-block
// pairs on separate workgroups (the wide kernels, same tiling, same bits as
// the one-workgroup tiled Jacobi): the host launches one kernel per round
// and reads the rotation flag after each sweep.  The decomposition of I for
// mu_0 goes the same way.  Such levels are never captured into graphs.
int run_plain_request(tilt_ctx* ctx, size_t lds, const SolverParams& sp, int L, int k, hipStream_t stream,
                      int graph_k, const RequestPlan& plan) {
    const PatchDesc* dl = reinterpret_cast<const PatchDesc*>(ctx->descs.p) + (size_t)k * L;
    PatchState* ds = reinterpret_cast<PatchState*>(ctx->states.p) + k;
    PatchState hs;
    auto fetch = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(&hs, ds, sizeof(PatchState), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return TILT_OK;
    };
    // [active list {0}, rotation flag, sweep count] for the wide kernels
    if (ctx->queue.reserve(256) != hipSuccess) return TILT_ERR_NOMEM;
    int* d_ints = reinterpret_cast<int*>(ctx->queue.p);
    HIP_TRY(hipMemsetAsync(d_ints, 0, 3 * sizeof(int), stream));
    bool configured = false;
    auto wide_svd = [&](const PatchDesc* d, const PatchDesc& hd, int form_m) -> int {
        HIP_TRY(launch_wide_stage(d, ds, d_ints, 1, form_m, d_ints + 1, stream));
        const size_t lr = sizeof(float) * 2 * (size_t)hd.sb * hd.ld;
        int sweeps = 0, flag = 1;
        for (int sw = 0; sw < sp.max_sweeps && flag; ++sw) {
            for (int r = 0; r < hd.nsb - 1; ++r) {
                HIP_TRY(launch_wide_round(d, ds, d_ints, 1, hd.nsb / 2, r, sp.jacobi_tol, form_m ? sp.eps2 : 0.0,
                                          d_ints + 1, lr, !configured, stream));
                configured = true;
            }
            HIP_TRY(hipMemcpyAsync(&flag, d_ints + 1, sizeof(int), hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            HIP_TRY(hipMemsetAsync(d_ints + 1, 0, sizeof(int), stream));
            ++sweeps;
        }
        HIP_TRY(hipMemcpyAsync(d_ints + 2, &sweeps, sizeof(int), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return TILT_OK;
    };
    HIP_TRY(launch_level_begin(dl + L - 1, ds, 1, stream));
    if (L > 1) HIP_TRY(launch_pyramid_build(dl, L, stream));
    for (int l = L - 1; l >= 0; --l) {
        const PatchDesc* d = dl + l;
        const PatchDesc& hd = plan.d[l];
        const bool wide = hd.sb > 0 && !hd.warm;
        SolverParams sp_setup = sp;
        if (wide && !(sp_setup.mu0 > 0.0)) sp_setup.mu0 = 1.0;  // mu_0 from the wide decomposition of I
        if (l < L - 1) {
            if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            if (hs.status < 0) break;
            HIP_TRY(launch_level_begin(d, ds, 0, stream));
            if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            if (hs.status < 0) break;
        }
        InnerGraph graph;
        for (;;) {
            HIP_TRY(launch_setup(d, ds, sp_setup, lds, stream));
            if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            if (hs.status < 0) break;
            if (wide && !(sp.mu0 > 0.0)) {
                const int w = wide_svd(d, hd, 0);
                if (w != TILT_OK) return w;
                HIP_TRY(launch_wide_finish(d, ds, d_ints, 1, sp, d_ints + 2, 1, lds, stream));
                if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
                if (hs.status < 0) break;
            }
            if (!wide && graph_k > 0 && !graph.ge) {
                const int c = capture_inner(&graph, d, ds, sp, lds, graph_k, stream);
                if (c != TILT_OK) return c;
                if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            }
            while (!hs.done_inner) {
                if (wide) {
                    const int w = wide_svd(d, hd, 1);
                    if (w != TILT_OK) return w;
                    HIP_TRY(launch_wide_finish(d, ds, d_ints, 1, sp, d_ints + 2, 0, lds, stream));
                    HIP_TRY(launch_update(d, ds, sp, stream));
                } else if (graph.ge) {
                    HIP_TRY(hipGraphLaunch(graph.ge, stream));
                } else {
                    HIP_TRY(launch_svt(d, ds, sp, lds, stream));
                    HIP_TRY(launch_update(d, ds, sp, stream));
                }
                if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            }
            if (hs.status < 0) break;
            HIP_TRY(launch_dtau(d, ds, sp, stream));
            if (fetch() != TILT_OK) return TILT_ERR_DEVICE;
            if (hs.done_outer) break;
        }
        HIP_TRY(launch_finalize(d, ds, 0, stream));
    }
    HIP_TRY(launch_mark_end(ds, stream));
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
    int worst = prepare(probs, count, prm, results, &P);
    // Only valid problems are sent to the device.
    std::vector<int> live;
    size_t max_lds = 0;
    for (int i = 0; i < count; ++i)
        if (P.status[i] == TILT_OK) {
            live.push_back(i);
            max_lds = std::max(max_lds, P.plans[i].lds);
        }
    if (!live.empty()) {
        std::vector<RequestPlan> plans;
        int u = upload(ctx, P, live, &plans, stream);
        if (u != TILT_OK) return u;
        const SolverParams sp = to_solver(prm);
        const int nlive = (int)live.size();
        const int L = P.levels;
        if (plain) {
            hipStream_t ps = stream;
            hipStream_t own = nullptr;
            if (prm->graph_inner > 0) {
                // capture needs a stream of our own (not the legacy default stream)
                HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
                HIP_TRY(hipEventRecord(ctx->ev0, stream));
                HIP_TRY(hipStreamWaitEvent(own, ctx->ev0, 0));
                ps = own;
            }
            int r = TILT_OK;
            for (int k = 0; k < nlive && r == TILT_OK; ++k)
                r = run_plain_request(ctx, max_lds, sp, L, k, ps, prm->graph_inner, plans[k]);
            if (own) {
                (void)hipEventRecord(ctx->ev1, own);
                (void)hipStreamWaitEvent(stream, ctx->ev1, 0);
                (void)hipStreamSynchronize(own);
                (void)hipStreamDestroy(own);
            }
            if (r != TILT_OK) return r;
        } else {
            // Control blocks: the queue and, for requests with a level whose
            // SVT is tiled, the block through which idle workgroups help.
            const size_t fc_bytes = (sizeof(FusedCtl) + 255) & ~(size_t)255;
            if (ctx->queue.reserve(fc_bytes + sizeof(GangCtl) * nlive) != hipSuccess) return TILT_ERR_NOMEM;
            FusedCtl* dfc = reinterpret_cast<FusedCtl*>(ctx->queue.p);
            GangCtl* dgang = reinterpret_cast<GangCtl*>(reinterpret_cast<char*>(ctx->queue.p) + fc_bytes);
            std::vector<char> blob(fc_bytes + sizeof(GangCtl) * nlive, 0);
            FusedCtl* hfc = reinterpret_cast<FusedCtl*>(blob.data());
            GangCtl* hgang = reinterpret_cast<GangCtl*>(blob.data() + fc_bytes);
            hfc->remaining = nlive;
            hfc->gangs = dgang;
            bool any_tiled = false;
            for (int k = 0; k < nlive; ++k) {
                hgang[k].slot = -1;
                hgang[k].fc = dfc;
                bool tiled = false;
                for (int l = 0; l < L; ++l) tiled |= plans[k].d[l].sb > 0;
                if (tiled && helpers_enabled())
                    for (int l = 0; l < L; ++l) plans[k].d[l].gang = dgang + k;
                any_tiled |= tiled;
            }
            HIP_TRY(hipMemcpyAsync(ctx->queue.p, blob.data(), blob.size(), hipMemcpyHostToDevice, stream));
            if (any_tiled && helpers_enabled()) {
                std::vector<PatchDesc> descs((size_t)L * nlive);
                for (int k = 0; k < nlive; ++k)
                    for (int l = 0; l < L; ++l) descs[(size_t)k * L + l] = plans[k].d[l];
                HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(PatchDesc) * L * nlive,
                                       hipMemcpyHostToDevice, stream));
            }
            if (ctx->order.reserve(sizeof(int) * nlive) != hipSuccess) return TILT_ERR_NOMEM;
            // longest predicted solve first (stable: equal shapes keep their order)
            std::vector<int> order(nlive);
            for (int k = 0; k < nlive; ++k) order[k] = k;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                return predicted_cost(plans[a].d[0]) > predicted_cost(plans[b].d[0]);
            });
            HIP_TRY(hipMemcpyAsync(ctx->order.p, order.data(), sizeof(int) * nlive, hipMemcpyHostToDevice, stream));
            const int per_cu = std::max<int>(1, (int)(LDS_LIMIT / (max_lds + kStaticLdsMargin)));
            const int grid = std::max(1, std::min(nlive, ctx->num_cus * std::min(per_cu, 2)));
            HIP_TRY(hipEventRecord(ctx->ev0, stream));
            HIP_TRY(launch_fused(reinterpret_cast<const PatchDesc*>(ctx->descs.p),
                                 reinterpret_cast<PatchState*>(ctx->states.p), sp, nlive, L,
                                 reinterpret_cast<const int*>(ctx->order.p), dfc,
                                 (any_tiled && helpers_enabled()) ? 1 : 0, grid, max_lds, stream));
            HIP_TRY(hipEventRecord(ctx->ev1, stream));
            ctx->live_count.store(nlive);
            ctx->live_fc.store(dfc);
        }
        std::vector<PatchState> out(nlive);
        HIP_TRY(hipMemcpyAsync(out.data(), ctx->states.p, sizeof(PatchState) * nlive, hipMemcpyDeviceToHost,
                               stream));
        const hipError_t se = hipStreamSynchronize(stream);
        ctx->live_fc.store(nullptr);
        HIP_TRY(se);
        if (!plain) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            ctx->last_kernel_ms = ms;
        }
        long long t0 = out[0].t_begin;
        for (int k = 1; k < nlive; ++k) t0 = std::min(t0, out[k].t_begin);
        for (int k = 0; k < nlive; ++k) {
            const int i = live[k];
            fill_result(plans[k].d[0], out[k], &results[i], ctx->wall_rate_khz, t0);
            worst = worse(worst, results[i].status);
        }
    }
    for (int i = 0; i < count; ++i)
        if (P.status[i] != TILT_OK) results[i].status = P.status[i];
    return worst;
}

}  // namespace

// ---------------------------------------------------------------------------
// Wide inner-loop path: a few large problems (tiled SVT shapes) run their
// Jacobi rounds on many workgroups, one launch per round, host-driven.
// ---------------------------------------------------------------------------

namespace {

struct WideTiling {
    int sb = 0, nsb = 0, ncp = 0, cfg = -1, ld = 0, tb = 0;
    size_t lds_round = 0, lds_finish = 0;
};

// Largest super-blocks whose staged pair is swept in one pass of the lane
// groups per round (block pairs <= groups) and whose LDS needs fit; the
// rounds then take about the same time whatever the size, so larger blocks
// mean fewer launches and fewer staged rows.
bool wide_tiling(int nc, int ldg, WideTiling* out) {
    const int nc4 = (nc + 3) & ~3;
    const size_t budget = (size_t)LDS_LIMIT - kStaticLdsMargin;
    for (int sb = std::min(128, ((nc4 / 2) + 3) & ~3); sb >= 4; sb -= 4) {
        const int cfg = pick_svt_cfg(2 * sb, ldg / 4, false);
        if (cfg < 0) continue;
        if (sb / svt_bs(cfg) > NT / svt_lpp(cfg)) continue;
        int nsb = (nc4 + sb - 1) / sb;
        nsb += nsb & 1;
        if (nsb < 2 || nsb * sb > SVT_MAX_TILED_ROWS) continue;
        const int ld = pick_ld(cfg);
        const size_t lr = sizeof(float) * 2 * (size_t)sb * ld;
        if (lr > budget) continue;
        for (int tb = 32; tb >= 16; tb -= 16) {
            const size_t lf = lds_bytes_tiled(sb, nsb * sb, ld, ldg, tb);
            if (lf <= budget) {
                out->sb = sb;
                out->nsb = nsb;
                out->ncp = nsb * sb;
                out->cfg = cfg;
                out->ld = ld;
                out->tb = tb;
                out->lds_round = lr;
                out->lds_finish = lf;
                return true;
            }
        }
    }
    return false;
}

int inner_wide(tilt_ctx* ctx, const float* I, const float* J, int count, int m, int n, int p, const tilt_params* prm,
               float* A, float* E, tilt_result* results, hipStream_t stream, const ShapeCfg& sc,
               const WideTiling& wt) {
    const size_t per = (((size_t)NPLANES * sc.nc * sc.ldg + (size_t)wt.ncp * sc.ldg) + 63) & ~(size_t)63;
    if (per * count * sizeof(float) > ctx->budget) return TILT_ERR_NOMEM;
    if (ctx->ws.reserve(per * count * sizeof(float)) != hipSuccess ||
        ctx->descs.reserve(sizeof(PatchDesc) * count) != hipSuccess ||
        ctx->states.reserve(sizeof(PatchState) * count) != hipSuccess ||
        ctx->scratch.reserve(sizeof(int) * 4 * (size_t)count) != hipSuccess)
        return TILT_ERR_NOMEM;
    int* d_active = reinterpret_cast<int*>(ctx->scratch.p);
    int* d_cur = d_active + count;
    int* d_flags = d_cur + count;
    int* d_sweeps = d_flags + count;
    const size_t mn = (size_t)m * n;
    std::vector<PatchDesc> descs(count);
    std::vector<PatchState> hs(count);
    for (int i = 0; i < count; ++i) {
        PatchDesc& d = descs[i];
        std::memset(&d, 0, sizeof(d));
        d.m = m;
        d.n = n;
        d.model = p + 3;
        d.pp = p;
        d.nc = sc.nc;
        d.nr = sc.nr;
        d.ldg = sc.ldg;
        d.colmajor = sc.colmajor;
        d.ld = wt.ld;
        d.svt_cfg = wt.cfg;
        d.tb = wt.tb;
        d.sb = wt.sb;
        d.nsb = wt.nsb;
        d.ncp = wt.ncp;
        d.s = 1.0;
        d.lam = prm->lambda > 0 ? prm->lambda : 1.0 / std::sqrt((double)std::max(m, n));
        d.ws = reinterpret_cast<float*>(ctx->ws.p) + per * i;
        d.A_out = A ? A + mn * i : nullptr;
        d.E_out = E ? E + mn * i : nullptr;
        std::memset(&hs[i], 0, sizeof(PatchState));
        hs[i].geo[2] = 1.0;
    }
    const PatchDesc* dd = reinterpret_cast<const PatchDesc*>(ctx->descs.p);
    PatchState* ds = reinterpret_cast<PatchState*>(ctx->states.p);
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(PatchDesc) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, hs.data(), sizeof(PatchState) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemsetAsync(ctx->scratch.p, 0, sizeof(int) * 4 * (size_t)count, stream));
    const SolverParams sp = to_solver(prm);
    SolverParams sp_setup = sp;
    if (!(sp_setup.mu0 > 0.0)) sp_setup.mu0 = 1.0;  // set below from the wide SVD of I
    HIP_TRY(hipEventRecord(ctx->ev0, stream));
    HIP_TRY(launch_wide_setup(dd, ds, sp_setup, I, J, count, 0, stream));
    auto read_states = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(hs.data(), ctx->states.p, sizeof(PatchState) * count, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return TILT_OK;
    };
    int st = read_states();
    if (st != TILT_OK) return st;
    std::vector<int> active;
    for (int i = 0; i < count; ++i)
        if (hs[i].status >= 0) active.push_back(i);
    std::vector<int> sweeps(count, 0), flags(count, 0);
    bool configured = false;
    // Stage, then sweep until a sweep rotates nothing (per problem), then
    // upload the sweep counts.
    auto wide_svd = [&](const std::vector<int>& act, int form_m) -> int {
        HIP_TRY(hipMemcpyAsync(d_active, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice, stream));
        HIP_TRY(launch_wide_stage(dd, ds, d_active, (int)act.size(), form_m, d_flags, stream));
        for (int i : act) sweeps[i] = 0;
        std::vector<int> cur = act;
        for (int sw = 0; sw < prm->max_sweeps && !cur.empty(); ++sw) {
            HIP_TRY(hipMemcpyAsync(d_cur, cur.data(), sizeof(int) * cur.size(), hipMemcpyHostToDevice, stream));
            for (int r = 0; r < wt.nsb - 1; ++r) {
                HIP_TRY(launch_wide_round(dd, ds, d_cur, (int)cur.size(), wt.nsb / 2, r, sp.jacobi_tol,
                                          form_m ? sp.eps2 : 0.0, d_flags, wt.lds_round, !configured, stream));
                configured = true;
            }
            HIP_TRY(hipMemcpyAsync(flags.data(), d_flags, sizeof(int) * count, hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            HIP_TRY(hipMemsetAsync(d_flags, 0, sizeof(int) * count, stream));
            std::vector<int> next;
            for (int i : cur) {
                sweeps[i] += 1;
                if (flags[i]) next.push_back(i);
            }
            cur.swap(next);
        }
        HIP_TRY(hipMemcpyAsync(d_sweeps, sweeps.data(), sizeof(int) * count, hipMemcpyHostToDevice, stream));
        return TILT_OK;
    };
    if (!active.empty() && !(sp.mu0 > 0.0)) {
        st = wide_svd(active, 0);
        if (st != TILT_OK) return st;
        HIP_TRY(launch_wide_finish(dd, ds, d_active, (int)active.size(), sp, d_sweeps, 1, wt.lds_finish, stream));
        st = read_states();
        if (st != TILT_OK) return st;
        std::vector<int> ok;
        for (int i : active)
            if (hs[i].status >= 0) ok.push_back(i);
        active.swap(ok);
    }
    // Every pass raises each active problem's inner count by one, and
    // dev_update stops a problem at max_inner, so the loop ends.
    while (!active.empty()) {
        st = wide_svd(active, 1);
        if (st != TILT_OK) return st;
        HIP_TRY(launch_wide_finish(dd, ds, d_active, (int)active.size(), sp, d_sweeps, 0, wt.lds_finish, stream));
        HIP_TRY(launch_wide_update(dd, ds, d_active, (int)active.size(), sp, stream));
        st = read_states();
        if (st != TILT_OK) return st;
        std::vector<int> next;
        for (int i : active)
            if (!hs[i].done_inner && hs[i].status >= 0) next.push_back(i);
        active.swap(next);
    }
    HIP_TRY(launch_wide_end(dd, ds, count, stream));
    HIP_TRY(hipEventRecord(ctx->ev1, stream));
    st = read_states();
    if (st != TILT_OK) return st;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_kernel_ms = ms;
    int worst = TILT_OK;
    long long t0 = hs[0].t_begin;
    for (int i = 1; i < count; ++i) t0 = std::min(t0, hs[i].t_begin);
    for (int i = 0; i < count; ++i) {
        tilt_result& r = results[i];
        float* hA = r.A;
        float* hE = r.E;
        fill_result(descs[i], hs[i], &r, ctx->wall_rate_khz, t0);
        for (int k = 0; k < 9; ++k) r.tau[k] = 0.0;
        r.A = hA;
        r.E = hE;
        worst = worse(worst, r.status);
    }
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
    p->pyramid_levels = 1;
    p->eps_obj = 0.0;
    p->eps_svd = 1e-3;
    p->svdws_every = 0;
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

const char* tilt_last_error(void) { return tilt::host::last_error_text(); }

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
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
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
    if (ctx->serve) serve_release(ctx->serve);
    ctx->serve = nullptr;
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
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return TILT_OK;
}

int tilt_ctx_progress(tilt_ctx* ctx, int* finished, int* total) {
    if (!ctx || !finished || !total) return TILT_ERR_ARG;
    *finished = 0;
    *total = 0;
    void* fc = ctx->live_fc.load();
    if (!fc) return TILT_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!ctx->side) HIP_TRY(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    if (!ctx->pinned) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), sizeof(int)));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, reinterpret_cast<char*>(fc) + offsetof(FusedCtl, remaining), sizeof(int),
                           hipMemcpyDeviceToHost, ctx->side));
    HIP_TRY(hipStreamSynchronize(ctx->side));
    const int n = ctx->live_count.load();
    *total = n;
    *finished = std::max(0, std::min(n, n - *ctx->pinned));
    return TILT_OK;
}

int tilt_ctx_last_kernel_ms(tilt_ctx* ctx, double* ms) {
    if (!ctx || !ms) return TILT_ERR_ARG;
    *ms = ctx->last_kernel_ms;
    return TILT_OK;
}

size_t tilt_workspace_bytes(const tilt_problem* prob) {
    if (!prob) return 0;
    // the larger of the cold and the warm-started layout (svt_mode 0-3)
    ShapeCfg sc{}, sw{};
    if (shape_config(prob->m, prob->n, &sc) != TILT_OK || shape_config(prob->m, prob->n, &sw, true) != TILT_OK)
        return 0;
    return std::max(sc.ws_floats, sw.ws_floats) * sizeof(float) + sizeof(PatchDesc) + sizeof(PatchState);
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
        double geo[3], tau0n[MAXP], H0[9];
        st = initial_transform(pr, H0);
        if (st != TILT_OK) return st;
        st = normalise_window(H0, m, n, model, geo, tau0n);
        if (st != TILT_OK) return st;
        // The transform being evaluated, expressed in the window's scaled
        // coordinates (centre = image of the grid centre under tau0).
        double H[9];
        for (int k = 0; k < 9; ++k) H[k] = taus[9 * i + k];
        if (!std::isfinite(H[0] + H[1] + H[2] + H[3] + H[4] + H[5] + H[6] + H[7] + H[8]) || H[8] == 0.0)
            return TILT_ERR_ARG;
        for (int k = 0; k < 9; ++k) H[k] /= taus[9 * i + 8];
        const double s = geo[2];
        double Hn[9];
        for (int j = 0; j < 3; ++j) {
            const double sc = (j < 2) ? s : 1.0;
            Hn[0 * 3 + j] = (H[0 * 3 + j] - geo[0] * H[2 * 3 + j]) / s * sc;
            Hn[1 * 3 + j] = (H[1 * 3 + j] - geo[1] * H[2 * 3 + j]) / s * sc;
            Hn[2 * 3 + j] = H[2 * 3 + j] * sc;
        }
        const double h22n = Hn[8];
        for (int k = 0; k < 9; ++k) Hn[k] /= h22n;
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
        d.cx = geo[0];
        d.cy = geo[1];
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
        ctx->states.reserve(sizeof(PatchState) * count) != hipSuccess ||
        ctx->scratch.reserve(sizeof(double) * (1 + MAXP) * STEP1_SLICES * (size_t)count) != hipSuccess)
        return TILT_ERR_NOMEM;
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(PatchDesc) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, states.data(), sizeof(PatchState) * count, hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(launch_step1(reinterpret_cast<const PatchDesc*>(ctx->descs.p),
                         reinterpret_cast<PatchState*>(ctx->states.p), count,
                         reinterpret_cast<double*>(ctx->scratch.p), I_out, J_out, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return TILT_OK;
}

int tilt_pyramid(tilt_ctx* ctx, const float* image, int height, int width, long long row_stride, float* out,
                 int levels, void* hip_stream) {
    if (!ctx || !image || !out || height < 2 || width < 2 || row_stride < width) return TILT_ERR_ARG;
    if (levels < 2 || levels > MAX_LEVELS) return TILT_ERR_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(launch_pyramid_jobs(image, height, width, row_stride, out, levels, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return TILT_OK;
}

int tilt_inner_batch(tilt_ctx* ctx, const float* I, const float* J, int count, int m, int n, int p,
                     const tilt_params* prm_in, float* A, float* E, tilt_result* results, void* hip_stream) {
    if (!ctx || !I || !J || !prm_in || !results || count < 0 || m < 2 || n < 2 || p < 1 || p > MAXPP)
        return TILT_ERR_ARG;
    int st = validate_params(prm_in);
    if (st != TILT_OK) return st;
    const tilt_params* prm = prm_in;
    if (prm->pyramid_levels > 1) return TILT_ERR_ARG;
    if (count == 0) return TILT_OK;
    ShapeCfg sc{};
    st = shape_config(m, n, &sc);
    if (st != TILT_OK) return st;
    const bool warm = prm->svt_mode >= 1 && sc.warm_lds > 0 && sc.sb == 0;
    const size_t lds = warm ? sc.warm_lds : sc.lds;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    // Few problems whose SVT does not fit LDS: spread each Jacobi round over
    // workgroups instead of one workgroup per problem.
    WideTiling wt;
    if (sc.sb > 0 && !warm && count * 8 <= ctx->num_cus && wide_tiling(sc.nc, sc.ldg, &wt))
        return inner_wide(ctx, I, J, count, m, n, p, prm, A, E, results, stream, sc, wt);
    const size_t per = (level_ws_floats(prm, sc) + 63) & ~(size_t)63;
    if (per * count * sizeof(float) > ctx->budget) return TILT_ERR_NOMEM;
    if (ctx->ws.reserve(per * count * sizeof(float)) != hipSuccess ||
        ctx->descs.reserve(sizeof(PatchDesc) * count) != hipSuccess ||
        ctx->states.reserve(sizeof(PatchState) * count) != hipSuccess)
        return TILT_ERR_NOMEM;
    const size_t mn = (size_t)m * n;
    std::vector<PatchDesc> descs(count);
    std::vector<PatchState> states(count);
    for (int i = 0; i < count; ++i) {
        PatchDesc& d = descs[i];
        std::memset(&d, 0, sizeof(d));
        d.m = m;
        d.n = n;
        d.model = p + 3;
        d.pp = p;
        d.nc = sc.nc;
        d.nr = sc.nr;
        d.ldg = sc.ldg;
        d.colmajor = sc.colmajor;
        d.ld = sc.ld;
        d.svt_cfg = sc.cfg;
        d.warm = warm ? prm->svt_mode : 0;
        d.tb = warm ? sc.warm_tb : sc.tb;
        d.sb = sc.sb;
        d.nsb = sc.nsb;
        d.ncp = sc.ncp;
        d.s = 1.0;
        d.lam = prm->lambda > 0 ? prm->lambda : 1.0 / std::sqrt((double)std::max(m, n));
        d.ws = reinterpret_cast<float*>(ctx->ws.p) + per * i;
        d.A_out = A ? A + mn * i : nullptr;
        d.E_out = E ? E + mn * i : nullptr;
        std::memset(&states[i], 0, sizeof(PatchState));
        states[i].geo[2] = 1.0;
    }
    HIP_TRY(hipMemcpyAsync(ctx->descs.p, descs.data(), sizeof(PatchDesc) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ctx->states.p, states.data(), sizeof(PatchState) * count, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(ctx->ev0, stream));
    HIP_TRY(launch_inner(reinterpret_cast<const PatchDesc*>(ctx->descs.p), reinterpret_cast<PatchState*>(ctx->states.p),
                         to_solver(prm), I, J, count, lds, stream));
    HIP_TRY(hipEventRecord(ctx->ev1, stream));
    HIP_TRY(hipMemcpyAsync(states.data(), ctx->states.p, sizeof(PatchState) * count, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_kernel_ms = ms;
    int worst = TILT_OK;
    long long t0 = states[0].t_begin;
    for (int i = 1; i < count; ++i) t0 = std::min(t0, states[i].t_begin);
    for (int i = 0; i < count; ++i) {
        tilt_result& r = results[i];
        float* hA = r.A;
        float* hE = r.E;
        fill_result(descs[i], states[i], &r, ctx->wall_rate_khz, t0);
        for (int k = 0; k < 9; ++k) r.tau[k] = 0.0;
        r.A = hA;
        r.E = hE;
        worst = worse(worst, r.status);
    }
    return worst;
}

int tilt_svt_layouts(int m, int n, int* bs, int* lpp, int max_count) {
    if (m < 1 || n < 1 || !bs || !lpp || max_count < 0) return TILT_ERR_ARG;
    const int nc = std::min(m, n), nr4 = (std::max(m, n) + 3) / 4;
    ShapeCfg sc{};
    if (shape_config(m, n, &sc) != TILT_OK || sc.sb > 0) return 0;  // tiled: not tunable here
    const size_t budget = (size_t)LDS_LIMIT - kStaticLdsMargin;
    int k = 0;
    const int lpps[3] = {4, 8, 16};
    for (int b = 1; b <= 2; ++b)
        for (int li = 0; li < 3; ++li) {
            const int nch = (nr4 + lpps[li] - 1) / lpps[li];
            if (nch > (b == 1 ? SVT_MAX_NCH : 4)) continue;
            const int ld = pick_ld(svt_make_cfg(b, lpps[li], nch));
            if (lds_bytes(nc, ld, 16) > budget) continue;
            if (k < max_count) {
                bs[k] = b;
                lpp[k] = lpps[li];
            }
            ++k;
        }
    return k;
}

int tilt_svt_layout(int m, int n, int* out) {
    if (m < 1 || n < 1 || !out) return TILT_ERR_ARG;
    ShapeCfg sc{};
    const int rc = shape_config(m, n, &sc);
    if (rc != TILT_OK) return rc;
    out[0] = svt_bs(sc.cfg);
    out[1] = svt_lpp(sc.cfg);
    out[2] = svt_nch(sc.cfg);
    out[3] = svt_tl(sc.cfg);
    out[4] = sc.sb > 0 ? 1 : 0;
    return TILT_OK;
}

int tilt_tune_set(int m, int n, int bs, int lpp) {
    if (m < 1 || n < 1 || (bs != 1 && bs != 2) || (lpp != 4 && lpp != 8 && lpp != 16)) return TILT_ERR_ARG;
    const int nc = std::min(m, n), nr = std::max(m, n);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (auto& e : g_tune)
        if (e.nc == nc && e.nr == nr) {
            e.bs = bs;
            e.lpp = lpp;
            return TILT_OK;
        }
    g_tune.push_back(TuneEntry{nc, nr, bs, lpp});
    return TILT_OK;
}

int tilt_tune_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    return TILT_OK;
}

}  // extern "C"
