// Host-side declarations shared by the batch driver (tilt_api.cpp) and the
// serving runtime (tilt_serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <vector>

#include "tilt.h"
#include "tilt_internal.h"

namespace tilt {
namespace host {

constexpr int kStaticLdsMargin = 8 * 1024;  // static __shared__ use of the kernels (checked at launch)
// Workgroups per tiled window the super-block size is planned for (the
// leader and the idle workgroups that help it in the fused kernel; see
// shape_config).
constexpr int kHelpPlan = 4;

// Device buffer that grows on demand.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t need);
    void release();
};

// Shape-dependent launch configuration of the SVT for one window.
struct ShapeCfg {
    int nc, nr, ldg, colmajor, cfg, ld, tb;
    int sb, nsb, ncp;  // tiled SVT (sb = 0: the whole matrix is held in LDS)
    size_t lds;
    size_t ws_floats;
    int warm_tb;       // warm-started SVT: reconstruction block rows (0: not possible)
    size_t warm_lds;   // warm-started SVT: dynamic LDS bytes
};

// warm: the layout of a warm-started solve (svt_mode 1), which takes the
// tiled layout where the rotation fits only there.
int shape_config(int m, int n, ShapeCfg* out, bool warm = false);
int tiled_config(const ShapeCfg& c, ShapeCfg* out, bool need_warm = false);
int help_plan();
// Whether idle workgroups help windows beyond LDS (TILT_HELPERS != 0).
bool helpers_enabled();
double predicted_cost(const PatchDesc& d);

int validate_params(const tilt_params* p);
int validate_problem(const tilt_problem* pr);
int initial_transform(const tilt_problem& pr, double* H);
SolverParams to_solver(const tilt_params* p);
int worse(int a, int b);
int record_hip_error(hipError_t e, const char* what, int line);
const char* last_error_text();
// Pixel homography -> scaled coordinates (cx, cy, s) of an m x n window and
// the p entries of tau; TILT_ERR_ARG for singular or non-affine input.
int normalise_window(const double* Hpx, int m, int n, int model, double* geo, double* tau);

// Descriptors of one request: `levels` level descriptors (level 0 first),
// the initial state (tau and scaled coordinates of the coarsest level),
// the workspace size in floats (planes, then the level images) and the
// dynamic LDS it needs.  Workspace pointers are offsets from 0 until the
// caller rebases them.
struct RequestPlan {
    PatchDesc d[MAX_LEVELS];
    PatchState init;
    int levels;
    size_t ws_floats;
    size_t lds;
};
int plan_request(const tilt_problem& pr, const tilt_params* prm, float* A_out, float* E_out, RequestPlan* out);
void rebase_plan(RequestPlan* plan, float* ws);
void fill_result(const PatchDesc& d0, const PatchState& s, tilt_result* r, double rate_khz, long long t0);

struct ServeState;
void serve_release(ServeState* s);

}  // namespace host
}  // namespace tilt

struct tilt_ctx {
    int device = 0;
    size_t budget = 0;
    tilt::host::DevBuf descs, states, ws, queue, order, scratch, jobs, counters, img;
    double wall_rate_khz = 100000.0;  // device wall clock
    int num_cus = 256;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_kernel_ms = 0.0;
    tilt::host::ServeState* serve = nullptr;
    // progress of a running fused launch (tilt_ctx_progress): its control
    // block, the request count, a side stream and a pinned word to read into
    std::atomic<void*> live_fc{nullptr};
    std::atomic<int> live_count{0};
    hipStream_t side = nullptr;
    int* pinned = nullptr;
};

#define HIP_TRY(x)                                                                   \
    do {                                                                             \
        hipError_t _e = (x);                                                         \
        if (_e != hipSuccess) return ::tilt::host::record_hip_error(_e, #x, __LINE__); \
    } while (0)
