// Serving runtime: request queue, device workspace arena and the
// persistent serving kernel behind tilt_submit / tilt_poll.
//
// Continuous batching: the serving kernel keeps one workgroup per compute
// unit alive; each takes the next published request the moment it is free,
// so requests of any size and arrival time share the GPU without waiting
// for a batch boundary.  The host side only publishes descriptors into a
// ring in pinned memory and collects results from it; no call blocks on
// the device except tilt_serve_stop.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "tilt.h"
#include "tilt_host.h"
#include "tilt_internal.h"

namespace tilt {
namespace host {

namespace {

constexpr int kRing = 1024;                         // request slots
constexpr size_t kArenaMax = 8ull << 30;            // device workspace arena cap
constexpr size_t kArenaAlign = 256;
constexpr double kIdleMs = 100.0;                   // serving kernel idle exit

// First-fit allocator over one device buffer; free blocks are coalesced.
class Arena {
  public:
    void reset(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + kArenaAlign - 1) & ~(kArenaAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_[*off] = bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }

  private:
    std::map<size_t, size_t> free_;
    std::map<size_t, size_t> used_;
};

enum ReqState { WAITING = 0, PUBLISHED = 1 };

struct Request {
    RequestPlan plan;
    SolverParams prm;
    int state = WAITING;
    unsigned long long seq = 0;
    size_t ws_off = 0, ws_bytes = 0;
};

}  // namespace

struct ServeState {
    std::mutex mu;
    ServeCtl* ctl = nullptr;      // pinned, coherent
    ServeSlot* slots = nullptr;   // pinned, coherent
    DevBuf head, ddesc, dstates, arena_buf;
    DevBuf help;                  // FusedCtl, then one GangCtl per ring slot (helpers)
    Arena arena;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool launched = false;
    size_t lds = 0;
    unsigned long long next_ticket = 1, next_seq = 0;
    std::deque<unsigned long long> waiting;
    std::unordered_map<unsigned long long, Request> reqs;
    std::vector<unsigned long long> slot_ticket;  // ticket in each slot (0 = free)
};

namespace {

int serve_init(tilt_ctx* ctx) {
    ServeState* S = new (std::nothrow) ServeState();
    if (!S) return TILT_ERR_NOMEM;
    auto fail = [&](int code) {
        serve_release(S);
        return code;
    };
    if (hipHostMalloc(reinterpret_cast<void**>(&S->ctl), sizeof(ServeCtl), hipHostMallocCoherent | hipHostMallocMapped) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&S->slots), sizeof(ServeSlot) * kRing,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
        return fail(TILT_ERR_NOMEM);
    std::memset(S->ctl, 0, sizeof(ServeCtl));
    std::memset(S->slots, 0, sizeof(ServeSlot) * kRing);
    S->arena_bytes = std::min(ctx->budget, kArenaMax);
    if (S->head.reserve(256) != hipSuccess || S->ddesc.reserve(sizeof(PatchDesc) * MAX_LEVELS * kRing) != hipSuccess ||
        S->dstates.reserve(sizeof(PatchState) * kRing) != hipSuccess ||
        S->arena_buf.reserve(S->arena_bytes) != hipSuccess)
        return fail(TILT_ERR_NOMEM);
    S->arena.reset(S->arena_bytes);
    // helpers' control blocks: a FusedCtl (idle count, registry) and the
    // GangCtl of each ring slot, unregistered; round ids and counters run
    // on across the requests of a slot
    {
        const size_t bytes = sizeof(FusedCtl) + sizeof(GangCtl) * kRing;
        if (S->help.reserve(bytes) != hipSuccess) return fail(TILT_ERR_NOMEM);
        std::vector<unsigned char> blob(bytes, 0);
        FusedCtl* dfc = reinterpret_cast<FusedCtl*>(S->help.p);
        GangCtl* dgang = reinterpret_cast<GangCtl*>(reinterpret_cast<unsigned char*>(S->help.p) + sizeof(FusedCtl));
        reinterpret_cast<FusedCtl*>(blob.data())->gangs = dgang;
        GangCtl* hgang = reinterpret_cast<GangCtl*>(blob.data() + sizeof(FusedCtl));
        for (int k = 0; k < kRing; ++k) {
            hgang[k].slot = -1;
            hgang[k].fc = dfc;
        }
        if (hipMemcpy(S->help.p, blob.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(TILT_ERR_DEVICE);
    }
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->done_ev, hipEventDisableTiming) != hipSuccess)
        return fail(TILT_ERR_DEVICE);
    if (hipMemsetAsync(S->head.p, 0, 256, S->stream) != hipSuccess || hipStreamSynchronize(S->stream) != hipSuccess)
        return fail(TILT_ERR_DEVICE);
    S->slot_ticket.assign(kRing, 0);
    S->lds = (size_t)LDS_LIMIT - kStaticLdsMargin;
    ctx->serve = S;
    return TILT_OK;
}

// Whether the kernel is still running: false if it was never started or
// its completion event has fired; a failed launch is reported.
int kernel_running(ServeState* S, bool* running) {
    *running = false;
    if (!S->launched) return TILT_OK;
    const hipError_t e = hipEventQuery(S->done_ev);
    if (e == hipErrorNotReady) {
        *running = true;
        return TILT_OK;
    }
    S->launched = false;
    if (e != hipSuccess) return record_hip_error(e, "serving kernel", __LINE__);
    return TILT_OK;
}

// Start the kernel if a published request has not finished and no kernel
// is running (it exits after kIdleMs without work).
int ensure_kernel(tilt_ctx* ctx, ServeState* S) {
    bool unfinished = false;
    for (const auto& kv : S->reqs) {
        const Request& R = kv.second;
        if (R.state == PUBLISHED &&
            __atomic_load_n(&S->slots[R.seq % kRing].done, __ATOMIC_ACQUIRE) != R.seq + 1) {
            unfinished = true;
            break;
        }
    }
    if (!unfinished) return TILT_OK;
    bool running = false;
    const int st = kernel_running(S, &running);
    if (st != TILT_OK) return st;
    if (running) return TILT_OK;
    __atomic_store_n(&S->ctl->stop, 0, __ATOMIC_RELEASE);
    // counters: claim index, requests in flight, closing latch, time of the
    // last finished request; a new launch starts with the latch open
    HIP_TRY(hipMemsetAsync(reinterpret_cast<unsigned long long*>(S->head.p) + 1, 0, 2 * sizeof(unsigned long long),
                           S->stream));
    const long long idle_ticks = (long long)(kIdleMs * ctx->wall_rate_khz);
    HIP_TRY(launch_serve(S->ctl, S->slots, reinterpret_cast<PatchDesc*>(S->ddesc.p),
                         reinterpret_cast<PatchState*>(S->dstates.p),
                         reinterpret_cast<unsigned long long*>(S->head.p), kRing, idle_ticks,
                         reinterpret_cast<FusedCtl*>(S->help.p), helpers_enabled() ? 1 : 0, ctx->num_cus, S->lds,
                         S->stream));
    HIP_TRY(hipEventRecord(S->done_ev, S->stream));
    S->launched = true;
    return TILT_OK;
}

// Publish waiting requests in order while slots and workspace are free.
int publish(tilt_ctx* ctx, ServeState* S) {
    float* base = reinterpret_cast<float*>(S->arena_buf.p);
    while (!S->waiting.empty()) {
        const unsigned long long ticket = S->waiting.front();
        Request& R = S->reqs[ticket];
        const int slot = (int)(S->next_seq % kRing);
        if (S->slot_ticket[slot] != 0) break;
        const size_t bytes = R.plan.ws_floats * sizeof(float);
        size_t off = 0;
        if (!S->arena.alloc(bytes, &off)) break;
        R.ws_off = off;
        R.ws_bytes = bytes;
        RequestPlan plan = R.plan;
        rebase_plan(&plan, base + off / sizeof(float));
        // a request with a tiled level names its slot's control block, so
        // that idle workgroups can help its Jacobi rounds
        bool tiled = false;
        for (int l = 0; l < plan.levels; ++l) tiled |= plan.d[l].sb > 0;
        GangCtl* gang = tiled && helpers_enabled()
                            ? reinterpret_cast<GangCtl*>(reinterpret_cast<unsigned char*>(S->help.p) + sizeof(FusedCtl)) + slot
                            : nullptr;
        for (int l = 0; l < plan.levels; ++l) plan.d[l].gang = gang;
        ServeSlot& sl = S->slots[slot];
        for (int l = 0; l < MAX_LEVELS; ++l) sl.d[l] = plan.d[l];
        sl.prm = R.prm;
        sl.init = plan.init;
        sl.levels = plan.levels;
        __atomic_store_n(&sl.done, 0ull, __ATOMIC_RELAXED);
        R.seq = S->next_seq;
        R.state = PUBLISHED;
        S->slot_ticket[slot] = ticket;
        S->waiting.pop_front();
        ++S->next_seq;
        __atomic_store_n(&S->ctl->tail, S->next_seq, __ATOMIC_RELEASE);
    }
    return ensure_kernel(ctx, S);
}

}  // namespace

void serve_release(ServeState* S) {
    if (!S) return;
    if (S->ctl && S->launched) {
        __atomic_store_n(&S->ctl->stop, 1, __ATOMIC_RELEASE);
        (void)hipEventSynchronize(S->done_ev);
    }
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    if (S->done_ev) (void)hipEventDestroy(S->done_ev);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    S->head.release();
    S->ddesc.release();
    S->dstates.release();
    S->arena_buf.release();
    S->help.release();
    if (S->slots) (void)hipHostFree(S->slots);
    if (S->ctl) (void)hipHostFree(S->ctl);
    delete S;
}

}  // namespace host
}  // namespace tilt

using namespace tilt;
using namespace tilt::host;

extern "C" {

int tilt_submit(tilt_ctx* ctx, const tilt_problem* prob, const tilt_params* prm, float* A_out, float* E_out,
                unsigned long long* ticket) {
    if (!ctx || !prob || !prm || !ticket) return TILT_ERR_ARG;
    int st = validate_params(prm);
    if (st != TILT_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!ctx->serve) {
        st = serve_init(ctx);
        if (st != TILT_OK) return st;
    }
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lock(S->mu);
    Request R;
    st = plan_request(*prob, prm, A_out, E_out, &R.plan);
    if (st != TILT_OK) return st;
    if (R.plan.ws_floats * sizeof(float) > S->arena_bytes) return TILT_ERR_NOMEM;
    R.prm = to_solver(prm);
    const unsigned long long t = S->next_ticket++;
    S->reqs.emplace(t, R);
    S->waiting.push_back(t);
    *ticket = t;
    return publish(ctx, S);
}

int tilt_poll(tilt_ctx* ctx, unsigned long long ticket, tilt_result* res) {
    if (!ctx || !res) return TILT_ERR_ARG;
    if (!ctx->serve) return TILT_ERR_NOT_FOUND;
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lock(S->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return TILT_ERR_NOT_FOUND;
    Request& R = it->second;
    if (R.state == PUBLISHED) {
        const int slot = (int)(R.seq % kRing);
        ServeSlot& sl = S->slots[slot];
        if (__atomic_load_n(&sl.done, __ATOMIC_ACQUIRE) == R.seq + 1) {
            PatchState out;
            std::memcpy(&out, &sl.result, sizeof(PatchState));
            fill_result(R.plan.d[0], out, res, ctx->wall_rate_khz, out.t_begin);
            const int status = res->status;
            S->arena.release(R.ws_off);
            S->slot_ticket[slot] = 0;
            S->reqs.erase(it);
            // the result is delivered: a device error while admitting the
            // queued requests is left in tilt_last_error; they stay queued
            // and the next submit or poll admits them again
            (void)publish(ctx, S);
            return status;
        }
    }
    const int p = publish(ctx, S);
    return p == TILT_OK ? TILT_PENDING : p;
}

int tilt_serve_stop(tilt_ctx* ctx) {
    if (!ctx) return TILT_ERR_ARG;
    if (!ctx->serve) return TILT_OK;
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lock(S->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    if (S->launched) {
        __atomic_store_n(&S->ctl->stop, 1, __ATOMIC_RELEASE);
        const hipError_t e = hipEventSynchronize(S->done_ev);
        S->launched = false;
        __atomic_store_n(&S->ctl->stop, 0, __ATOMIC_RELEASE);
        if (e != hipSuccess) return record_hip_error(e, "serving kernel", __LINE__);
    }
    return TILT_OK;
}

}  // extern "C"
