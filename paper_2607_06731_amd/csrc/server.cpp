// server.cpp -- scoring service over gp_eval_batched: resident datasets,
// admission against a device-memory budget, chunking, continuous batching
// over several in-flight streams, per-request latency, failure isolation
// and cancellation.
//
// The scheduling policy is gpsrv::Core (server_core.h), which makes no
// device call; this file gives it its device (HipDev: pinned staging, a
// copy stream, launch streams with done-events, gp_eval_batched) and runs
// it on one scheduler thread per server.  Its loop:
//   1. completions: a launch whose done-event has fired hands the results
//      of the requests it finished to the callers' arrays and frees their
//      buffers; a failed launch sends each of its requests to a retry of
//      its own, and a request that fails again completes with the error;
//   2. admission: waiting requests, oldest first, get a block of the device
//      arena and of pinned staging; their programs are staged (offsets
//      rebased per chunk) and copied up on the copy stream;
//   3. launches: each free stream takes the next batch: one chunk from
//      every admitted request first (oldest first), then further chunks
//      oldest first, up to the batch's chunk, work and workspace caps; the
//      batch is one gp_eval_batched call, followed by the copy-back of the
//      requests whose last chunk it holds.
// Requests that arrive while launches run are admitted at once and join the
// next launch.  Nothing in the arithmetic depends on the batch a program
// lands in, so results equal gp_eval of each population alone.

#include "gpeval.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "server_core.h"

void gp_internal_set_error(int code, const char* msg);
void gp_internal_release_stream_workspace(hipStream_t stream);

namespace {

using gpsrv::align_up;
using gpsrv::kMaxBatch;
using gpsrv::kMaxStreams;
using Clock = std::chrono::steady_clock;

static_assert(gpsrv::kCoreCancelled == GP_E_CANCELLED, "status codes");

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    gp_internal_set_error(code, buf);
    return code;
}

#define SRV_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(GP_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct HipSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* h_tables = nullptr;           // pinned: requests then datasets
    char* d_tables = nullptr;
};

// The device of the scheduling core: HIP streams, events and kernels.
struct HipDev {
    Clock::time_point t0 = Clock::now();
    char* d_arena = nullptr;
    char* h_arena = nullptr;
    hipStream_t up = nullptr;
    std::vector<HipSlot> slots;
    std::vector<hipEvent_t> free_events;
    const std::vector<gpsrv::Dataset>* datasets = nullptr;
    uint32_t allowed_op_mask = GP_BASE_OPS;
    bool one_launch_per_request = false;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    }

    // Copies a request's programs into its pinned block (offsets rebased
    // per chunk) and queues the upload on the copy stream.
    int upload(gpsrv::Request& R)
    {
        char* h = h_arena + R.host_off;
        std::memcpy(h, R.nodes, (size_t)R.n_nodes * 4);
        int64_t* ho = reinterpret_cast<int64_t*>(h + R.o_offs);
        size_t k = 0;
        for (const gpsrv::Chunk& c : R.chunks) {
            const int64_t base = R.offsets[c.b];
            for (int64_t p = c.b; p <= c.e; ++p) ho[k++] = R.offsets[p] - base;
        }
        if (R.n_consts) std::memcpy(h + R.o_consts, R.consts, (size_t)R.n_consts * 4);
        SRV_HIP(hipMemcpyAsync(d_arena + R.dev_off, h, R.o_out, hipMemcpyHostToDevice, up));
        if (free_events.empty()) {
            hipEvent_t e = nullptr;
            SRV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            free_events.push_back(e);
        }
        hipEvent_t e = free_events.back();
        free_events.pop_back();
        R.upload = e;
        SRV_HIP(hipEventRecord(e, up));
        return GP_OK;
    }

    void release_upload(gpsrv::Request& R)
    {
        if (R.upload) free_events.push_back(static_cast<hipEvent_t>(R.upload));
    }

    size_t workspace_bytes(int64_t P, int64_t N, int32_t n_req, int32_t n_ds, int32_t max_vars,
                           int64_t max_cases) const
    {
        size_t ws = 0;
        if (gp_workspace_size(P, N, n_req, n_ds, max_vars, max_cases, &ws) != GP_OK)
            return ~size_t(0);
        return ws;
    }

    int launch(int si, const gpsrv::Batch& B)
    {
        HipSlot& S = slots[(size_t)si];
        for (gpsrv::Request* R : B.touched)
            SRV_HIP(hipStreamWaitEvent(S.stream, static_cast<hipEvent_t>(R->upload), 0));
        for (const auto& w : B.waits) SRV_HIP(hipStreamWaitEvent(S.stream, slots[(size_t)w.first].done, 0));
        if (one_launch_per_request) {
            gpsrv::Request* R = B.ent[0].R;
            const gpsrv::Dataset& D = (*datasets)[(size_t)R->ds];
            char* d = d_arena + R->dev_off;
            // one chunk: offsets rebased to the first program's first node
            const int rc = gp_eval(reinterpret_cast<const uint32_t*>(d) + R->offsets[0],
                                   reinterpret_cast<const int64_t*>(d + R->o_offs), R->P,
                                   R->offsets[R->P] - R->offsets[0],
                                   reinterpret_cast<const float*>(d + R->o_consts), R->n_consts,
                                   D.X, D.n_vars, D.n_cases, D.y, D.n_cases, D.tax,
                                   allowed_op_mask, reinterpret_cast<double*>(d + R->o_out),
                                   reinterpret_cast<int32_t*>(d + R->o_st), S.stream);
            if (rc != GP_OK) return rc;
        } else {
            gp_request* hr = reinterpret_cast<gp_request*>(S.h_tables);
            gp_dataset* hd = reinterpret_cast<gp_dataset*>(S.h_tables + kMaxBatch * sizeof(gp_request));
            for (size_t i = 0; i < B.ent.size(); ++i) {
                gpsrv::Request* R = B.ent[i].R;
                const gpsrv::Chunk c = R->chunks[B.ent[i].chunk];
                // chunk j's rebased offsets start at entry c.b + j
                char* d = d_arena + R->dev_off;
                gp_request q;
                q.nodes = reinterpret_cast<const uint32_t*>(d) + R->offsets[c.b];
                q.offsets = reinterpret_cast<const int64_t*>(d + R->o_offs) + c.b + (int64_t)B.ent[i].chunk;
                q.consts = reinterpret_cast<const float*>(d + R->o_consts);
                q.n_programs = c.e - c.b;
                q.n_nodes = R->offsets[c.e] - R->offsets[c.b];
                q.n_consts = R->n_consts;
                q.out_fitness = reinterpret_cast<double*>(d + R->o_out) + c.b;
                q.out_status = reinterpret_cast<int32_t*>(d + R->o_st) + c.b;
                q.dataset = B.ds_local[(size_t)R->ds];
                q.reserved = 0;
                hr[i] = q;
            }
            for (size_t k = 0; k < B.ds_list.size(); ++k) {
                const gpsrv::Dataset& D = (*datasets)[(size_t)B.ds_list[k]];
                gp_dataset g;
                g.X = D.X;
                g.y = D.y;
                g.ld_x = D.n_cases;
                g.n_cases = D.n_cases;
                g.tax_on_length = D.tax;
                g.n_vars = D.n_vars;
                g.reserved = 0;
                hd[k] = g;
            }
            SRV_HIP(hipMemcpyAsync(S.d_tables, S.h_tables, B.ent.size() * sizeof(gp_request),
                                   hipMemcpyHostToDevice, S.stream));
            char* d_ds = S.d_tables + kMaxBatch * sizeof(gp_request);
            SRV_HIP(hipMemcpyAsync(d_ds, hd, B.ds_list.size() * sizeof(gp_dataset),
                                   hipMemcpyHostToDevice, S.stream));
            const int rc = gp_eval_batched(reinterpret_cast<const gp_request*>(S.d_tables),
                                           (int32_t)B.ent.size(), reinterpret_cast<const gp_dataset*>(d_ds),
                                           (int32_t)B.ds_list.size(), B.P, B.N, B.max_vars, B.max_cases,
                                           allowed_op_mask, S.stream);
            if (rc != GP_OK) return rc;
        }
        for (const gpsrv::ReqPtr& R : B.finishing) {
            const size_t n = R->o_st + (size_t)R->P * 4 - R->o_out;
            SRV_HIP(hipMemcpyAsync(h_arena + R->host_off + R->o_out, d_arena + R->dev_off + R->o_out,
                                   n, hipMemcpyDeviceToHost, S.stream));
        }
        SRV_HIP(hipEventRecord(S.done, S.stream));
        return GP_OK;
    }

    int poll(int si)
    {
        const hipError_t q = hipEventQuery(slots[(size_t)si].done);
        if (q == hipSuccess) return 1;
        if (q == hipErrorNotReady) return 0;
        (void)hipGetLastError();
        return fail(GP_E_HIP, "launch failed: %s", hipGetErrorString(q));
    }

    void deliver(gpsrv::Request& R)
    {
        const char* h = h_arena + R.host_off;
        std::memcpy(R.out_f, h + R.o_out, (size_t)R.P * 8);
        if (R.out_st) std::memcpy(R.out_st, h + R.o_st, (size_t)R.P * 4);
    }
};

}  // namespace

struct gp_server {
    gp_server_config cfg{};
    int device = 0;
    HipDev dev;
    std::unique_ptr<gpsrv::Core<HipDev>> core;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
};

namespace {

void scheduler(gp_server* s)
{
    (void)hipSetDevice(s->device);
    gpsrv::Core<HipDev>& C = *s->core;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        const bool progress = C.step();
        if (progress) s->cv_done.notify_all();
        const bool idle = C.idle();
        if (s->stop && C.live.empty() && idle) break;
        if (!progress) {
            if (!idle) s->cv_work.wait_for(lk, std::chrono::microseconds(50));
            else s->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

void destroy_all(gp_server* s)
{
    HipDev& d = s->dev;
    for (HipSlot& S : d.slots) {
        if (S.stream) {
            (void)hipStreamSynchronize(S.stream);
            gp_internal_release_stream_workspace(S.stream);
            (void)hipStreamDestroy(S.stream);
        }
        if (S.done) (void)hipEventDestroy(S.done);
        if (S.h_tables) (void)hipHostFree(S.h_tables);
        if (S.d_tables) (void)hipFree(S.d_tables);
    }
    if (d.up) {
        (void)hipStreamSynchronize(d.up);
        (void)hipStreamDestroy(d.up);
    }
    for (hipEvent_t e : d.free_events) (void)hipEventDestroy(e);
    if (d.d_arena) (void)hipFree(d.d_arena);
    if (d.h_arena) (void)hipHostFree(d.h_arena);
    delete s;
}

}  // namespace

extern "C" {

int gp_server_create(gp_server** server, const gp_server_config* config)
{
    if (!server) return fail(GP_E_INVALID_ARG, "server is NULL");
    *server = nullptr;
    gp_server_config c{};
    if (config) c = *config;
    if (c.device_budget_bytes < 0 || c.pinned_bytes < 0 || c.chunk_node_evals < 0 ||
        c.batch_node_evals < 0 || c.n_streams < 0 || c.n_streams > kMaxStreams ||
        c.max_batch_chunks < 0 || c.max_batch_chunks > kMaxBatch)
        return fail(GP_E_INVALID_ARG, "server configuration out of range");
    if (!c.device_budget_bytes) c.device_budget_bytes = int64_t(8) << 30;
    if (!c.pinned_bytes) c.pinned_bytes = std::min<int64_t>(c.device_budget_bytes, int64_t(1) << 30);
    if (!c.chunk_node_evals) c.chunk_node_evals = int64_t(1) << 35;
    if (!c.batch_node_evals) c.batch_node_evals = 4 * c.chunk_node_evals;
    if (!c.n_streams) c.n_streams = 2;
    if (!c.max_batch_chunks) c.max_batch_chunks = 1024;
    if (c.one_launch_per_request) c.n_streams = 1;
    if (!c.allowed_op_mask) c.allowed_op_mask = GP_BASE_OPS;
    if (c.allowed_op_mask & ~GP_ALL_OPS)
        return fail(GP_E_INVALID_ARG, "allowed_op_mask has bits beyond GP_ALL_OPS");
    if (c.device_budget_bytes < (int64_t(16) << 20))
        return fail(GP_E_INVALID_ARG, "device budget below 16 MiB");

    gp_server* s = new gp_server();
    s->cfg = c;
    auto bail = [&](int code) {
        destroy_all(s);
        return code;
    };
    if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(GP_E_HIP, "hipGetDevice failed"));
    gpsrv::Config k;
    k.chunk_node_evals = c.chunk_node_evals;
    k.batch_node_evals = c.batch_node_evals;
    k.n_streams = c.n_streams;
    k.max_batch_chunks = c.max_batch_chunks;
    k.one_launch_per_request = c.one_launch_per_request;
    // a quarter of the budget is left to the launch workspaces
    k.ws_cap = (size_t)(c.device_budget_bytes / 4 / c.n_streams);
    const size_t arena = (size_t)c.device_budget_bytes - k.ws_cap * (size_t)c.n_streams;
    size_t w0 = 0, wp = 0, wn = 0;
    if (gp_workspace_size(0, 0, 1, 1, 20, int64_t(1) << 40, &w0) != GP_OK ||
        gp_workspace_size(1 << 20, 0, 1, 1, 20, int64_t(1) << 40, &wp) != GP_OK ||
        gp_workspace_size(0, 1 << 24, 1, 1, 20, int64_t(1) << 40, &wn) != GP_OK)
        return bail(fail(GP_E_HIP, "workspace model"));
    // linear model of the workspace (the most tiles per program), with the
    // alignment slack of its sections
    k.ws_fixed = (double)w0 + 65536.0;
    k.ws_per_prog = (double)(wp - w0) / (double)(1 << 20);
    k.ws_per_node = (double)(wn - w0) / (double)(1 << 24);
    HipDev& d = s->dev;
    d.allowed_op_mask = c.allowed_op_mask;
    d.one_launch_per_request = c.one_launch_per_request != 0;
    if (hipMalloc(&d.d_arena, arena) != hipSuccess) {
        (void)hipGetLastError();
        d.d_arena = nullptr;
        return bail(fail(GP_E_NO_MEMORY, "device arena of %zu bytes", arena));
    }
    if (hipHostMalloc(&d.h_arena, (size_t)c.pinned_bytes, 0) != hipSuccess) {
        (void)hipGetLastError();
        d.h_arena = nullptr;
        return bail(fail(GP_E_NO_MEMORY, "pinned staging of %lld bytes", (long long)c.pinned_bytes));
    }
    if (hipStreamCreateWithFlags(&d.up, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(GP_E_HIP, "copy stream"));
    d.slots.resize((size_t)c.n_streams);
    const size_t tables = kMaxBatch * (sizeof(gp_request) + sizeof(gp_dataset));
    for (HipSlot& S : d.slots) {
        if (hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&S.h_tables, tables, 0) != hipSuccess ||
            hipMalloc(&S.d_tables, tables) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(GP_E_HIP, "launch stream setup"));
        }
    }
    s->core.reset(new gpsrv::Core<HipDev>(d, k, arena, (size_t)c.pinned_bytes));
    d.datasets = &s->core->datasets;
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        return bail(fail(GP_E_HIP, "scheduler thread"));
    }
    *server = s;
    return GP_OK;
}

int gp_server_add_dataset(gp_server* s, const float* X, int32_t n_vars, int64_t ld_x,
                          const float* y, int64_t n_cases, double tax_on_length,
                          int32_t* dataset_id)
{
    if (!s || !y || !dataset_id || (n_vars > 0 && !X)) return fail(GP_E_INVALID_ARG, "NULL argument");
    if (n_vars < 0 || n_vars > 4096 || n_cases < 1 || (n_vars > 0 && ld_x < n_cases) ||
        !std::isfinite(tax_on_length))
        return fail(GP_E_INVALID_ARG, "dataset sizes out of range");
    std::lock_guard<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    const size_t xb = align_up((size_t)n_vars * (size_t)n_cases * 4);
    const size_t bytes = xb + (size_t)n_cases * 4;
    size_t off = 0;
    if (!C.darena.alloc(bytes, &off))
        return fail(GP_E_NO_MEMORY, "dataset of %zu bytes does not fit the arena now", bytes);
    gpsrv::Dataset D;
    D.live = true;
    D.off = off;
    D.bytes = bytes;
    D.X = reinterpret_cast<float*>(s->dev.d_arena + off);
    D.y = reinterpret_cast<float*>(s->dev.d_arena + off + xb);
    D.n_vars = n_vars;
    D.n_cases = n_cases;
    D.tax = tax_on_length;
    hipError_t e = hipSuccess;
    if (n_vars > 0)
        e = hipMemcpy2DAsync(D.X, (size_t)n_cases * 4, X, (size_t)ld_x * 4, (size_t)n_cases * 4,
                             (size_t)n_vars, hipMemcpyHostToDevice, s->dev.up);
    if (e == hipSuccess)
        e = hipMemcpyAsync(D.y, y, (size_t)n_cases * 4, hipMemcpyHostToDevice, s->dev.up);
    if (e == hipSuccess) e = hipStreamSynchronize(s->dev.up);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        C.darena.release(off, bytes);
        return fail(GP_E_HIP, "dataset upload: %s", hipGetErrorString(e));
    }
    int id = -1;
    for (size_t i = 0; i < C.datasets.size(); ++i)
        if (!C.datasets[i].live) { id = (int)i; break; }
    if (id < 0) {
        id = (int)C.datasets.size();
        C.datasets.push_back(D);
    } else {
        C.datasets[(size_t)id] = D;
    }
    *dataset_id = id;
    return GP_OK;
}

int gp_server_remove_dataset(gp_server* s, int32_t id)
{
    if (!s) return fail(GP_E_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    if (id < 0 || id >= (int)C.datasets.size() || !C.datasets[(size_t)id].live)
        return fail(GP_E_INVALID_ARG, "unknown dataset %d", id);
    gpsrv::Dataset& D = C.datasets[(size_t)id];
    if (D.pending) return fail(GP_E_INVALID_ARG, "dataset %d has %d pending requests", id, D.pending);
    C.darena.release(D.off, D.bytes);
    D = gpsrv::Dataset();
    return GP_OK;
}

int gp_server_submit(gp_server* s, int32_t id, const uint32_t* nodes, int64_t n_nodes,
                     const int64_t* offsets, int64_t n_programs, const float* consts,
                     int64_t n_consts, double* out_fitness, int32_t* out_status, int64_t* ticket)
{
    if (!s || !ticket || !offsets) return fail(GP_E_INVALID_ARG, "NULL argument");
    if (n_programs < 0 || n_programs > INT32_MAX - 1 || n_nodes < 0 || n_consts < 0 ||
        n_consts > GP_MAX_CONSTS)
        return fail(GP_E_INVALID_ARG, "request sizes out of range");
    if ((n_nodes > 0 && !nodes) || (n_consts > 0 && !consts) || (n_programs > 0 && !out_fitness))
        return fail(GP_E_INVALID_ARG, "NULL array");
    if (offsets[0] < 0 || offsets[n_programs] > n_nodes)
        return fail(GP_E_INVALID_ARG, "offsets outside [0, n_nodes]");
    for (int64_t p = 0; p < n_programs; ++p)
        if (offsets[p + 1] < offsets[p]) return fail(GP_E_INVALID_ARG, "offsets decrease at %lld", (long long)p);
    auto R = std::make_shared<gpsrv::Request>();
    R->nodes = nodes;
    R->n_nodes = n_nodes;
    R->offsets = offsets;
    R->P = n_programs;
    R->consts = consts;
    R->n_consts = n_consts;
    R->out_f = out_fitness;
    R->out_st = out_status;
    R->ds = id;
    std::unique_lock<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    if (s->stop) return fail(GP_E_INVALID_ARG, "server is shutting down");
    if (id < 0 || id >= (int)C.datasets.size() || !C.datasets[(size_t)id].live)
        return fail(GP_E_INVALID_ARG, "unknown dataset %d", id);
    if (C.submit(R, ticket) != GP_OK)
        return fail(GP_E_TOO_LARGE, "request needs %zu bytes: more than the budget", R->bytes);
    lk.unlock();
    s->cv_work.notify_one();
    return GP_OK;
}

int gp_server_cancel(gp_server* s, int64_t ticket)
{
    if (!s) return fail(GP_E_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->core->cancel(ticket) != GP_OK)
        return fail(GP_E_INVALID_ARG, "ticket %lld is not pending", (long long)ticket);
    lk.unlock();
    s->cv_done.notify_all();
    s->cv_work.notify_one();
    return GP_OK;
}

int gp_server_poll(gp_server* s, double timeout_ms, int64_t* tickets, int32_t* results,
                   int32_t max_n, int32_t* n_done)
{
    if (!s || !n_done || max_n < 0 || (max_n > 0 && (!tickets || !results)))
        return fail(GP_E_INVALID_ARG, "bad poll arguments");
    *n_done = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    auto have = [&] {
        while (!C.done_q.empty() && !C.done_rc.count(C.done_q.front())) C.done_q.pop_front();
        return !C.done_q.empty();
    };
    if (timeout_ms < 0) s->cv_done.wait(lk, have);
    else if (timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), have);
    int n = 0;
    while (n < max_n && have()) {
        const int64_t t = C.done_q.front();
        C.done_q.pop_front();
        tickets[n] = t;
        results[n] = C.done_rc[t];
        C.done_rc.erase(t);
        ++n;
    }
    *n_done = n;
    return GP_OK;
}

int gp_server_wait(gp_server* s, int64_t ticket, double timeout_ms, int32_t* done, int32_t* result)
{
    if (!s || !done || !result) return fail(GP_E_INVALID_ARG, "NULL argument");
    *done = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    if (!C.live.count(ticket) && !C.done_rc.count(ticket))
        return fail(GP_E_INVALID_ARG, "unknown or consumed ticket %lld", (long long)ticket);
    auto have = [&] { return C.done_rc.count(ticket) != 0; };
    if (timeout_ms < 0) s->cv_done.wait(lk, have);
    else if (timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), have);
    if (!have()) return GP_OK;
    *done = 1;
    *result = C.done_rc[ticket];
    C.done_rc.erase(ticket);
    return GP_OK;
}

int gp_server_get_stats(gp_server* s, gp_server_stats* out)
{
    if (!s || !out) return fail(GP_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    gp_server_stats r{};
    const double now = s->dev.now_ms();
    r.submitted = C.n_submitted;
    r.completed = C.n_completed;
    r.failed = C.n_failed;
    r.launches = C.n_launches;
    r.chunks_launched = C.n_chunks;
    r.node_evals = C.node_evals;
    r.busy_ms = C.busy_ms + (C.busy_slots ? now - C.busy_since_ms : 0.0);
    r.wall_ms = now - C.t_reset_ms;
    r.device_bytes_in_use = (int64_t)C.darena.used();
    r.device_bytes_peak = (int64_t)C.darena.peak();
    r.waiting = (int32_t)C.waiting.size();
    r.in_flight = (int32_t)(C.live.size() - C.waiting.size());
    if (!C.latencies.empty()) {
        r.latency_p50_ms = C.latency_pct(0.50);
        r.latency_p99_ms = C.latency_pct(0.99);
        r.latency_max_ms = *std::max_element(C.latencies.begin(), C.latencies.end());
        double sum = 0.0;
        for (double x : C.latencies) sum += x;
        r.latency_mean_ms = sum / (double)C.latencies.size();
    }
    r.cancelled = C.n_cancelled;
    r.retried = C.n_retried;
    *out = r;
    return GP_OK;
}

int gp_server_reset_stats(gp_server* s)
{
    if (!s) return fail(GP_E_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    gpsrv::Core<HipDev>& C = *s->core;
    const double now = s->dev.now_ms();
    C.t_reset_ms = now;
    C.n_submitted = C.n_completed = C.n_failed = C.n_launches = C.n_chunks = 0;
    C.n_cancelled = C.n_retried = 0;
    C.node_evals = 0.0;
    C.busy_ms = 0.0;
    if (C.busy_slots) C.busy_since_ms = now;
    C.latencies.clear();
    C.darena.reset_peak();
    return GP_OK;
}

void gp_server_destroy(gp_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    destroy_all(s);
}

}  // extern "C"
