// server.cpp -- scoring service over gp_eval_batched: resident datasets,
// admission against a device-memory budget, chunking, continuous batching
// over several in-flight streams, per-request latency.
//
// One scheduler thread per server does all device work.  Its loop:
//   1. completions: a launch whose done-event has fired hands the results
//      of the requests it finished to the callers' arrays and frees their
//      buffers;
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
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

void gp_internal_set_error(int code, const char* msg);
void gp_internal_release_stream_workspace(hipStream_t stream);

namespace {

using Clock = std::chrono::steady_clock;

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

constexpr size_t kAlign = 256;
constexpr int kMaxStreams = 8;
constexpr int kMaxBatch = 4096;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over offsets of one contiguous region; free blocks are
// coalesced with their neighbours on release.
class Arena {
public:
    void init(size_t cap)
    {
        cap_ = cap;
        free_.clear();
        used_ = peak_ = 0;
        if (cap) free_[0] = cap;
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[*off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Chunk {
    int64_t b, e;           // program range [b, e)
};

// Layout of a request's device block (mirrored in its pinned block):
// nodes | per-chunk rebased offsets | constants | fitness | status.
struct Request {
    int64_t ticket = 0;
    int32_t ds = 0;
    const uint32_t* nodes = nullptr;
    int64_t n_nodes = 0;
    const int64_t* offsets = nullptr;
    int64_t P = 0;
    const float* consts = nullptr;
    int64_t n_consts = 0;
    double* out_f = nullptr;
    int32_t* out_st = nullptr;
    double node_evals = 0.0;
    Clock::time_point t_submit;
    std::vector<Chunk> chunks;
    size_t next_chunk = 0;
    size_t bytes = 0, o_offs = 0, o_consts = 0, o_out = 0, o_st = 0;
    size_t dev_off = 0, host_off = 0;
    bool admitted = false;              // holds arena and staging blocks
    hipEvent_t uploaded = nullptr;
    std::vector<std::pair<int, uint64_t>> batches;  // (slot, launch) of earlier chunks
};

using ReqPtr = std::shared_ptr<Request>;

struct Dataset {
    bool live = false;
    size_t off = 0, bytes = 0;
    float* X = nullptr;
    float* y = nullptr;
    int32_t n_vars = 0;
    int64_t n_cases = 0;
    double tax = 0.0;
    int pending = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t seq = 0;
    std::vector<ReqPtr> finishing;      // requests whose last chunk is in this launch
    char* h_tables = nullptr;           // pinned: requests then datasets
    char* d_tables = nullptr;
    Clock::time_point t_launch;
};

}  // namespace

struct gp_server {
    gp_server_config cfg{};
    int device = 0;
    char* d_arena = nullptr;
    char* h_arena = nullptr;
    Arena dev, host;
    size_t ws_cap = 0;                  // workspace per launch stream
    double ws_per_prog = 0.0, ws_per_node = 0.0, ws_fixed = 0.0;
    hipStream_t up = nullptr;
    std::vector<Slot> slots;
    std::vector<Dataset> datasets;
    std::vector<hipEvent_t> free_events;
    std::deque<ReqPtr> waiting;         // submitted, not admitted
    std::deque<ReqPtr> ready;           // admitted, chunks left to launch
    std::unordered_map<int64_t, ReqPtr> live;
    std::deque<int64_t> done_q;
    std::unordered_map<int64_t, int> done_rc;
    int64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
    int broken = GP_OK;
    // statistics since creation / reset
    Clock::time_point t_reset;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_launches = 0, n_chunks = 0;
    double node_evals = 0.0, busy_ms = 0.0;
    int busy_slots = 0;
    Clock::time_point busy_since;
    std::vector<double> latencies;
};

namespace {

// Bytes of a request's block and its section offsets.
void size_request(Request& R)
{
    size_t off = align_up((size_t)R.n_nodes * 4);
    R.o_offs = off;
    off = align_up(off + (size_t)(R.P + (int64_t)R.chunks.size()) * 8);
    R.o_consts = off;
    off = align_up(off + (size_t)R.n_consts * 4);
    R.o_out = off;
    off += (size_t)R.P * 8;             // fitness and status are adjacent: one copy back
    R.o_st = off;
    off = align_up(off + (size_t)R.P * 4);
    R.bytes = off;
}

// Program ranges of at most chunk_node_evals work and ws_cap workspace each
// (one range in comparison mode).
void split_request(const gp_server* s, Request& R, int64_t n_cases)
{
    R.chunks.clear();
    if (s->cfg.one_launch_per_request || R.P == 0) {
        R.chunks.push_back({0, R.P});
        return;
    }
    const double cap = (double)s->cfg.chunk_node_evals;
    int64_t b = 0;
    while (b < R.P) {
        int64_t e = b;
        double ev = 0.0;
        while (e < R.P) {
            const double len = (double)(R.offsets[e + 1] - R.offsets[e]);
            const double w = len * (double)n_cases;
            const double ws = s->ws_fixed + s->ws_per_prog * (double)(e + 1 - b) +
                              s->ws_per_node * (double)(R.offsets[e + 1] - R.offsets[b]);
            if (e > b && (ev + w > cap || ws > (double)s->ws_cap)) break;
            ev += w;
            ++e;
        }
        R.chunks.push_back({b, e});
        b = e;
    }
}

void complete(gp_server* s, const ReqPtr& R, int rc)
{
    const auto now = Clock::now();
    if (rc == GP_OK) {
        const char* h = s->h_arena + R->host_off;
        std::memcpy(R->out_f, h + R->o_out, (size_t)R->P * 8);
        if (R->out_st) std::memcpy(R->out_st, h + R->o_st, (size_t)R->P * 4);
        s->n_completed += 1;
        s->node_evals += R->node_evals;
        s->latencies.push_back(ms_between(R->t_submit, now));
    } else {
        s->n_failed += 1;
    }
    if (R->admitted) {
        s->dev.release(R->dev_off, R->bytes);
        s->host.release(R->host_off, R->bytes);
        R->admitted = false;
    }
    s->datasets[R->ds].pending -= 1;
    if (R->uploaded) s->free_events.push_back(R->uploaded);
    R->uploaded = nullptr;
    s->live.erase(R->ticket);
    s->done_q.push_back(R->ticket);
    s->done_rc[R->ticket] = rc;
}

// Copy a request's programs into its pinned block (offsets rebased per
// chunk) and queue the upload on the copy stream.  Scheduler thread only.
int stage(gp_server* s, Request& R)
{
    char* h = s->h_arena + R.host_off;
    std::memcpy(h, R.nodes, (size_t)R.n_nodes * 4);
    int64_t* ho = reinterpret_cast<int64_t*>(h + R.o_offs);
    size_t k = 0;
    for (const Chunk& c : R.chunks) {
        const int64_t base = R.offsets[c.b];
        for (int64_t p = c.b; p <= c.e; ++p) ho[k++] = R.offsets[p] - base;
    }
    if (R.n_consts) std::memcpy(h + R.o_consts, R.consts, (size_t)R.n_consts * 4);
    SRV_HIP(hipMemcpyAsync(s->d_arena + R.dev_off, h, R.o_out, hipMemcpyHostToDevice, s->up));
    if (s->free_events.empty()) {
        hipEvent_t e = nullptr;
        SRV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        s->free_events.push_back(e);
    }
    R.uploaded = s->free_events.back();
    s->free_events.pop_back();
    SRV_HIP(hipEventRecord(R.uploaded, s->up));
    return GP_OK;
}

// Admit every waiting request that fits, oldest first.  The staging copy
// runs with the lock released: only this thread touches the arenas, the
// ready list and admitted requests.
int admit(gp_server* s, std::unique_lock<std::mutex>& lk, bool* progress)
{
    while (!s->waiting.empty()) {
        const ReqPtr R = s->waiting.front();
        size_t od = 0, oh = 0;
        if (!s->dev.alloc(R->bytes, &od)) break;
        if (!s->host.alloc(R->bytes, &oh)) {
            s->dev.release(od, R->bytes);
            break;
        }
        R->dev_off = od;
        R->host_off = oh;
        R->admitted = true;
        s->waiting.pop_front();
        lk.unlock();
        const int rc = stage(s, *R);
        lk.lock();
        s->ready.push_back(R);          // on failure the server fails it below
        if (rc != GP_OK) return rc;
        *progress = true;
    }
    return GP_OK;
}

struct Entry {
    Request* R;
    size_t chunk;
};

// Form the next batch for slot `si` and enqueue it.
int launch(gp_server* s, int si)
{
    Slot& S = s->slots[si];
    std::vector<Entry> ent;
    std::vector<int> ds_local(s->datasets.size(), -1);
    std::vector<int32_t> ds_list;
    int64_t P = 0, N = 0;
    int32_t maxv = 0;
    int64_t maxc = 1;
    double work = 0.0;
    const int max_chunks = s->cfg.one_launch_per_request ? 1 : s->cfg.max_batch_chunks;
    const double max_work = (double)s->cfg.batch_node_evals;

    // try to add chunk `ci` of R; false when a cap is reached
    auto take = [&](Request* R) -> bool {
        if ((int)ent.size() >= max_chunks) return false;
        const Chunk c = R->chunks[R->next_chunk];
        const Dataset& D = s->datasets[R->ds];
        const int64_t cn = R->offsets[c.e] - R->offsets[c.b];
        const double cw = (double)cn * (double)D.n_cases;
        if (!ent.empty()) {
            if (work + cw > max_work) return false;
            const int nds = (int)ds_list.size() + (ds_local[R->ds] < 0 ? 1 : 0);
            size_t ws = 0;
            if (gp_workspace_size(P + (c.e - c.b), N + cn, (int32_t)ent.size() + 1, nds,
                                  std::max(maxv, D.n_vars), std::max(maxc, D.n_cases),
                                  &ws) != GP_OK || ws > s->ws_cap)
                return false;
        }
        if (ds_local[R->ds] < 0) {
            ds_local[R->ds] = (int)ds_list.size();
            ds_list.push_back(R->ds);
        }
        ent.push_back({R, R->next_chunk});
        R->next_chunk += 1;
        P += c.e - c.b;
        N += cn;
        work += cw;
        maxv = std::max(maxv, D.n_vars);
        maxc = std::max(maxc, D.n_cases);
        return true;
    };
    // one chunk from every admitted request (oldest first), then fill up
    bool full = false;
    for (const ReqPtr& R : s->ready) {
        if (R->next_chunk < R->chunks.size() && !take(R.get())) { full = true; break; }
    }
    for (const ReqPtr& R : s->ready) {
        if (full) break;
        while (R->next_chunk < R->chunks.size()) {
            if (!take(R.get())) { full = true; break; }
        }
    }
    if (ent.empty()) return GP_OK;

    // requests finished by this launch leave the ready list
    std::vector<Request*> touched;
    for (const Entry& e : ent)
        if (touched.empty() || touched.back() != e.R) touched.push_back(e.R);
    std::sort(touched.begin(), touched.end());
    touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
    S.finishing.clear();
    for (auto it = s->ready.begin(); it != s->ready.end();) {
        if ((*it)->next_chunk == (*it)->chunks.size()) {
            S.finishing.push_back(*it);
            it = s->ready.erase(it);
        } else {
            ++it;
        }
    }

    S.seq += 1;
    for (Request* R : touched) SRV_HIP(hipStreamWaitEvent(S.stream, R->uploaded, 0));
    for (const ReqPtr& R : S.finishing) {
        for (const auto& b : R->batches) {
            const Slot& O = s->slots[b.first];
            if (b.first != si && O.busy && O.seq == b.second)
                SRV_HIP(hipStreamWaitEvent(S.stream, O.done, 0));
        }
    }
    if (s->cfg.one_launch_per_request) {
        Request* R = ent[0].R;
        const Dataset& D = s->datasets[R->ds];
        char* d = s->d_arena + R->dev_off;
        // one chunk: offsets rebased to the first program's first node
        const int rc = gp_eval(reinterpret_cast<const uint32_t*>(d) + R->offsets[0],
                               reinterpret_cast<const int64_t*>(d + R->o_offs), R->P,
                               R->offsets[R->P] - R->offsets[0],
                               reinterpret_cast<const float*>(d + R->o_consts), R->n_consts, D.X,
                               D.n_vars, D.n_cases, D.y, D.n_cases, D.tax, s->cfg.allowed_op_mask,
                               reinterpret_cast<double*>(d + R->o_out),
                               reinterpret_cast<int32_t*>(d + R->o_st), S.stream);
        if (rc != GP_OK) return rc;
    } else {
        gp_request* hr = reinterpret_cast<gp_request*>(S.h_tables);
        gp_dataset* hd = reinterpret_cast<gp_dataset*>(S.h_tables + kMaxBatch * sizeof(gp_request));
        for (size_t i = 0; i < ent.size(); ++i) {
            Request* R = ent[i].R;
            const Chunk c = R->chunks[ent[i].chunk];
            // chunk j's rebased offsets start at entry c.b + j
            char* d = s->d_arena + R->dev_off;
            gp_request q;
            q.nodes = reinterpret_cast<const uint32_t*>(d) + R->offsets[c.b];
            q.offsets = reinterpret_cast<const int64_t*>(d + R->o_offs) + c.b + (int64_t)ent[i].chunk;
            q.consts = reinterpret_cast<const float*>(d + R->o_consts);
            q.n_programs = c.e - c.b;
            q.n_nodes = R->offsets[c.e] - R->offsets[c.b];
            q.n_consts = R->n_consts;
            q.out_fitness = reinterpret_cast<double*>(d + R->o_out) + c.b;
            q.out_status = reinterpret_cast<int32_t*>(d + R->o_st) + c.b;
            q.dataset = ds_local[R->ds];
            q.reserved = 0;
            hr[i] = q;
        }
        for (size_t k = 0; k < ds_list.size(); ++k) {
            const Dataset& D = s->datasets[ds_list[k]];
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
        SRV_HIP(hipMemcpyAsync(S.d_tables, S.h_tables, ent.size() * sizeof(gp_request),
                               hipMemcpyHostToDevice, S.stream));
        char* d_ds = S.d_tables + kMaxBatch * sizeof(gp_request);
        SRV_HIP(hipMemcpyAsync(d_ds, hd, ds_list.size() * sizeof(gp_dataset),
                               hipMemcpyHostToDevice, S.stream));
        const int rc = gp_eval_batched(reinterpret_cast<const gp_request*>(S.d_tables),
                                       (int32_t)ent.size(), reinterpret_cast<const gp_dataset*>(d_ds),
                                       (int32_t)ds_list.size(), P, N, maxv, maxc,
                                       s->cfg.allowed_op_mask, S.stream);
        if (rc != GP_OK) return rc;
    }
    for (const ReqPtr& R : S.finishing) {
        const size_t n = R->o_st + (size_t)R->P * 4 - R->o_out;
        SRV_HIP(hipMemcpyAsync(s->h_arena + R->host_off + R->o_out,
                               s->d_arena + R->dev_off + R->o_out, n, hipMemcpyDeviceToHost,
                               S.stream));
    }
    SRV_HIP(hipEventRecord(S.done, S.stream));
    for (Request* R : touched) R->batches.push_back({si, S.seq});
    S.busy = true;
    S.t_launch = Clock::now();
    if (s->busy_slots++ == 0) s->busy_since = S.t_launch;
    s->n_launches += 1;
    s->n_chunks += (int64_t)ent.size();
    return GP_OK;
}

void finish(gp_server* s, int si)
{
    Slot& S = s->slots[si];
    for (const ReqPtr& R : S.finishing) complete(s, R, GP_OK);
    S.finishing.clear();
    S.busy = false;
    if (--s->busy_slots == 0) s->busy_ms += ms_between(s->busy_since, Clock::now());
}

// A device error ends the server: every unfinished request fails with rc.
void break_server(gp_server* s, int rc)
{
    s->broken = rc;
    std::vector<ReqPtr> all;
    for (auto& kv : s->live) all.push_back(kv.second);
    for (const ReqPtr& R : all) complete(s, R, rc);
    s->waiting.clear();
    s->ready.clear();
    for (Slot& S : s->slots) {
        S.finishing.clear();
        S.busy = false;
    }
    s->busy_slots = 0;
}

void scheduler(gp_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        int rc = GP_OK;
        if (s->broken == GP_OK) {
            for (int i = 0; i < (int)s->slots.size() && rc == GP_OK; ++i) {
                Slot& S = s->slots[i];
                if (!S.busy) continue;
                const hipError_t q = hipEventQuery(S.done);
                if (q == hipSuccess) {
                    finish(s, i);
                    progress = true;
                } else if (q != hipErrorNotReady) {
                    rc = fail(GP_E_HIP, "launch failed: %s", hipGetErrorString(q));
                }
            }
            if (rc == GP_OK) rc = admit(s, lk, &progress);
            for (int i = 0; i < (int)s->slots.size() && rc == GP_OK; ++i) {
                if (s->slots[i].busy || s->ready.empty()) continue;
                rc = launch(s, i);
                progress = progress || s->slots[i].busy;
            }
            if (rc != GP_OK) {
                break_server(s, rc);
                progress = true;
            }
        }
        if (progress) s->cv_done.notify_all();
        const bool idle = s->busy_slots == 0;
        if (s->stop && s->live.empty() && idle) break;
        if (s->broken != GP_OK && s->stop) break;
        if (!progress) {
            if (!idle) s->cv_work.wait_for(lk, std::chrono::microseconds(50));
            else s->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

void destroy_all(gp_server* s)
{
    for (Slot& S : s->slots) {
        if (S.stream) {
            (void)hipStreamSynchronize(S.stream);
            gp_internal_release_stream_workspace(S.stream);
            (void)hipStreamDestroy(S.stream);
        }
        if (S.done) (void)hipEventDestroy(S.done);
        if (S.h_tables) (void)hipHostFree(S.h_tables);
        if (S.d_tables) (void)hipFree(S.d_tables);
    }
    if (s->up) {
        (void)hipStreamSynchronize(s->up);
        (void)hipStreamDestroy(s->up);
    }
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->h_arena) (void)hipHostFree(s->h_arena);
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
    if (c.allowed_op_mask & ~GP_BASE_OPS)
        return fail(GP_E_INVALID_ARG, "allowed_op_mask reaches beyond GP_BASE_OPS (scoring takes the benchmark set)");
    if (c.device_budget_bytes < (int64_t(16) << 20))
        return fail(GP_E_INVALID_ARG, "device budget below 16 MiB");

    gp_server* s = new gp_server();
    s->cfg = c;
    int rc = GP_OK;
    auto bail = [&](int code) {
        destroy_all(s);
        return code;
    };
    if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(GP_E_HIP, "hipGetDevice failed"));
    // a quarter of the budget is left to the launch workspaces
    s->ws_cap = (size_t)(c.device_budget_bytes / 4 / c.n_streams);
    const size_t arena = (size_t)c.device_budget_bytes - s->ws_cap * (size_t)c.n_streams;
    size_t w0 = 0, wp = 0, wn = 0;
    if (gp_workspace_size(0, 0, 1, 1, 20, int64_t(1) << 40, &w0) != GP_OK ||
        gp_workspace_size(1 << 20, 0, 1, 1, 20, int64_t(1) << 40, &wp) != GP_OK ||
        gp_workspace_size(0, 1 << 24, 1, 1, 20, int64_t(1) << 40, &wn) != GP_OK)
        return bail(fail(GP_E_HIP, "workspace model"));
    // linear model of the workspace (the most tiles per program), with the
    // alignment slack of its sections
    s->ws_fixed = (double)w0 + 65536.0;
    s->ws_per_prog = (double)(wp - w0) / (double)(1 << 20);
    s->ws_per_node = (double)(wn - w0) / (double)(1 << 24);
    if (hipMalloc(&s->d_arena, arena) != hipSuccess) {
        (void)hipGetLastError();
        s->d_arena = nullptr;
        return bail(fail(GP_E_NO_MEMORY, "device arena of %zu bytes", arena));
    }
    if (hipHostMalloc(&s->h_arena, (size_t)c.pinned_bytes, 0) != hipSuccess) {
        (void)hipGetLastError();
        s->h_arena = nullptr;
        return bail(fail(GP_E_NO_MEMORY, "pinned staging of %lld bytes", (long long)c.pinned_bytes));
    }
    s->dev.init(arena);
    s->host.init((size_t)c.pinned_bytes);
    if (hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(GP_E_HIP, "copy stream"));
    s->slots.resize((size_t)c.n_streams);
    const size_t tables = kMaxBatch * (sizeof(gp_request) + sizeof(gp_dataset));
    for (Slot& S : s->slots) {
        if (hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&S.h_tables, tables, 0) != hipSuccess ||
            hipMalloc(&S.d_tables, tables) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(GP_E_HIP, "launch stream setup"));
        }
    }
    s->t_reset = Clock::now();
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        return bail(fail(GP_E_HIP, "scheduler thread"));
    }
    (void)rc;
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
    if (s->broken != GP_OK) return fail(s->broken, "server stopped after a device error");
    const size_t xb = align_up((size_t)n_vars * (size_t)n_cases * 4);
    const size_t bytes = xb + (size_t)n_cases * 4;
    size_t off = 0;
    if (!s->dev.alloc(bytes, &off))
        return fail(GP_E_NO_MEMORY, "dataset of %zu bytes does not fit the arena now", bytes);
    Dataset D;
    D.live = true;
    D.off = off;
    D.bytes = bytes;
    D.X = reinterpret_cast<float*>(s->d_arena + off);
    D.y = reinterpret_cast<float*>(s->d_arena + off + xb);
    D.n_vars = n_vars;
    D.n_cases = n_cases;
    D.tax = tax_on_length;
    hipError_t e = hipSuccess;
    if (n_vars > 0)
        e = hipMemcpy2DAsync(D.X, (size_t)n_cases * 4, X, (size_t)ld_x * 4, (size_t)n_cases * 4,
                             (size_t)n_vars, hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess)
        e = hipMemcpyAsync(D.y, y, (size_t)n_cases * 4, hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = hipStreamSynchronize(s->up);
    if (e != hipSuccess) {
        s->dev.release(off, bytes);
        return fail(GP_E_HIP, "dataset upload: %s", hipGetErrorString(e));
    }
    int id = -1;
    for (size_t i = 0; i < s->datasets.size(); ++i)
        if (!s->datasets[i].live) { id = (int)i; break; }
    if (id < 0) {
        id = (int)s->datasets.size();
        s->datasets.push_back(D);
    } else {
        s->datasets[(size_t)id] = D;
    }
    *dataset_id = id;
    return GP_OK;
}

int gp_server_remove_dataset(gp_server* s, int32_t id)
{
    if (!s) return fail(GP_E_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int)s->datasets.size() || !s->datasets[(size_t)id].live)
        return fail(GP_E_INVALID_ARG, "unknown dataset %d", id);
    Dataset& D = s->datasets[(size_t)id];
    if (D.pending) return fail(GP_E_INVALID_ARG, "dataset %d has %d pending requests", id, D.pending);
    s->dev.release(D.off, D.bytes);
    D = Dataset();
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
    auto R = std::make_shared<Request>();
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
    if (s->broken != GP_OK) return fail(s->broken, "server stopped after a device error");
    if (s->stop) return fail(GP_E_INVALID_ARG, "server is shutting down");
    if (id < 0 || id >= (int)s->datasets.size() || !s->datasets[(size_t)id].live)
        return fail(GP_E_INVALID_ARG, "unknown dataset %d", id);
    const Dataset& D = s->datasets[(size_t)id];
    R->node_evals = (double)(offsets[n_programs] - offsets[0]) * (double)D.n_cases;
    split_request(s, *R, D.n_cases);
    size_request(*R);
    if (R->bytes > s->dev.capacity() || R->bytes > s->host.capacity())
        return fail(GP_E_TOO_LARGE, "request needs %zu bytes: more than the budget", R->bytes);
    R->ticket = s->next_ticket++;
    R->t_submit = Clock::now();
    s->datasets[(size_t)id].pending += 1;
    s->live[R->ticket] = R;
    s->waiting.push_back(R);
    s->n_submitted += 1;
    *ticket = R->ticket;
    lk.unlock();
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
    auto have = [&] {
        while (!s->done_q.empty() && !s->done_rc.count(s->done_q.front())) s->done_q.pop_front();
        return !s->done_q.empty();
    };
    if (timeout_ms < 0) s->cv_done.wait(lk, have);
    else if (timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), have);
    int n = 0;
    while (n < max_n && have()) {
        const int64_t t = s->done_q.front();
        s->done_q.pop_front();
        tickets[n] = t;
        results[n] = s->done_rc[t];
        s->done_rc.erase(t);
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
    if (!s->live.count(ticket) && !s->done_rc.count(ticket))
        return fail(GP_E_INVALID_ARG, "unknown or consumed ticket %lld", (long long)ticket);
    auto have = [&] { return s->done_rc.count(ticket) != 0; };
    if (timeout_ms < 0) s->cv_done.wait(lk, have);
    else if (timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), have);
    if (!have()) return GP_OK;
    *done = 1;
    *result = s->done_rc[ticket];
    s->done_rc.erase(ticket);
    return GP_OK;
}

int gp_server_get_stats(gp_server* s, gp_server_stats* out)
{
    if (!s || !out) return fail(GP_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    gp_server_stats r{};
    const auto now = Clock::now();
    r.submitted = s->n_submitted;
    r.completed = s->n_completed;
    r.failed = s->n_failed;
    r.launches = s->n_launches;
    r.chunks_launched = s->n_chunks;
    r.node_evals = s->node_evals;
    r.busy_ms = s->busy_ms + (s->busy_slots ? ms_between(s->busy_since, now) : 0.0);
    r.wall_ms = ms_between(s->t_reset, now);
    r.device_bytes_in_use = (int64_t)s->dev.used();
    r.device_bytes_peak = (int64_t)s->dev.peak();
    r.waiting = (int32_t)s->waiting.size();
    r.in_flight = (int32_t)(s->live.size() - s->waiting.size());
    if (!s->latencies.empty()) {
        std::vector<double> v = s->latencies;
        std::sort(v.begin(), v.end());
        // nearest-rank percentiles
        auto pct = [&](double q) {
            size_t k = (size_t)std::ceil(q * (double)v.size());
            k = k < 1 ? 1 : (k > v.size() ? v.size() : k);
            return v[k - 1];
        };
        r.latency_p50_ms = pct(0.50);
        r.latency_p99_ms = pct(0.99);
        r.latency_max_ms = v.back();
        double sum = 0.0;
        for (double x : v) sum += x;
        r.latency_mean_ms = sum / (double)v.size();
    }
    *out = r;
    return GP_OK;
}

int gp_server_reset_stats(gp_server* s)
{
    if (!s) return fail(GP_E_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    const auto now = Clock::now();
    s->t_reset = now;
    s->n_submitted = s->n_completed = s->n_failed = s->n_launches = s->n_chunks = 0;
    s->node_evals = 0.0;
    s->busy_ms = 0.0;
    if (s->busy_slots) s->busy_since = now;
    s->latencies.clear();
    s->dev.reset_peak();
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
