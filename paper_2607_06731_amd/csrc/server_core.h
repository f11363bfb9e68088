// server_core.h -- the scheduling policy of the scoring service, with no
// device call in it: admission against the device and staging budgets,
// chunking, batch formation (continuous batching over several launch
// slots), completion, failure isolation and cancellation.
//
// The device side is a template parameter `Dev` (server.cpp: HIP streams,
// events and gp_eval_batched; tests/server_harness.cpp: a simulated device
// on a fake clock).  Dev provides
//   double now_ms();                                   clock
//   int    upload(Request&);                           stage + queue the copy up
//   int    launch(int slot, const Batch&);             enqueue one batch
//   int    poll(int slot);                             1 done, 0 running, <0 error
//   void   deliver(Request&);                          results -> caller arrays
//   void   release_upload(Request&);                   drop the upload handle
//   size_t workspace_bytes(P, N, n_req, n_ds, max_vars, max_cases);
// A Core is driven by one thread (the scheduler); the caller serializes
// every call into it.
//
// Failure isolation: when a launch fails (at enqueue or when polled), each
// request it held is retried alone once (its chunks in launches of its own,
// a new generation: results of older launches are ignored); a request that
// fails again completes with the error, the others are unaffected.
// Cancellation: a request that has not started completes at once with
// GP_E_CANCELLED; one with chunks in flight launches no further chunk and
// completes with GP_E_CANCELLED when they drain (its results are not
// delivered).  A request's device and staging blocks are released only
// when no launch holds any of its chunks.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <unordered_map>
#include <utility>
#include <vector>

namespace gpsrv {

constexpr size_t kAlign = 256;
constexpr int kMaxStreams = 8;
constexpr int kMaxBatch = 4096;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

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
    double t_submit_ms = 0.0;
    std::vector<Chunk> chunks;
    size_t next_chunk = 0;
    size_t bytes = 0, o_offs = 0, o_consts = 0, o_out = 0, o_st = 0;
    size_t dev_off = 0, host_off = 0;
    bool admitted = false;              // holds device and staging blocks
    void* upload = nullptr;             // the device's handle of the upload
    // (slot, launch sequence) of launches holding earlier chunks of this
    // generation: the launch holding the last chunk waits for them
    std::vector<std::pair<int, uint64_t>> batches;
    int in_flight = 0;                  // launches (any generation) holding its chunks
    uint32_t gen = 0;                   // launches of older generations are ignored
    bool solo = false;                  // retried: its chunks launch alone
    bool cancelled = false;
    int failed_rc = 0;                  // final error, set when the retry failed too
};

using ReqPtr = std::shared_ptr<Request>;

struct Dataset {
    bool live = false;
    size_t off = 0, bytes = 0;
    float* X = nullptr;                 // device addresses (unused by the core)
    float* y = nullptr;
    int32_t n_vars = 0;
    int64_t n_cases = 0;
    double tax = 0.0;
    int pending = 0;
};

struct Entry {
    Request* R;
    size_t chunk;
};

// One launch as the device sees it.
struct Batch {
    std::vector<Entry> ent;
    std::vector<int32_t> ds_list;       // datasets of the launch, in table order
    std::vector<int> ds_local;          // dataset id -> index in ds_list (or -1)
    std::vector<Request*> touched;      // requests with a chunk in it (wait on their uploads)
    std::vector<ReqPtr> finishing;      // requests whose last chunk it holds (copy back)
    std::vector<std::pair<int, uint64_t>> waits;   // earlier launches the copy-back waits for
    int64_t P = 0, N = 0;
    int32_t max_vars = 0;
    int64_t max_cases = 1;
};

struct Slot {
    bool busy = false;
    uint64_t seq = 0;
    std::vector<ReqPtr> finishing;
    std::vector<std::pair<ReqPtr, uint32_t>> members;   // (request, generation)
    double t_launch_ms = 0.0;
};

struct Config {
    int64_t chunk_node_evals = int64_t(1) << 35;
    int64_t batch_node_evals = int64_t(1) << 37;
    int32_t n_streams = 2;
    int32_t max_batch_chunks = 1024;
    int32_t one_launch_per_request = 0;
    size_t ws_cap = 0;                  // workspace per launch slot
    // linear model of the workspace (for chunking)
    double ws_fixed = 0.0, ws_per_prog = 0.0, ws_per_node = 0.0;
};

enum : int { kCoreOk = 0, kCoreCancelled = -6 };

template <class Dev>
struct Core {
    Dev& dev;
    Config cfg;
    Arena darena, harena;
    std::vector<Slot> slots;
    std::vector<Dataset> datasets;
    std::deque<ReqPtr> waiting;         // submitted, not admitted
    std::deque<ReqPtr> ready;           // admitted, chunks left to launch
    std::unordered_map<int64_t, ReqPtr> live;
    std::vector<ReqPtr> draining;       // failed or cancelled, launches still hold chunks
    std::deque<int64_t> done_q;
    std::unordered_map<int64_t, int> done_rc;
    int64_t next_ticket = 1;
    // statistics since creation / reset
    double t_reset_ms = 0.0;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_cancelled = 0, n_retried = 0;
    int64_t n_launches = 0, n_chunks = 0;
    double node_evals = 0.0, busy_ms = 0.0;
    int busy_slots = 0;
    double busy_since_ms = 0.0;
    std::vector<double> latencies;

    Core(Dev& d, const Config& c, size_t device_bytes, size_t staging_bytes) : dev(d), cfg(c)
    {
        darena.init(device_bytes);
        harena.init(staging_bytes);
        slots.resize((size_t)std::max(1, c.n_streams));
        t_reset_ms = dev.now_ms();
    }

    // Bytes of a request's block and its section offsets.
    static void size_request(Request& R)
    {
        size_t off = align_up((size_t)R.n_nodes * 4);
        R.o_offs = off;
        off = align_up(off + (size_t)(R.P + (int64_t)R.chunks.size()) * 8);
        R.o_consts = off;
        off = align_up(off + (size_t)R.n_consts * 4);
        R.o_out = off;
        off += (size_t)R.P * 8;         // fitness and status are adjacent: one copy back
        R.o_st = off;
        off = align_up(off + (size_t)R.P * 4);
        R.bytes = off;
    }

    // Program ranges of at most chunk_node_evals work and ws_cap workspace
    // each (one range in comparison mode).
    void split_request(Request& R, int64_t n_cases) const
    {
        R.chunks.clear();
        if (cfg.one_launch_per_request || R.P == 0) {
            R.chunks.push_back({0, R.P});
            return;
        }
        const double cap = (double)cfg.chunk_node_evals;
        int64_t b = 0;
        while (b < R.P) {
            int64_t e = b;
            double ev = 0.0;
            while (e < R.P) {
                const double len = (double)(R.offsets[e + 1] - R.offsets[e]);
                const double w = len * (double)n_cases;
                const double ws = cfg.ws_fixed + cfg.ws_per_prog * (double)(e + 1 - b) +
                                  cfg.ws_per_node * (double)(R.offsets[e + 1] - R.offsets[b]);
                if (e > b && (ev + w > cap || ws > (double)cfg.ws_cap)) break;
                ev += w;
                ++e;
            }
            R.chunks.push_back({b, e});
            b = e;
        }
    }

    // Queues a validated request; returns 0, or -3 (GP_E_TOO_LARGE) when it
    // could never fit the budgets.
    int submit(const ReqPtr& R, int64_t* ticket)
    {
        Dataset& D = datasets[(size_t)R->ds];
        R->node_evals = (double)(R->offsets[R->P] - R->offsets[0]) * (double)D.n_cases;
        split_request(*R, D.n_cases);
        size_request(*R);
        if (R->bytes > darena.capacity() || R->bytes > harena.capacity()) return -3;
        R->ticket = next_ticket++;
        R->t_submit_ms = dev.now_ms();
        D.pending += 1;
        live[R->ticket] = R;
        waiting.push_back(R);
        n_submitted += 1;
        *ticket = R->ticket;
        return kCoreOk;
    }

    void release_blocks(Request& R)
    {
        if (R.admitted) {
            darena.release(R.dev_off, R.bytes);
            harena.release(R.host_off, R.bytes);
            R.admitted = false;
        }
        if (R.upload) dev.release_upload(R);
        R.upload = nullptr;
    }

    void complete(const ReqPtr& R, int rc)
    {
        const double now = dev.now_ms();
        if (rc == kCoreOk) {
            dev.deliver(*R);
            n_completed += 1;
            node_evals += R->node_evals;
            latencies.push_back(now - R->t_submit_ms);
        } else if (rc == kCoreCancelled) {
            n_cancelled += 1;
        } else {
            n_failed += 1;
        }
        release_blocks(*R);
        datasets[(size_t)R->ds].pending -= 1;
        live.erase(R->ticket);
        done_q.push_back(R->ticket);
        done_rc[R->ticket] = rc;
    }

    static void drop(std::deque<ReqPtr>& q, const Request* R)
    {
        for (auto it = q.begin(); it != q.end(); ++it)
            if (it->get() == R) { q.erase(it); return; }
    }

    // A failed or cancelled request completes once no launch holds its
    // chunks (their kernels may still write its output block).
    void settle(const ReqPtr& R)
    {
        if (R->in_flight > 0) {
            if (std::find(draining.begin(), draining.end(), R) == draining.end())
                draining.push_back(R);
            return;
        }
        draining.erase(std::remove(draining.begin(), draining.end(), R), draining.end());
        complete(R, R->cancelled ? kCoreCancelled : R->failed_rc);
    }

    // A launch holding chunks of R failed with rc.
    void fail_request(const ReqPtr& R, uint32_t gen, int rc)
    {
        if (!live.count(R->ticket) || gen != R->gen) return;   // done, or an old generation
        if (R->cancelled || R->failed_rc) return;               // already settling
        if (!R->solo) {
            // first failure: a new generation, launched alone
            R->solo = true;
            R->gen += 1;
            R->next_chunk = 0;
            R->batches.clear();
            n_retried += 1;
            drop(ready, R.get());
            ready.push_front(R);
            return;
        }
        R->failed_rc = rc;
        drop(ready, R.get());
        settle(R);
    }

    // Cancels a request: 0, or -1 (GP_E_INVALID_ARG) for an unknown,
    // completed or already cancelled ticket.
    int cancel(int64_t ticket)
    {
        auto it = live.find(ticket);
        if (it == live.end()) return -1;
        const ReqPtr R = it->second;
        if (R->cancelled || R->failed_rc) return -1;
        R->cancelled = true;
        drop(waiting, R.get());
        drop(ready, R.get());
        settle(R);
        return kCoreOk;
    }

    // Admits every waiting request that fits, oldest first.
    bool admit()
    {
        bool progress = false;
        while (!waiting.empty()) {
            const ReqPtr R = waiting.front();
            size_t od = 0, oh = 0;
            if (!darena.alloc(R->bytes, &od)) break;
            if (!harena.alloc(R->bytes, &oh)) {
                darena.release(od, R->bytes);
                break;
            }
            R->dev_off = od;
            R->host_off = oh;
            R->admitted = true;
            waiting.pop_front();
            progress = true;
            const int rc = dev.upload(*R);
            if (rc != kCoreOk) {
                // nothing launched yet: the request fails alone
                R->solo = true;
                R->failed_rc = rc;
                settle(R);
                continue;
            }
            ready.push_back(R);
        }
        return progress;
    }

    // Forms the next batch for slot si and enqueues it; true if launched.
    bool launch(int si)
    {
        Slot& S = slots[(size_t)si];
        Batch B;
        B.ds_local.assign(datasets.size(), -1);
        double work = 0.0;
        const int max_chunks = cfg.one_launch_per_request ? 1 : cfg.max_batch_chunks;
        const double max_work = (double)cfg.batch_node_evals;

        auto take = [&](Request* R) -> bool {
            if ((int)B.ent.size() >= max_chunks) return false;
            const Chunk c = R->chunks[R->next_chunk];
            const Dataset& D = datasets[(size_t)R->ds];
            const int64_t cn = R->offsets[c.e] - R->offsets[c.b];
            const double cw = (double)cn * (double)D.n_cases;
            if (!B.ent.empty()) {
                if (work + cw > max_work) return false;
                const int nds = (int)B.ds_list.size() + (B.ds_local[(size_t)R->ds] < 0 ? 1 : 0);
                const size_t ws = dev.workspace_bytes(B.P + (c.e - c.b), B.N + cn,
                                                      (int32_t)B.ent.size() + 1, nds,
                                                      std::max(B.max_vars, D.n_vars),
                                                      std::max(B.max_cases, D.n_cases));
                if (ws > cfg.ws_cap) return false;
            }
            if (B.ds_local[(size_t)R->ds] < 0) {
                B.ds_local[(size_t)R->ds] = (int)B.ds_list.size();
                B.ds_list.push_back(R->ds);
            }
            B.ent.push_back({R, R->next_chunk});
            R->next_chunk += 1;
            B.P += c.e - c.b;
            B.N += cn;
            work += cw;
            B.max_vars = std::max(B.max_vars, D.n_vars);
            B.max_cases = std::max(B.max_cases, D.n_cases);
            return true;
        };
        bool full = false;
        if (!ready.empty() && ready.front()->solo) {
            // a retried request launches alone
            Request* R = ready.front().get();
            while (R->next_chunk < R->chunks.size())
                if (!take(R)) break;
        } else {
            // one chunk from every admitted request (oldest first), then fill up
            for (const ReqPtr& R : ready) {
                if (R->solo) continue;
                if (R->next_chunk < R->chunks.size() && !take(R.get())) { full = true; break; }
            }
            for (const ReqPtr& R : ready) {
                if (full) break;
                if (R->solo) continue;
                while (R->next_chunk < R->chunks.size()) {
                    if (!take(R.get())) { full = true; break; }
                }
            }
        }
        if (B.ent.empty()) return false;

        for (const Entry& e : B.ent)
            if (B.touched.empty() || B.touched.back() != e.R) B.touched.push_back(e.R);
        std::sort(B.touched.begin(), B.touched.end());
        B.touched.erase(std::unique(B.touched.begin(), B.touched.end()), B.touched.end());
        for (auto it = ready.begin(); it != ready.end();) {
            if ((*it)->next_chunk == (*it)->chunks.size()) {
                B.finishing.push_back(*it);
                it = ready.erase(it);
            } else {
                ++it;
            }
        }
        S.seq += 1;
        for (const ReqPtr& R : B.finishing)
            for (const auto& b : R->batches) {
                const Slot& O = slots[(size_t)b.first];
                if (b.first != si && O.busy && O.seq == b.second) B.waits.push_back(b);
            }
        // the members, by generation, before the device sees the batch
        std::vector<std::pair<ReqPtr, uint32_t>> members;
        for (Request* R : B.touched) members.push_back({live.at(R->ticket), R->gen});
        const int rc = dev.launch(si, B);
        if (rc != kCoreOk) {
            // nothing of this batch runs: undo, then isolate
            S.seq -= 1;
            for (const auto& m : members) {
                if (!m.first->solo) {
                    // the chunks taken go back; a requeued request starts over
                    if (std::find(ready.begin(), ready.end(), m.first) == ready.end())
                        ready.push_back(m.first);
                }
                fail_request(m.first, m.second, rc);
            }
            return false;
        }
        for (Request* R : B.touched) {
            R->batches.push_back({si, S.seq});
            R->in_flight += 1;
        }
        S.finishing = std::move(B.finishing);
        S.members = std::move(members);
        S.busy = true;
        S.t_launch_ms = dev.now_ms();
        if (busy_slots++ == 0) busy_since_ms = S.t_launch_ms;
        n_launches += 1;
        n_chunks += (int64_t)B.ent.size();
        return true;
    }

    // A launch slot finished (rc 0) or failed (rc < 0).
    void finish(int si, int rc)
    {
        Slot& S = slots[(size_t)si];
        std::vector<std::pair<ReqPtr, uint32_t>> members = std::move(S.members);
        std::vector<ReqPtr> fin = std::move(S.finishing);
        S.members.clear();
        S.finishing.clear();
        S.busy = false;
        if (--busy_slots == 0) busy_ms += dev.now_ms() - busy_since_ms;
        for (auto& m : members) m.first->in_flight -= 1;
        if (rc != kCoreOk) {
            for (auto& m : members) fail_request(m.first, m.second, rc);
        } else {
            for (const ReqPtr& R : fin) {
                if (!live.count(R->ticket) || R->cancelled || R->failed_rc) continue;
                // only the current generation's last chunk finishes a request
                bool current = false;
                for (const auto& m : members)
                    if (m.first == R && m.second == R->gen) current = true;
                if (current) complete(R, kCoreOk);
            }
        }
        // failed or cancelled requests whose last launch just drained
        std::vector<ReqPtr> d = draining;
        for (const ReqPtr& R : d)
            if (R->in_flight == 0 && live.count(R->ticket)) settle(R);
    }

    // One pass of the scheduler: completions, admission, launches.  True
    // when something changed.
    bool step()
    {
        bool progress = false;
        for (int i = 0; i < (int)slots.size(); ++i) {
            if (!slots[(size_t)i].busy) continue;
            const int q = dev.poll(i);
            if (q == 1) {
                finish(i, kCoreOk);
                progress = true;
            } else if (q < 0) {
                finish(i, q);
                progress = true;
            }
        }
        progress = admit() || progress;
        for (int i = 0; i < (int)slots.size(); ++i) {
            if (slots[(size_t)i].busy || ready.empty()) continue;
            if (launch(i)) progress = true;
            else if (!ready.empty()) progress = true;     // a failed enqueue requeued work
        }
        return progress;
    }

    bool idle() const { return busy_slots == 0; }

    // Nearest-rank percentile of the recorded latencies.
    double latency_pct(double q) const
    {
        if (latencies.empty()) return 0.0;
        std::vector<double> v = latencies;
        std::sort(v.begin(), v.end());
        size_t k = (size_t)std::ceil(q * (double)v.size());
        k = k < 1 ? 1 : (k > v.size() ? v.size() : k);
        return v[k - 1];
    }
};

}  // namespace gpsrv
