// Host harness for the serving scheduler (paper_2607_06731_amd/csrc/
// server_core.h), built by tests/test_server_core.py with the host
// compiler (also under ASan and UBSan).
//
// TEST INFRASTRUCTURE.  A simulated device on a fake clock stands in for
// the GPU: a launch takes 5 us plus its work at 1e13 node evaluations per
// second, starts when its slot and the launches it waits for are done, and
// "delivers" a known value per program (its length plus 1000 x its
// dataset), so a result in the wrong request, a lost chunk or a double
// delivery shows.  Poisoned requests make every launch holding them fail at
// enqueue or when polled.  After every scheduler step the harness checks
// the bookkeeping: device and staging arenas within capacity and equal to
// the blocks held, no request delivered twice, no cancelled or failed
// request delivered, in-flight counts never negative; at the end every
// request is done and only the datasets hold device memory.
//
// Usage: server_harness SCENARIO SEED.  Prints one line of key=value pairs.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "server_core.h"

using namespace gpsrv;

static int g_check_failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond);  \
            ++g_check_failures;                                                      \
        }                                                                            \
    } while (0)

struct SimLaunch {
    double t_done = 0.0;
    int rc = 0;
    std::vector<Entry> ent;
};

struct MockDev {
    double now = 0.0;
    std::vector<SimLaunch> slot;
    std::set<int64_t> poison_enqueue, poison_poll, poison_upload;   // tickets
    std::map<int64_t, int> deliveries;
    int64_t launches = 0, max_chunks_in_launch = 0;
    double max_launch_work = 0.0;
    std::vector<double> chunk_work;       // work of every launched chunk
    const std::vector<Dataset>* datasets = nullptr;

    double now_ms() const { return now; }
    int upload(Request& R)
    {
        if (poison_upload.count(R.ticket)) return -5;
        R.upload = &R;
        return 0;
    }
    void release_upload(Request&) {}
    size_t workspace_bytes(int64_t P, int64_t N, int32_t n_req, int32_t n_ds, int32_t, int64_t) const
    {
        return 4096 + (size_t)P * 40 + (size_t)N * 8 + (size_t)n_req * 80 + (size_t)n_ds * 40;
    }
    int launch(int si, const Batch& B)
    {
        for (const Entry& e : B.ent)
            if (poison_enqueue.count(e.R->ticket)) return -5;
        double work = 0.0, start = now;
        for (const Entry& e : B.ent) {
            const Chunk c = e.R->chunks[e.chunk];
            const double w = (double)(e.R->offsets[c.e] - e.R->offsets[c.b]) *
                             (double)(*datasets)[(size_t)e.R->ds].n_cases;
            work += w;
            chunk_work.push_back(w);
        }
        for (const auto& w : B.waits) start = std::max(start, slot[(size_t)w.first].t_done);
        SimLaunch L;
        L.t_done = start + 0.005 + work / 1e10;      // ms: 5 us + work at 1e13 / s
        L.rc = 0;
        for (const Entry& e : B.ent)
            if (poison_poll.count(e.R->ticket)) L.rc = -5;
        L.ent = B.ent;
        slot[(size_t)si] = L;
        launches += 1;
        max_chunks_in_launch = std::max<int64_t>(max_chunks_in_launch, (int64_t)B.ent.size());
        max_launch_work = std::max(max_launch_work, work);
        return 0;
    }
    int poll(int si)
    {
        const SimLaunch& L = slot[(size_t)si];
        if (now < L.t_done) return 0;
        return L.rc ? L.rc : 1;
    }
    void deliver(Request& R)
    {
        deliveries[R.ticket] += 1;
        for (int64_t p = 0; p < R.P; ++p)
            R.out_f[p] = (double)(R.offsets[p + 1] - R.offsets[p]) + 1000.0 * R.ds;
    }
    double next_event() const
    {
        double t = 1e300;
        for (const SimLaunch& L : slot)
            if (L.t_done > now) t = std::min(t, L.t_done);
        return t;
    }
};

struct Client {
    std::vector<uint32_t> nodes;
    std::vector<int64_t> offsets;
    std::vector<double> out;
    std::vector<int32_t> st;
    int32_t ds = 0;
    int64_t ticket = 0;
    double t_arrive = 0.0;
    bool submitted = false, poisoned = false, cancel_at_submit = false;
    double cancel_after = -1.0;        // ms after submit
    bool cancel_done = false;
};

static void make_pop(std::mt19937_64& rng, Client& c, int64_t P, int maxlen)
{
    std::uniform_int_distribution<int> L(1, maxlen);
    c.offsets.assign((size_t)P + 1, 0);
    for (int64_t p = 0; p < P; ++p) c.offsets[(size_t)p + 1] = c.offsets[(size_t)p] + L(rng);
    c.nodes.assign((size_t)c.offsets.back(), 0u);
    c.out.assign((size_t)P, -1.0);
    c.st.assign((size_t)P, 0);
}

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    const std::string sc = argv[1];
    std::mt19937_64 rng(std::strtoull(argv[2], nullptr, 10));

    Config cfg;
    cfg.n_streams = 2;
    cfg.max_batch_chunks = 64;
    cfg.chunk_node_evals = int64_t(1) << 22;
    cfg.batch_node_evals = int64_t(1) << 24;
    cfg.ws_cap = 4u << 20;
    cfg.ws_fixed = 4096 + 65536;
    cfg.ws_per_prog = 40;
    cfg.ws_per_node = 8;
    size_t dev_bytes = 64u << 20, host_bytes = 64u << 20;
    int n_clients = 40;
    int64_t max_pop = 4000;
    double arrival_span = 2.0;           // ms
    if (sc == "backpressure") { dev_bytes = 3u << 20; host_bytes = 3u << 20; n_clients = 60; arrival_span = 0.0; }
    if (sc == "oneshot") { cfg.one_launch_per_request = 1; cfg.n_streams = 1; }
    if (sc == "random") { n_clients = 200; dev_bytes = 3u << 20; host_bytes = 2u << 20; arrival_span = 0.1; cfg.n_streams = 3; }

    MockDev dev;
    dev.slot.resize((size_t)cfg.n_streams);
    Core<MockDev> core(dev, cfg, dev_bytes, host_bytes);
    dev.datasets = &core.datasets;

    // datasets: resident blocks in the device arena
    const int n_ds = 4;
    size_t ds_bytes = 0;
    for (int d = 0; d < n_ds; ++d) {
        Dataset D;
        D.live = true;
        D.n_vars = 1 + d;
        D.n_cases = 256 << d;
        D.bytes = align_up((size_t)D.n_vars * (size_t)D.n_cases * 4) + (size_t)D.n_cases * 4;
        CHECK(core.darena.alloc(D.bytes, &D.off));
        ds_bytes += align_up(D.bytes);
        core.datasets.push_back(D);
    }

    std::vector<Client> cl((size_t)n_clients);
    std::uniform_int_distribution<int> dsd(0, n_ds - 1);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    for (int i = 0; i < n_clients; ++i) {
        Client& c = cl[(size_t)i];
        const int64_t P = 1 + (int64_t)std::exp(u01(rng) * std::log((double)max_pop));
        make_pop(rng, c, P, 64);
        c.ds = dsd(rng);
        c.t_arrive = arrival_span * u01(rng);
        if ((sc == "fail_enqueue" || sc == "fail_poll" || sc == "fail_upload") && i % 7 == 3) c.poisoned = true;
        if (sc == "random" && u01(rng) < 0.05) c.poisoned = true;
        if (sc == "cancel") {
            if (i % 5 == 1) c.cancel_at_submit = true;
            if (i % 5 == 2) c.cancel_after = 0.001 + 0.01 * u01(rng);
        }
        if (sc == "random" && u01(rng) < 0.1) c.cancel_after = 0.05 * u01(rng);
    }
    std::map<int64_t, size_t> by_ticket;
    int64_t max_waiting = 0, rejected = 0;
    size_t max_dev_used = 0;
    int steps = 0;
    for (;;) {
        // arrivals
        for (Client& c : cl) {
            if (c.submitted || c.t_arrive > dev.now) continue;
            auto R = std::make_shared<Request>();
            R->nodes = c.nodes.data();
            R->n_nodes = (int64_t)c.nodes.size();
            R->offsets = c.offsets.data();
            R->P = (int64_t)c.out.size();
            R->out_f = c.out.data();
            R->out_st = c.st.data();
            R->ds = c.ds;
            c.submitted = true;
            if (core.submit(R, &c.ticket) != 0) {
                rejected += 1;
                c.ticket = -1;
                continue;
            }
            by_ticket[c.ticket] = (size_t)(&c - cl.data());
            if (c.poisoned) {
                if (sc == "fail_enqueue" || (sc == "random" && (c.ticket & 1))) dev.poison_enqueue.insert(c.ticket);
                else if (sc == "fail_upload") dev.poison_upload.insert(c.ticket);
                else dev.poison_poll.insert(c.ticket);
            }
            if (c.cancel_at_submit) {
                CHECK(core.cancel(c.ticket) == 0);
                CHECK(core.cancel(c.ticket) != 0);           // a second cancel is refused
                c.cancel_done = true;
            }
        }
        // timed cancellations
        for (Client& c : cl) {
            if (!c.submitted || c.ticket <= 0 || c.cancel_done || c.cancel_after < 0) continue;
            if (dev.now < c.t_arrive + c.cancel_after) continue;
            c.cancel_done = true;
            const bool pending = core.live.count(c.ticket) != 0;
            const int rc = core.cancel(c.ticket);
            if (!pending) CHECK(rc != 0);
        }
        const bool progress = core.step();
        ++steps;
        // bookkeeping invariants
        size_t held = ds_bytes;
        for (const auto& kv : core.live) {
            const Request& R = *kv.second;
            CHECK(R.in_flight >= 0);
            if (R.admitted) held += align_up(R.bytes);
        }
        CHECK(core.darena.used() == held);
        CHECK(core.darena.used() <= core.darena.capacity());
        CHECK(core.harena.used() <= core.harena.capacity());
        max_waiting = std::max<int64_t>(max_waiting, (int64_t)core.waiting.size());
        max_dev_used = std::max(max_dev_used, core.darena.used());
        bool all_in = true;
        for (const Client& c : cl) all_in = all_in && c.submitted;
        if (all_in && core.live.empty() && core.idle()) break;
        if (!progress) {
            double t = dev.next_event();
            for (const Client& c : cl) {
                if (!c.submitted) t = std::min(t, c.t_arrive);
                else if (c.ticket > 0 && !c.cancel_done && c.cancel_after >= 0)
                    t = std::min(t, c.t_arrive + c.cancel_after);
            }
            if (t >= 1e300) {
                CHECK(!"scheduler stalled with work left");
                break;
            }
            dev.now = std::max(dev.now, t);
        }
        if (steps > 2000000) {
            CHECK(!"too many steps");
            break;
        }
    }
    // outcomes
    int64_t ok = 0, failed = 0, cancelled = 0, wrong = 0, poisoned_ok = 0, innocent_failed = 0;
    for (const auto& kv : core.done_rc) {
        const Client& c = cl[by_ticket.at(kv.first)];
        const int rc = kv.second;
        const int nd = dev.deliveries.count(kv.first) ? dev.deliveries.at(kv.first) : 0;
        if (rc == 0) {
            ++ok;
            CHECK(nd == 1);
            for (size_t p = 0; p < c.out.size(); ++p) {
                const double want = (double)(c.offsets[p + 1] - c.offsets[p]) + 1000.0 * c.ds;
                if (c.out[p] != want) ++wrong;
            }
            if (c.poisoned) ++poisoned_ok;
        } else {
            CHECK(nd == 0);
            for (double v : c.out) CHECK(v == -1.0);
            if (rc == kCoreCancelled) ++cancelled;
            else {
                ++failed;
                if (!c.poisoned) ++innocent_failed;
            }
        }
    }
    CHECK((int64_t)core.done_rc.size() + rejected == n_clients);
    CHECK(core.live.empty());
    CHECK(core.darena.used() == ds_bytes);
    CHECK(core.harena.used() == 0);
    double max_chunk = 0.0;
    for (double w : dev.chunk_work) max_chunk = std::max(max_chunk, w);
    int64_t n_poisoned = 0;
    for (const Client& c : cl) n_poisoned += c.poisoned;
    std::printf("scenario=%s requests=%d ok=%lld failed=%lld cancelled=%lld rejected=%lld wrong=%lld "
                "poisoned=%lld poisoned_ok=%lld innocent_failed=%lld retried=%lld launches=%lld "
                "max_waiting=%lld max_dev_used=%zu dev_capacity=%zu max_chunks=%lld "
                "max_launch_work=%.0f batch_cap=%lld max_chunk_work=%.0f chunk_cap=%lld "
                "sim_ms=%.4f p50_ms=%.4f p99_ms=%.4f checks_failed=%d\n",
                sc.c_str(), n_clients, (long long)ok, (long long)failed, (long long)cancelled,
                (long long)rejected, (long long)wrong, (long long)n_poisoned, (long long)poisoned_ok,
                (long long)innocent_failed, (long long)core.n_retried, (long long)dev.launches,
                (long long)max_waiting, max_dev_used, core.darena.capacity(),
                (long long)dev.max_chunks_in_launch, dev.max_launch_work,
                (long long)cfg.batch_node_evals, max_chunk, (long long)cfg.chunk_node_evals, dev.now,
                core.latency_pct(0.5), core.latency_pct(0.99), g_check_failures);
    return g_check_failures ? 1 : 0;
}
