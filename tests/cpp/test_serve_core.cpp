// Host-only tests of the serving scheduler core with a fake executor: FIFO
// admission by footprint and slots, budget rejection, executor failures,
// continuous batching (late requests join a running batch), drain on
// shutdown. Built with g++ by tests/test_serve_core.py; no GPU involved.
#include <atomic>
#include <cassert>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_2602_12105_amd/csrc/serve_core.hpp"

using namespace dgo::srv;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

struct Fake {
    std::atomic<int> prepared{0}, ticks{0}, finished{0}, released{0};
    std::atomic<int> max_batch{0};
    std::mutex mu;
    std::vector<std::vector<uint64_t>> batches;  // user tags per tick
    int fail_prepare_tag = -1;                   // request user tag whose prepare fails
    int fail_tick_when = -1;                     // tick index that fails
    double tick_sleep = 0.002;
    int64_t footprint(const dgo_request &r) const { return (int64_t)r.nV * 1000; }
    dgo_status prepare(Req &r) {
        if ((int)r.in.user == fail_prepare_tag) return DGO_ERR_NOMEM;
        r.exec = (void *)1;
        prepared++;
        return DGO_OK;
    }
    dgo_status tick(std::vector<Req *> &a, int32_t chunk) {
        const int t = ticks++;
        std::vector<uint64_t> tags;
        for (Req *q : a) {
            tags.push_back(q->in.user);
            q->done_iters = std::min(q->target, q->done_iters + chunk);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            batches.push_back(tags);
        }
        int m = max_batch.load();
        while ((int)a.size() > m && !max_batch.compare_exchange_weak(m, (int)a.size())) {
        }
        std::this_thread::sleep_for(std::chrono::duration<double>(tick_sleep));
        if (t == fail_tick_when) return DGO_ERR_DEVICE;
        return DGO_OK;
    }
    dgo_status finish(Req &r) {
        float *u = r.in.h_u;
        if (u) u[0] = (float)r.done_iters;
        finished++;
        return DGO_OK;
    }
    void release(Req &r) {
        if (r.exec) released++;
        r.exec = nullptr;
    }
};

static dgo_server_opts opts(int slots, int64_t budget, int iters, int chunk) {
    dgo_server_opts o{};
    o.max_slots = slots;
    o.hbm_budget_bytes = budget;
    o.cg_iters = iters;
    o.cg_chunk = chunk;
    o.batched = 1;
    o.prep_threads = 2;
    return o;
}

static dgo_request req(int nV, uint64_t tag, float *u) {
    dgo_request r{};
    r.nV = nV;
    r.k = 1;
    r.nF = 2 * nV;
    r.h_u = u;
    r.user = tag;
    return r;
}

static void test_arena() {
    Arena a(4096);
    int64_t x, y, z;
    CHECK(a.alloc(1000, &x) && x == 0);
    CHECK(a.alloc(1000, &y) && y == 1024);
    CHECK(a.alloc(2048, &z) && z == 2048);
    CHECK(!a.alloc(1, &z));
    a.release(1024, 1000);
    CHECK(a.alloc(256, &z) && z == 1024);
    a.release(0, 1000);
    a.release(1024, 256);
    a.release(2048, 2048);
    CHECK(a.in_use() == 0 && a.pieces() == 1 && a.peak() == 4096);
}

static void test_basic_and_batching() {
    Fake f;
    f.tick_sleep = 0.01;
    Scheduler<Fake> s(f, opts(8, 1 << 30, 10, 2));
    std::vector<float> out(8, -1);
    std::vector<uint64_t> t(8);
    // four requests start together; four more arrive while they run
    for (int i = 0; i < 4; ++i) CHECK(s.submit(req(100, i, &out[i]), &t[i]) == DGO_OK);
    std::this_thread::sleep_for(std::chrono::milliseconds(25));
    for (int i = 4; i < 8; ++i) CHECK(s.submit(req(100, i, &out[i]), &t[i]) == DGO_OK);
    for (int i = 0; i < 8; ++i) {
        dgo_req_stats st;
        CHECK(s.wait(t[i], 10.0, &st) == DGO_OK);
        CHECK(st.iters == 10 && out[i] == 10.0f);
        CHECK(st.t_submit <= st.t_admit && st.t_admit <= st.t_start && st.t_start <= st.t_done);
        CHECK(st.slot >= 0 && st.slot < 8);
    }
    CHECK(f.max_batch.load() <= 8);
    // continuous batching: a later request ran in a tick together with an
    // earlier one still in flight
    bool mixed = false;
    std::lock_guard<std::mutex> lk(f.mu);
    for (auto &b : f.batches) {
        std::set<uint64_t> tags(b.begin(), b.end());
        bool early = false, late = false;
        for (auto x : tags) (x < 4 ? early : late) = true;
        mixed = mixed || (early && late);
    }
    CHECK(mixed);
    dgo_server_counters st;
    s.stats(&st);
    CHECK(st.completed == 8 && st.failed == 0 && st.hbm_in_use == 0 && st.active == 0);
    CHECK(s.wait(t[0], 0.1, nullptr) == DGO_ERR_INVALID_ARG);  // waited once already
}

static void test_budget_and_fifo() {
    Fake f;
    // budget fits one 100-vertex request (100000 B) at a time
    Scheduler<Fake> s(f, opts(8, 150000, 4, 4));
    uint64_t t;
    CHECK(s.submit(req(1000, 99, nullptr), &t) == DGO_ERR_BUDGET);  // can never fit
    std::vector<uint64_t> ts(5);
    for (int i = 0; i < 5; ++i) CHECK(s.submit(req(100, i, nullptr), &ts[i]) == DGO_OK);
    std::vector<double> admit(5);
    for (int i = 0; i < 5; ++i) {
        dgo_req_stats st;
        CHECK(s.wait(ts[i], 10.0, &st) == DGO_OK);
        admit[i] = st.t_admit;
    }
    for (int i = 1; i < 5; ++i) CHECK(admit[i] >= admit[i - 1]);  // FIFO
    CHECK(f.max_batch.load() == 1);  // memory admits one at a time
    dgo_server_counters st;
    s.stats(&st);
    CHECK(st.rejected == 1 && st.completed == 5 && st.hbm_peak <= 150000);
}

static void test_failures() {
    Fake f;
    f.fail_prepare_tag = 2;
    Scheduler<Fake> s(f, opts(4, 1 << 30, 4, 4));
    std::vector<uint64_t> ts(4);
    for (int i = 0; i < 4; ++i) CHECK(s.submit(req(10, i, nullptr), &ts[i]) == DGO_OK);
    for (int i = 0; i < 4; ++i) {
        dgo_req_stats st;
        const dgo_status r = s.wait(ts[i], 10.0, &st);
        CHECK(r == (i == 2 ? DGO_ERR_NOMEM : DGO_OK));
    }
    dgo_server_counters st;
    s.stats(&st);
    CHECK(st.failed == 1 && st.completed == 3 && st.hbm_in_use == 0);
    CHECK(f.released.load() == 3);  // the failed request held nothing
}

static void test_tick_failure_isolated() {
    Fake f;
    f.fail_tick_when = 0;
    f.tick_sleep = 0.01;
    Scheduler<Fake> s(f, opts(1, 1 << 30, 4, 4));  // one slot: each tick one request
    std::vector<uint64_t> ts(3);
    for (int i = 0; i < 3; ++i) CHECK(s.submit(req(10, i, nullptr), &ts[i]) == DGO_OK);
    CHECK(s.wait(ts[0], 10.0, nullptr) == DGO_ERR_DEVICE);
    CHECK(s.wait(ts[1], 10.0, nullptr) == DGO_OK);
    CHECK(s.wait(ts[2], 10.0, nullptr) == DGO_OK);
}

static void test_drain_on_shutdown_and_timeout() {
    Fake f;
    f.tick_sleep = 0.005;
    std::vector<float> out(6, -1);
    {
        Scheduler<Fake> s(f, opts(2, 1 << 30, 6, 2));
        std::vector<uint64_t> ts(6);
        for (int i = 0; i < 6; ++i) CHECK(s.submit(req(10, i, &out[i]), &ts[i]) == DGO_OK);
        CHECK(s.wait(ts[5], 0.0, nullptr) == DGO_ERR_TIMEOUT);
        s.shutdown();  // drains: every queued request still completes
        uint64_t t;
        CHECK(s.submit(req(10, 7, nullptr), &t) == DGO_ERR_SHUTDOWN);
    }
    for (int i = 0; i < 6; ++i) CHECK(out[i] == 6.0f);
    CHECK(f.finished.load() == 6 && f.released.load() == 6);
}

int main() {
    test_arena();
    test_basic_and_batching();
    test_budget_and_fifo();
    test_failures();
    test_tick_failure_isolated();
    test_drain_on_shutdown_and_timeout();
    printf("serve core tests passed\n");
    return 0;
}
