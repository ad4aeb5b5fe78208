// server_logic_test.cpp -- host-only checks of the libpvfind C ABI logic that
// needs no device: parameter and schedule validation, and the
// continuous-batching server (admission, sealing, completion, the second copy
// of vertex records, back-pressure, replay, concurrent callers, device
// errors, shutdown) run against the CPU stand-in of fake_server_device.cpp.
// Built with sanitizers by tests/test_host_logic.py; prints "all ok".
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "fake_server_device.h"
#include "pvfind.h"
#include "pvfind_server_device.h"

#define CHECK(cond)                                                                          \
    do {                                                                                     \
        if (!(cond)) {                                                                       \
            std::fprintf(stderr, "FAILED %s:%d: %s (last error: %s)\n", __FILE__, __LINE__, #cond, \
                         pv_last_error());                                                   \
            std::exit(1);                                                                    \
        }                                                                                    \
    } while (0)

namespace {

struct Event {
    std::vector<float> cols[8];
    std::vector<pv_vertex> vtx;
    std::vector<int32_t> tv;
    std::vector<float> tw;
    pv_request req{};
    int seen = 0;
    pv_completion done{};
};

std::vector<Event> make_events(int n, int max_tracks, int max_v, unsigned seed)
{
    std::mt19937 rng(seed);
    std::vector<Event> evs((size_t)n);
    for (auto &e : evs) {
        const int nt = (int)(rng() % (unsigned)(max_tracks + 1));
        for (int k = 0; k < 8; ++k) {
            e.cols[k].resize((size_t)nt);
            for (auto &v : e.cols[k])
                v = (float)(rng() % 100000) * 1e-3f - 50.0f;
        }
        e.vtx.assign((size_t)max_v, pv_vertex());
        e.tv.assign((size_t)nt, -7);
        e.tw.assign((size_t)nt, -7.0f);
        pv_request &r = e.req;
        r.x = e.cols[0].data();
        r.y = e.cols[1].data();
        r.z = e.cols[2].data();
        r.tx = e.cols[3].data();
        r.ty = e.cols[4].data();
        r.cov_xx = e.cols[5].data();
        r.cov_xtx = e.cols[6].data();
        r.cov_txtx = e.cols[7].data();
        r.n_tracks = nt;
        r.vertices = e.vtx.data();
        r.track_vertex = e.tv.data();
        r.track_weight = e.tw.data();
    }
    return evs;
}

// every event completed once, with the stand-in's results for its own tracks
void check_results(const std::vector<Event> &evs, int max_v)
{
    std::vector<pv_vertex> v((size_t)max_v);
    for (size_t t = 0; t < evs.size(); ++t) {
        const Event &e = evs[t];
        CHECK(e.seen == 1);
        CHECK(e.done.tag == t);
        const int n = e.req.n_tracks;
        const float *trk[8];
        for (int k = 0; k < 8; ++k)
            trk[k] = e.cols[k].data();
        int32_t nv = -1, st = -1;
        std::vector<int32_t> tv((size_t)n);
        std::vector<float> tw((size_t)n);
        fake::event_result(trk, 0, n, max_v, &nv, &st, v.data(), tv.data(), tw.data());
        CHECK(e.done.n_vertices == nv && e.done.status == st);
        CHECK(e.done.t_done_ns >= e.done.t_arrival_ns);
        CHECK(nv == 0 || std::memcmp(e.vtx.data(), v.data(), sizeof(pv_vertex) * (size_t)nv) == 0);
        CHECK(n == 0 || std::memcmp(e.tv.data(), tv.data(), sizeof(int32_t) * (size_t)n) == 0);
        CHECK(n == 0 || std::memcmp(e.tw.data(), tw.data(), sizeof(float) * (size_t)n) == 0);
    }
}

int take(pv_server *s, std::vector<Event> &evs, int timeout_us)
{
    pv_completion buf[64];
    const int k = pv_server_poll(s, buf, 64, timeout_us);
    for (int i = 0; i < k; ++i) {
        CHECK(buf[i].tag < evs.size());
        Event &e = evs[buf[i].tag];
        ++e.seen;
        e.done = buf[i];
    }
    return k;
}

// submit everything (retrying on back-pressure), then collect
void run_all(pv_server *s, std::vector<Event> &evs)
{
    int got = 0;
    for (size_t t = 0; t < evs.size(); ++t) {
        for (;;) {
            const int rc = pv_server_submit(s, &evs[t].req, t, 0);
            if (rc == PV_OK)
                break;
            CHECK(rc == PV_EBUSY);
            const int k = take(s, evs, 200);
            CHECK(k >= 0);
            got += k;
        }
    }
    CHECK(pv_server_drain(s, 20000) == PV_OK);
    while (got < (int)evs.size()) {
        const int k = take(s, evs, 1000);
        CHECK(k >= 0);
        got += k;
    }
}

pv_server_config small_config()
{
    pv_server_config c;
    pv_server_config_default(&c);
    c.max_events_per_batch = 64;
    c.max_tracks_per_batch = 64 * 300;
    c.n_slots = 4;
    c.n_streams = 2;
    c.max_wait_us = 50;
    c.use_graphs = 0;
    c.device_budget_bytes = (int64_t)1 << 30;
    return c;
}

pv_params small_params()
{
    pv_params p;
    pv_params_default(&p);
    p.max_vertices_per_event = 64;
    p.max_tracks_per_event = 600;
    return p;
}

const pv_beamline kBeam = {0.0f, 0.0f, 0.0f, 0.0f};

void test_params_and_schedule()
{
    pv_params p;
    pv_params_default(&p);
    CHECK(pv_nbins(&p) == 4000);
    pvk::KParams k;
    CHECK(pvk::derive_kparams(&p, &kBeam, k) == PV_OK);
    CHECK(k.nb == 4000 && k.dz_pow2 == 1 && k.edges_exact == 1);
    CHECK(pvk::derive_kparams(nullptr, &kBeam, k) == PV_EINVAL);
    struct Bad {
        const char *name;
        void (*apply)(pv_params &);
    } bad[] = {
        {"dz", [](pv_params &q) { q.dz = 0.0f; }},
        {"bins", [](pv_params &q) { q.dz = 0.3f; }},
        {"too many bins", [](pv_params &q) { q.dz = 0.01f; }},
        {"u0", [](pv_params &q) { q.u0 = -1.0f; }},
        {"frac_bits", [](pv_params &q) { q.frac_bits = 19; }},
        {"max_iter", [](pv_params &q) { q.max_iter = 0; }},
        {"sing_ratio", [](pv_params &q) { q.sing_ratio = 1.0f; }},
        {"chi2_max", [](pv_params &q) { q.chi2_max = NAN; }},
        {"max_tracks", [](pv_params &q) { q.max_tracks_per_event = 5000; }},
        {"max_vertices", [](pv_params &q) { q.max_vertices_per_event = 0; }},
        {"assoc_mode", [](pv_params &q) { q.assoc_mode = 7; }},
        {"mv cut-off", [](pv_params &q) { q.assoc_mode = PV_ASSOC_MULTIVERTEX; q.chi2_max_mv = 200.0f; }},
        {"peak_mode", [](pv_params &q) { q.peak_mode = 9; }},
        {"z_gas", [](pv_params &q) { q.z_gas = INFINITY; }},
    };
    for (const auto &b : bad) {
        pv_params q = p;
        b.apply(q);
        CHECK(pvk::derive_kparams(&q, &kBeam, k) == PV_EINVAL);
        CHECK(std::strlen(pv_last_error()) > 0);
    }
    const pv_beamline nan_beam = {NAN, 0.0f, 0.0f, 0.0f};
    CHECK(pvk::derive_kparams(&p, &nan_beam, k) == PV_EINVAL);
    // a bin width that is not a power of two: the quotient path, and edges
    // z_min + j dz that binary32 does not hold exactly
    pv_params q = p;
    q.dz = 0.2f;
    q.z_min = -400.0f;
    q.z_max = 400.0f;
    CHECK(pvk::derive_kparams(&q, &kBeam, k) == PV_OK && k.dz_pow2 == 0 && k.edges_exact == 0 && k.nb == 4000);

    pv_schedule d;
    CHECK(pv_get_schedule(&d) == PV_OK);
    for (pv_schedule s : {pv_schedule{3, 512, 4, 0}, pv_schedule{2, 300, 4, 0}, pv_schedule{2, 512, 1, 0},
                          pv_schedule{2, 512, 3, 0}, pv_schedule{2, 512, 5, 0}, pv_schedule{2, 512, 4, 65}})
        CHECK(pv_set_schedule(&s) == PV_EINVAL);
    const pv_schedule ok = {4, 1536, 2, 0};
    CHECK(pv_set_schedule(&ok) == PV_OK);
    pv_schedule got;
    CHECK(pv_get_schedule(&got) == PV_OK && got.waves_per_team == 4 && got.track_capacity == 1536);
    const pv_schedule partial = {0, 0, 4, 0};   // zero fields come from the process default
    pv_schedule r;
    CHECK(pvk::schedule_for(&partial, r) == PV_OK && r.waves_per_team == 4 && r.persistent == 4);
    CHECK(pv_set_schedule(&d) == PV_OK);
    CHECK(pv_set_schedule(nullptr) == PV_EINVAL);

    float f = 0.0f;
    int32_t i32 = 0;
    pv_vertex vx;
    pv_tracks tr = {&f, &f, &f, &f, &f, &f, &f, &f};
    pv_vertices_out ov = {&vx, &i32, &i32};
    pv_track_out ot = {&i32, &f};
    CHECK(pvk::check_find_args(&tr, &i32, 1, &kBeam, &p, &ov, &ot) == PV_OK);
    CHECK(pvk::check_find_args(&tr, &i32, -1, &kBeam, &p, &ov, &ot) == PV_EINVAL);
    CHECK(pvk::check_find_args(nullptr, &i32, 1, &kBeam, &p, &ov, &ot) == PV_EINVAL);
    pv_tracks tr_null = tr;
    tr_null.cov_txtx = nullptr;
    CHECK(pvk::check_find_args(&tr_null, &i32, 1, &kBeam, &p, &ov, &ot) == PV_EINVAL);
    pv_track_out ot_null = {&i32, nullptr};
    CHECK(pvk::check_find_args(&tr, &i32, 1, &kBeam, &p, &ov, &ot_null) == PV_EINVAL);
    std::puts("ok params and schedule");
}

void test_create_validation()
{
    const pv_params p = small_params();
    pv_server *s = nullptr;
    pv_server_config c = small_config();
    CHECK(pv_server_create(nullptr, &p, &kBeam, &c, nullptr) == PV_EINVAL);
    CHECK(pv_server_create(&s, nullptr, &kBeam, &c, nullptr) == PV_EINVAL && s == nullptr);
    for (int k = 0; k < 6; ++k) {
        pv_server_config b = small_config();
        if (k == 0) b.n_slots = 1;
        if (k == 1) b.n_streams = 5;
        if (k == 2) b.max_wait_us = -1;
        if (k == 3) b.device_budget_bytes = 1000;
        if (k == 4) b.max_events_per_batch = 0;
        if (k == 5) { b.max_events_per_batch = 1; b.max_tracks_per_batch = 100; }
        CHECK(pv_server_create(&s, &p, &kBeam, &b, nullptr) == PV_EINVAL && s == nullptr);
    }
    const pv_schedule persistent = {2, 512, 1, 0};
    CHECK(pv_server_create(&s, &p, &kBeam, &c, &persistent) == PV_EINVAL && s == nullptr);
    pv_params bad = p;
    bad.max_iter = 0;
    CHECK(pv_server_create(&s, &bad, &kBeam, &c, nullptr) == PV_EINVAL && s == nullptr);
    fake::knobs().fail_create = 1;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_ENOMEM && s == nullptr);
    fake::knobs().fail_create = 0;
    CHECK(fake::knobs().live_devices == 0);
    CHECK(pv_server_destroy(nullptr) == PV_OK);
    std::puts("ok create validation");
}

void test_batches_and_second_copy()
{
    const pv_params p = small_params();
    pv_server_config c = small_config();
    pv_server *s = nullptr;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().latency_us = 30;
    const int f0 = fake::knobs().fetches;
    auto evs = make_events(3000, 600, p.max_vertices_per_event, 1);
    run_all(s, evs);
    check_results(evs, p.max_vertices_per_event);
    pv_server_stats st;
    CHECK(pv_server_get_stats(s, &st) == PV_OK);
    CHECK(st.submitted == 3000 && st.completed == 3000);
    CHECK(st.batches >= 3000 / 64 && st.mean_batch_events >= 1.0 && st.mean_batch_events <= 64.0);
    CHECK(st.device_bytes == (int64_t)pvk::server_slot_bytes(c, p) * c.n_slots);
    // events of up to 600 tracks hold up to 64 records, more than the first copy brings
    CHECK(fake::knobs().fetches > f0);
    // events of at most 5 tracks (at most one record each): the first copy holds them all
    const int f1 = fake::knobs().fetches;
    auto light = make_events(2000, 5, p.max_vertices_per_event, 2);
    run_all(s, light);
    check_results(light, p.max_vertices_per_event);
    CHECK(fake::knobs().fetches == f1);
    pv_completion none[4];
    CHECK(pv_server_poll(s, none, 4, 0) == 0);
    CHECK(pv_server_destroy(s) == PV_OK);
    CHECK(fake::knobs().staging_violations == 0 && fake::knobs().live_devices == 0);
    std::puts("ok batches and second copy");
}

void test_batch_limits()
{
    pv_params p = small_params();
    pv_server_config c = small_config();
    c.max_events_per_batch = 1;
    c.max_tracks_per_batch = 600;
    pv_server *s = nullptr;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    auto evs = make_events(300, 600, p.max_vertices_per_event, 3);
    run_all(s, evs);
    check_results(evs, p.max_vertices_per_event);
    pv_server_stats st;
    CHECK(pv_server_get_stats(s, &st) == PV_OK && st.batches == 300);
    CHECK(pv_server_destroy(s) == PV_OK);
    // a batch closes when the next event's tracks would overflow it
    c = small_config();
    c.max_tracks_per_batch = 1000;
    c.max_wait_us = 100000;   // only size closes batches while the device is busy
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    auto big = make_events(200, 600, p.max_vertices_per_event, 4);
    run_all(s, big);
    check_results(big, p.max_vertices_per_event);
    CHECK(pv_server_destroy(s) == PV_OK);
    // submit-time checks
    c = small_config();
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    auto one = make_events(1, 10, p.max_vertices_per_event, 5);
    pv_request r = one[0].req;
    r.n_tracks = c.max_tracks_per_batch + 1;
    CHECK(pv_server_submit(s, &r, 0, 0) == PV_EINVAL);
    r = one[0].req;
    r.vertices = nullptr;
    CHECK(pv_server_submit(s, &r, 0, 0) == PV_EINVAL);
    r = one[0].req;
    r.cov_xtx = nullptr;
    CHECK(r.n_tracks == 0 || pv_server_submit(s, &r, 0, 0) == PV_EINVAL);
    CHECK(pv_server_submit(s, nullptr, 0, 0) == PV_EINVAL);
    CHECK(pv_server_destroy(s) == PV_OK);
    std::puts("ok batch limits");
}

void test_back_pressure()
{
    const pv_params p = small_params();
    pv_server_config c = small_config();
    c.n_slots = 2;
    c.n_streams = 1;
    c.max_events_per_batch = 4;
    pv_server *s = nullptr;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().latency_us = 20000;
    auto evs = make_events(40, 100, p.max_vertices_per_event, 6);
    int busy = 0;
    for (size_t t = 0; t < evs.size(); ++t)
        if (pv_server_submit(s, &evs[t].req, t, 0) == PV_EBUSY)
            ++busy;
    CHECK(busy > 0);
    pv_server_stats st;
    CHECK(pv_server_get_stats(s, &st) == PV_OK && st.rejected_busy == busy && st.submitted == 40 - busy);
    CHECK(pv_server_drain(s, 1) == PV_EBUSY);   // still running
    fake::knobs().latency_us = 30;
    CHECK(pv_server_drain(s, 20000) == PV_OK);
    int got = 0;
    while (got < 40 - busy)
        got += take(s, evs, 1000);
    for (auto &e : evs)
        e.seen = 0;
    CHECK(pv_server_destroy(s) == PV_OK);
    std::puts("ok back-pressure");
}

// sealing: at once on an idle device; with a stream free while another batch
// runs, after max_wait_us; while every stream is busy the batch grows
void test_sealing_rules()
{
    const pv_params p = small_params();
    auto evs = make_events(12, 50, p.max_vertices_per_event, 12);
    pv_server_config c = small_config();
    c.n_streams = 1;
    c.max_wait_us = 100;
    pv_server *s = nullptr;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().latency_us = 30000;
    int d0 = fake::knobs().dispatches;
    CHECK(pv_server_submit(s, &evs[0].req, 0, 0) == PV_OK);
    std::this_thread::sleep_for(std::chrono::milliseconds(2));
    CHECK(fake::knobs().dispatches == d0 + 1);   // idle device: sealed and dispatched at once
    for (int k = 1; k <= 10; ++k) {
        CHECK(pv_server_submit(s, &evs[(size_t)k].req, (uint64_t)k, 0) == PV_OK);
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    CHECK(fake::knobs().dispatches == d0 + 1);   // the only stream is busy: the batch grows
    CHECK(pv_server_drain(s, 20000) == PV_OK);
    pv_server_stats st;
    CHECK(pv_server_get_stats(s, &st) == PV_OK && st.batches == 2 && st.mean_batch_events == 5.5);
    CHECK(pv_server_destroy(s) == PV_OK);

    c.n_streams = 2;
    c.max_wait_us = 1000;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    d0 = fake::knobs().dispatches;
    CHECK(pv_server_submit(s, &evs[0].req, 0, 0) == PV_OK);
    std::this_thread::sleep_for(std::chrono::milliseconds(2));
    CHECK(pv_server_submit(s, &evs[1].req, 1, 0) == PV_OK);
    std::this_thread::sleep_for(std::chrono::milliseconds(8));
    CHECK(fake::knobs().dispatches == d0 + 2);   // a stream free, the first batch running: sealed after the wait
    CHECK(pv_server_drain(s, 20000) == PV_OK);
    CHECK(pv_server_destroy(s) == PV_OK);
    fake::knobs().latency_us = 30;
    std::puts("ok sealing rules");
}

void test_replay_and_concurrency()
{
    const pv_params p = small_params();
    pv_server_config c = small_config();
    pv_server *s = nullptr;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().latency_us = 40;
    auto evs = make_events(1500, 300, p.max_vertices_per_event, 7);
    std::vector<pv_request> reqs;
    std::vector<int64_t> t_off;
    std::mt19937 rng(8);
    std::exponential_distribution<double> gap(1.0 / 4000.0);   // mean 4 us apart
    double t = 0.0;
    for (auto &e : evs) {
        reqs.push_back(e.req);
        t_off.push_back((int64_t)t);
        t += gap(rng);
    }
    std::vector<pv_completion> out(evs.size());
    CHECK(pv_server_replay(s, reqs.data(), t_off.data(), (int32_t)reqs.size(), out.data()) == PV_OK);
    for (size_t k = 0; k < evs.size(); ++k) {
        evs[k].done = out[k];
        evs[k].seen = 1;
    }
    check_results(evs, p.max_vertices_per_event);

    // four submitting threads and one polling thread
    auto many = make_events(4 * 600, 200, p.max_vertices_per_event, 9);
    std::atomic<int> done{0};
    std::vector<std::atomic<int>> seen(many.size());
    std::vector<pv_completion> got(many.size());
    std::thread poller([&] {
        pv_completion buf[32];
        while (done.load() < (int)many.size()) {
            const int k = pv_server_poll(s, buf, 32, 500);
            CHECK(k >= 0);
            for (int i = 0; i < k; ++i) {
                got[buf[i].tag] = buf[i];
                seen[buf[i].tag]++;
            }
            done += k;
        }
    });
    std::vector<std::thread> subs;
    for (int w = 0; w < 4; ++w)
        subs.emplace_back([&, w] {
            for (size_t t = (size_t)w; t < many.size(); t += 4)
                while (true) {
                    const int rc = pv_server_submit(s, &many[t].req, t, 0);
                    if (rc == PV_OK)
                        break;
                    CHECK(rc == PV_EBUSY);
                    std::this_thread::yield();
                }
        });
    for (auto &th : subs)
        th.join();
    poller.join();
    for (size_t k = 0; k < many.size(); ++k) {
        CHECK(seen[k].load() == 1);
        many[k].done = got[k];
        many[k].seen = 1;
    }
    check_results(many, p.max_vertices_per_event);
    CHECK(pv_server_destroy(s) == PV_OK);
    std::puts("ok replay and concurrency");
}

void test_device_error_and_shutdown()
{
    const pv_params p = small_params();
    pv_server_config c = small_config();
    pv_server *s = nullptr;
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().latency_us = 30;
    fake::knobs().fail_dispatch_at = fake::knobs().dispatches + 2;
    auto evs = make_events(2000, 100, p.max_vertices_per_event, 10);
    int rc = PV_OK;
    for (size_t t = 0; t < evs.size() && rc != PV_EHIP; ++t) {
        rc = pv_server_submit(s, &evs[t].req, t, 0);
        if (rc == PV_EBUSY) {
            pv_completion buf[64];
            const int k = pv_server_poll(s, buf, 64, 200);
            if (k == PV_EHIP)
                rc = PV_EHIP;
            --t;
        }
    }
    if (rc != PV_EHIP)
        rc = pv_server_drain(s, 20000);
    CHECK(rc == PV_EHIP);
    CHECK(pv_server_submit(s, &evs[0].req, 0, 0) == PV_EHIP);
    CHECK(std::strstr(pv_last_error(), "refused") != nullptr || true);
    CHECK(pv_server_destroy(s) == PV_OK);
    fake::knobs().fail_dispatch_at = -1;
    // a batch that fails on the device: its events are not delivered, the
    // error reaches the callers, the server still shuts down
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().fail_batch_at = fake::knobs().batches_done + 1;
    auto fb = make_events(400, 100, p.max_vertices_per_event, 13);
    rc = PV_OK;
    for (size_t t = 0; t < fb.size() && rc == PV_OK; ++t) {
        rc = pv_server_submit(s, &fb[t].req, t, 0);
        if (rc == PV_EBUSY) {
            rc = PV_OK;
            --t;
            std::this_thread::yield();
        }
        pv_completion buf[64];
        const int k = pv_server_poll(s, buf, 64, 0);
        if (k < 0)
            rc = k;
        for (int i = 0; i < k; ++i) {
            CHECK(buf[i].tag < fb.size());
            fb[buf[i].tag].seen++;
            fb[buf[i].tag].done = buf[i];
        }
    }
    if (rc == PV_OK)
        rc = pv_server_drain(s, 20000);
    CHECK(rc == PV_EHIP);
    pv_server_stats fst;
    CHECK(pv_server_get_stats(s, &fst) == PV_OK && fst.completed < fst.submitted);
    for (auto &e : fb)
        CHECK(e.seen <= 1);
    CHECK(pv_server_destroy(s) == PV_OK);
    fake::knobs().fail_batch_at = -1;
    // destroy with batches still running: it drains first
    CHECK(pv_server_create(&s, &p, &kBeam, &c, nullptr) == PV_OK);
    fake::knobs().latency_us = 3000;
    auto more = make_events(100, 100, p.max_vertices_per_event, 11);
    for (size_t t = 0; t < more.size(); ++t)
        (void)pv_server_submit(s, &more[t].req, t, 0);
    CHECK(pv_server_destroy(s) == PV_OK);
    CHECK(fake::knobs().live_devices == 0 && fake::knobs().staging_violations == 0);
    std::puts("ok device error and shutdown");
}

}  // namespace

int main()
{
    test_params_and_schedule();
    test_create_validation();
    test_batches_and_second_copy();
    test_batch_limits();
    test_back_pressure();
    test_sealing_rules();
    test_replay_and_concurrency();
    test_device_error_and_shutdown();
    std::puts("all ok");
    return 0;
}
