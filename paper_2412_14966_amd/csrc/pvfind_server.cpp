// pvfind_server.cpp -- continuous-batching server on top of pv_find: a pool
// of batch slots, admission by free slot, a worker thread that seals,
// dispatches and completes batches on several streams.  The device side of a
// slot (buffers, streams, graphs, launches) sits behind pvk::ServerDevice
// (pvfind_server_hip.cpp); this file holds no device code.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "pvfind_server_device.h"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t tag;
    int64_t t_arrival;
    int32_t n_tracks;
    int32_t first_track;   // within the batch
    pv_vertex *vertices;
    int32_t *track_vertex;
    float *track_weight;
};

enum class SlotState { Free, Open, Sealed, InFlight };

// The vertex records come back in a copy sized before their number is
// known: kDenseBase per event plus one per kDenseTracks tracks, which holds a
// batch's records with room to spare at every pile-up (about one vertex per
// 25 tracks).  A batch with more records gets a second copy of the rest once
// its counts are back, and completes when that copy has; the worker does not
// wait for it.
constexpr size_t kDenseBase = 2;
constexpr size_t kDenseTracks = 16;

struct Slot {
    int id = 0;
    SlotState state = SlotState::Free;
    pvk::SlotHost h;
    int n_events = 0, n_tracks = 0;
    int dense_copied = 0;           // records the batch's first copy-back brings
    bool rest_issued = false;       // the second copy (records past dense_copied) was started
    int rest_rc = PV_OK;            // its start status
    int64_t t_oldest = 0;
    std::vector<Request> reqs;
};

}  // namespace

struct pv_server {
    pv_params params{};
    pv_beamline beamline{};
    pv_server_config cfg{};
    pv_schedule sched{};
    pvk::KParams kp{};
    std::unique_ptr<pvk::ServerDevice> dev;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    int open = -1;
    std::deque<int> sealed;
    std::vector<int> inflight;
    std::deque<pv_completion> completed;
    std::thread worker;
    bool stop = false;
    int64_t submitted = 0, n_completed = 0, rejected = 0, batches = 0, batched_events = 0;
    int64_t device_bytes = 0;
    int worker_error = PV_OK;
};

namespace pvk {

size_t server_slot_bytes(const pv_server_config &c, const pv_params &p)
{
    const size_t T = (size_t)c.max_tracks_per_batch, E = (size_t)c.max_events_per_batch;
    const size_t mv = (size_t)p.max_vertices_per_event;
    return T * 8 * sizeof(float) + (E + 2) * sizeof(int32_t)       // track columns, offsets, event count
           + E * mv * sizeof(pv_vertex) + 2 * E * sizeof(int32_t)  // vertex slots, counts and status
           + T * (sizeof(int32_t) + sizeof(float))                 // per-track outputs
           + sizeof(WorkQueue) + 2 * E * sizeof(int32_t)           // work queue: deferred list, order
           + E * mv * sizeof(pv_vertex) + (E + 1) * sizeof(int32_t);   // dense records, their offsets
}

}  // namespace pvk

namespace {

// Start a sealed slot's batch on the device.
int dispatch(pv_server &s, Slot &sl)
{
    const size_t E = (size_t)sl.n_events, T = (size_t)sl.n_tracks;
    const size_t mv = (size_t)s.params.max_vertices_per_event;
    sl.dense_copied = (int)std::min(mv * E, kDenseBase * E + T / kDenseTracks);
    sl.rest_issued = false;
    sl.rest_rc = PV_OK;
    return s.dev->dispatch(sl.id, sl.n_events, sl.n_tracks, sl.dense_copied);
}

// Second copy-back of a finished batch: the records past the first copy.
// Returns true when the batch must wait for it.
bool fetch_rest(pv_server &s, Slot &sl)
{
    if (sl.rest_issued)
        return false;
    const int total = sl.h.first[sl.n_events];
    if (total <= sl.dense_copied)
        return false;
    sl.rest_issued = true;
    const int rc = s.dev->fetch(sl.id, sl.dense_copied, total - sl.dense_copied);
    if (rc != PV_OK) {
        sl.rest_rc = rc;
        return false;
    }
    return true;
}

// Scatter a finished slot's results into the callers' buffers.
int complete(Slot &sl, std::vector<pv_completion> &out)
{
    const int total = sl.h.first[sl.n_events];
    int rc = sl.rest_rc;
    if (rc == PV_OK && total > sl.dense_copied && !sl.rest_issued)
        rc = pvk::set_error(PV_EHIP, "server: vertex records past the first copy were not fetched");
    for (int e = 0; e < sl.n_events; ++e) {
        const Request &r = sl.reqs[e];
        const int nv = sl.h.nv[e];
        if (nv > 0 && r.vertices && rc == PV_OK)
            std::memcpy(r.vertices, sl.h.vtx + sl.h.first[e], sizeof(pv_vertex) * (size_t)nv);
        if (r.n_tracks > 0) {
            std::memcpy(r.track_vertex, sl.h.tv + r.first_track, sizeof(int32_t) * (size_t)r.n_tracks);
            std::memcpy(r.track_weight, sl.h.tw + r.first_track, sizeof(float) * (size_t)r.n_tracks);
        }
        pv_completion c;
        c.tag = r.tag;
        c.status = sl.h.status[e];
        c.n_vertices = nv;
        c.t_arrival_ns = r.t_arrival;
        c.t_done_ns = now_ns();
        out.push_back(c);
    }
    return rc;
}

void release(Slot &sl)
{
    sl.state = SlotState::Free;
    sl.n_events = sl.n_tracks = 0;
    sl.reqs.clear();
}

void seal_open(pv_server &s)
{
    if (s.open >= 0) {
        Slot &sl = s.slots[s.open];
        sl.state = SlotState::Sealed;
        s.sealed.push_back(s.open);
        s.open = -1;
        s.cv_work.notify_one();
    }
}

void worker_main(pv_server *sp)
{
    pv_server &s = *sp;
    s.dev->bind_thread();
    std::vector<pv_completion> done;
    std::vector<int> finished, failed;
    // s.inflight is only touched by this thread; the lock guards the slot
    // states, the open / sealed queues and the completion list, which the
    // callers share.  No device call is made with the lock held.
    std::unique_lock<std::mutex> lk(s.mu);
    while (!s.stop) {
        // completions
        if (!s.inflight.empty()) {
            lk.unlock();
            finished.clear();
            failed.clear();
            int crc = PV_OK;
            for (size_t i = 0; i < s.inflight.size();) {
                const int id = s.inflight[i];
                const int q = s.dev->query(id);
                if (q == 1 || (q == PV_OK && fetch_rest(s, s.slots[id]))) {
                    ++i;
                    continue;
                }
                s.inflight.erase(s.inflight.begin() + (long)i);
                if (q == PV_OK) {
                    finished.push_back(id);
                } else {
                    // the batch failed on the device: its results are not
                    // delivered, and every later call reports the error
                    failed.push_back(id);
                    if (crc == PV_OK)
                        crc = q;
                }
            }
            done.clear();
            for (int id : finished) {
                const int rc = complete(s.slots[id], done);
                if (rc != PV_OK && crc == PV_OK)
                    crc = rc;
            }
            lk.lock();
            if (crc != PV_OK && s.worker_error == PV_OK)
                s.worker_error = crc;
            for (const auto &c : done)
                s.completed.push_back(c);
            s.n_completed += (int64_t)done.size();
            for (int id : finished)
                release(s.slots[id]);
            for (int id : failed)
                release(s.slots[id]);
            if (!finished.empty() || !failed.empty())
                s.cv_done.notify_all();
        }
        // continuous batching: a batch is sealed when it is full, or when a
        // stream is free and either the device is idle or its oldest event
        // has waited max_wait_us.  While every stream is busy the open batch
        // keeps growing, so batches grow with the load.
        if (s.open >= 0) {
            const Slot &o = s.slots[s.open];
            const int busy = (int)(s.inflight.size() + s.sealed.size());
            const bool stream_free = busy < s.cfg.n_streams;
            const bool idle = busy == 0;
            const bool waited = now_ns() - o.t_oldest >= (int64_t)s.cfg.max_wait_us * 1000;
            if (o.n_events > 0 && (o.n_events >= s.cfg.max_events_per_batch || (stream_free && (idle || waited))))
                seal_open(s);
        }
        // dispatch, oldest batch first, without the lock; a batch the device
        // refuses is dropped and its error reported by every later call
        while (!s.sealed.empty() && (int)s.inflight.size() < s.cfg.n_streams) {
            const int id = s.sealed.front();
            s.sealed.pop_front();
            Slot &sl = s.slots[id];
            sl.state = SlotState::InFlight;
            ++s.batches;
            s.batched_events += sl.n_events;
            lk.unlock();
            const int rc = dispatch(s, sl);
            lk.lock();
            if (rc != PV_OK) {
                if (s.worker_error == PV_OK)
                    s.worker_error = rc;
                release(sl);
                s.cv_done.notify_all();
            } else {
                s.inflight.push_back(id);
            }
        }
        if (s.inflight.empty() && s.sealed.empty() && (s.open < 0 || s.slots[s.open].n_events == 0)) {
            s.cv_work.wait_for(lk, std::chrono::milliseconds(5));
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

int64_t pv_clock_ns(void)
{
    return now_ns();
}

void pv_server_config_default(pv_server_config *c)
{
    if (!c)
        return;
    c->max_events_per_batch = 2048;
    c->max_tracks_per_batch = 2048 * 400;
    c->n_slots = 4;
    c->n_streams = 2;
    c->device_budget_bytes = (int64_t)4 << 30;
    c->max_wait_us = 200;
    c->use_graphs = 1;
}

int pv_server_create(pv_server **out, const pv_params *params, const pv_beamline *beamline,
                     const pv_server_config *config, const pv_schedule *schedule)
{
    if (!out || !params || !beamline || !config)
        return pvk::set_error(PV_EINVAL, "server: null argument");
    *out = nullptr;
    const pv_server_config &c = *config;
    if (c.max_events_per_batch < 1 || c.max_tracks_per_batch < 1 || c.n_slots < 2 || c.n_streams < 1 ||
        c.n_streams > c.n_slots || c.max_wait_us < 0 || c.device_budget_bytes <= 0)
        return pvk::set_error(PV_EINVAL, "server: bad configuration");
    if (c.max_tracks_per_batch < params->max_tracks_per_event && c.max_events_per_batch == 1)
        return pvk::set_error(PV_EINVAL, "server: a single-event slot must hold max_tracks_per_event tracks");
    std::unique_ptr<pv_server> s(new pv_server());
    s->params = *params;
    s->beamline = *beamline;
    s->cfg = c;
    int rc = pvk::derive_kparams(params, beamline, s->kp);
    if (rc == PV_OK)
        rc = pvk::schedule_for(schedule, s->sched);
    if (rc != PV_OK)
        return rc;
    const size_t per_slot = pvk::server_slot_bytes(c, *params);
    if ((double)per_slot * c.n_slots > (double)c.device_budget_bytes)
        return pvk::set_error(PV_EINVAL, "server: %d slots of %zu bytes exceed the device budget of %lld bytes",
                              c.n_slots, per_slot, (long long)c.device_budget_bytes);
    rc = pvk::make_server_device(c, *params, s->kp, s->sched, &s->dev);
    if (rc != PV_OK)
        return rc;
    s->slots.resize((size_t)c.n_slots);
    for (int k = 0; k < c.n_slots; ++k) {
        s->slots[k].id = k;
        s->slots[k].h = s->dev->host(k);
        s->slots[k].reqs.reserve((size_t)c.max_events_per_batch);
    }
    s->device_bytes = s->dev->device_bytes();
    s->worker = std::thread(worker_main, s.get());
    *out = s.release();
    return PV_OK;
}

int pv_server_submit(pv_server *s, const pv_request *req, uint64_t tag, int64_t t_arrival_ns)
{
    if (!s || !req)
        return pvk::set_error(PV_EINVAL, "server submit: null argument");
    const int n = req->n_tracks;
    if (n < 0 || n > s->cfg.max_tracks_per_batch)
        return pvk::set_error(PV_EINVAL, "server submit: %d tracks do not fit a batch slot (%d)", n,
                              s->cfg.max_tracks_per_batch);
    const float *cols[8] = {req->x, req->y, req->z, req->tx, req->ty, req->cov_xx, req->cov_xtx, req->cov_txtx};
    if (n > 0)
        for (const float *c : cols)
            if (!c)
                return pvk::set_error(PV_EINVAL, "server submit: null track array");
    if (!req->vertices || (n > 0 && (!req->track_vertex || !req->track_weight)))
        return pvk::set_error(PV_EINVAL, "server submit: null output buffer");
    const int64_t t_arr = t_arrival_ns ? t_arrival_ns : now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->worker_error != PV_OK)
        return s->worker_error;
    if (s->open >= 0) {
        const Slot &o = s->slots[s->open];
        if (o.n_events >= s->cfg.max_events_per_batch || o.n_tracks + n > s->cfg.max_tracks_per_batch)
            seal_open(*s);
    }
    if (s->open < 0) {
        for (auto &sl : s->slots)
            if (sl.state == SlotState::Free) {
                sl.state = SlotState::Open;
                sl.n_events = sl.n_tracks = 0;
                sl.h.offsets[0] = 0;
                s->open = sl.id;
                break;
            }
        if (s->open < 0) {
            ++s->rejected;
            return PV_EBUSY;
        }
    }
    Slot &sl = s->slots[s->open];
    for (int k = 0; k < 8 && n > 0; ++k)
        std::memcpy(sl.h.trk[k] + sl.n_tracks, cols[k], sizeof(float) * (size_t)n);
    Request r;
    r.tag = tag;
    r.t_arrival = t_arr;
    r.n_tracks = n;
    r.first_track = sl.n_tracks;
    r.vertices = req->vertices;
    r.track_vertex = req->track_vertex;
    r.track_weight = req->track_weight;
    sl.reqs.push_back(r);
    if (sl.n_events == 0)
        sl.t_oldest = t_arr;
    sl.n_tracks += n;
    sl.n_events += 1;
    sl.h.offsets[sl.n_events] = sl.n_tracks;
    ++s->submitted;
    if (sl.n_events >= s->cfg.max_events_per_batch)
        seal_open(*s);
    s->cv_work.notify_one();
    return PV_OK;
}
int pv_server_poll(pv_server *s, pv_completion *out, int32_t max_out, int32_t timeout_us)
{
    if (!s || (!out && max_out > 0) || max_out < 0)
        return pvk::set_error(PV_EINVAL, "server poll: bad argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completed.empty() && timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [s] { return !s->completed.empty(); });
    int k = 0;
    while (k < max_out && !s->completed.empty()) {
        out[k++] = s->completed.front();
        s->completed.pop_front();
    }
    if (k == 0 && s->worker_error != PV_OK)
        return s->worker_error;
    return k;
}

int pv_server_drain(pv_server *s, int32_t timeout_ms)
{
    if (!s)
        return pvk::set_error(PV_EINVAL, "server drain: null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto idle = [s] {
        if (s->worker_error != PV_OK)
            return true;
        for (const auto &sl : s->slots)
            if (sl.state == SlotState::Sealed || sl.state == SlotState::InFlight ||
                (sl.state == SlotState::Open && sl.n_events > 0))
                return false;
        return true;
    };
    s->cv_work.notify_one();
    if (timeout_ms < 0)
        s->cv_done.wait(lk, idle);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle))
        return pvk::set_error(PV_EBUSY, "server drain: timed out");
    return s->worker_error;
}

int pv_server_replay(pv_server *s, const pv_request *reqs, const int64_t *t_offset_ns, int32_t n,
                     pv_completion *out)
{
    if (!s || n < 0 || (n > 0 && (!reqs || !t_offset_ns || !out)))
        return pvk::set_error(PV_EINVAL, "server replay: bad argument");
    std::vector<char> seen((size_t)n, 0);
    std::vector<pv_completion> buf(256);
    const int64_t t0 = now_ns();
    int next = 0, got = 0;
    while (got < n) {
        // submit every request whose arrival time has passed
        bool busy = false;
        while (next < n && now_ns() >= t0 + t_offset_ns[next]) {
            const int rc = pv_server_submit(s, &reqs[next], (uint64_t)next, t0 + t_offset_ns[next]);
            if (rc == PV_EBUSY) {
                busy = true;   // retried after a completion; its latency keeps counting from the arrival
                break;
            }
            if (rc != PV_OK)
                return rc;
            ++next;
        }
        // with every slot taken, wait for a completion rather than spin on the lock
        const int k = pv_server_poll(s, buf.data(), (int32_t)buf.size(), busy ? 50 : 0);
        if (k < 0)
            return k;
        for (int i = 0; i < k; ++i) {
            const uint64_t tag = buf[(size_t)i].tag;
            if (tag < (uint64_t)n && !seen[tag]) {
                seen[tag] = 1;
                out[tag] = buf[(size_t)i];
                ++got;
            }
        }
        if (k == 0)
            std::this_thread::yield();
    }
    return PV_OK;
}

int pv_server_get_stats(pv_server *s, pv_server_stats *st)
{
    if (!s || !st)
        return pvk::set_error(PV_EINVAL, "server stats: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->submitted;
    st->completed = s->n_completed;
    st->rejected_busy = s->rejected;
    st->batches = s->batches;
    st->mean_batch_events = s->batches ? (double)s->batched_events / (double)s->batches : 0.0;
    st->device_bytes = s->device_bytes;
    return PV_OK;
}

int pv_server_destroy(pv_server *s)
{
    if (!s)
        return PV_OK;
    (void)pv_server_drain(s, 60000);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable())
        s->worker.join();
    s->dev->synchronize();
    delete s;   // the device side frees its buffers
    return PV_OK;
}

}  // extern "C"
