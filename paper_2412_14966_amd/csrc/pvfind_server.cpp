// pvfind_server.cpp -- continuous-batching server on top of the pv_find
// kernels: a pool of batch slots (pinned staging, device buffers, optional
// hipGraph of the launches), admission by free slot, a worker thread that
// seals, launches and completes batches on several streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "pvfind_internal.h"

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

// Each slot keeps its buffers in a few contiguous blocks so that a batch
// moves with six copies: the eight track columns (one 2-D copy of rows of
// cap_tracks floats), offsets and event count, vertex counts and status (one
// 2-D copy), per-event offsets of the written vertex records, the records
// themselves (gathered into one dense array on the device, at most
// kDenseBudget per event in this copy), and per-track vertex ids and weights
// (one 2-D copy).  A batch with more records than that budget fetches the
// rest when it completes.
constexpr int kDenseBudget = 16;
struct Slot {
    int id = 0;
    hipStream_t stream = nullptr;
    SlotState state = SlotState::Free;
    // device
    float *d_in = nullptr;          // 8 columns of cap_tracks floats, then cap_events + 2 ints
    float *d_trk[8] = {};
    int32_t *d_offsets = nullptr;   // cap_events + 1 offsets, then the event count
    int32_t *d_nev = nullptr;
    pv_vertex *d_vtx = nullptr;
    int32_t *d_ns = nullptr;        // vertex counts, then status: 2 rows of cap_events
    int32_t *d_nv = nullptr, *d_status = nullptr;
    int32_t *d_tout = nullptr;      // vertex ids, then weights: 2 rows of cap_tracks
    int32_t *d_tv = nullptr;
    float *d_tw = nullptr;
    pv_vertex *d_dense = nullptr;   // written vertex records, event after event
    int32_t *d_first = nullptr;     // cap_events + 1: offsets of each event's records, then the total
    // pinned host, same layouts
    float *h_in = nullptr;
    float *h_trk[8] = {};
    int32_t *h_offsets = nullptr;
    pv_vertex *h_vtx = nullptr;     // the dense records
    int32_t *h_first = nullptr;
    int32_t *h_ns = nullptr, *h_nv = nullptr, *h_status = nullptr;
    int32_t *h_tout = nullptr, *h_tv = nullptr;
    float *h_tw = nullptr;
    pvk::WorkQueue *wq = nullptr;   // this slot's own queue counters (baked into its graph)
    hipGraphExec_t graph = nullptr;
    hipEvent_t done = nullptr;
    int n_events = 0, n_tracks = 0;
    int dense_copied = 0;           // records the batch's copy-back brought
    int64_t t_oldest = 0;
    std::vector<Request> reqs;
};

}  // namespace

struct pv_server {
    int device = 0;
    pv_params params{};
    pv_beamline beamline{};
    pv_server_config cfg{};
    pv_schedule sched{};
    pvk::KParams kp{};
    std::vector<hipStream_t> streams;
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

namespace {

void free_slot(Slot &s)
{
    for (void *p : {(void *)s.d_in, (void *)s.d_vtx, (void *)s.d_ns, (void *)s.d_tout, (void *)s.wq,
                    (void *)s.d_dense, (void *)s.d_first})
        if (p)
            (void)hipFree(p);
    for (void *p : {(void *)s.h_in, (void *)s.h_vtx, (void *)s.h_ns, (void *)s.h_tout, (void *)s.h_first})
        if (p)
            (void)hipHostFree(p);
    if (s.graph)
        (void)hipGraphExecDestroy(s.graph);
    if (s.done)
        (void)hipEventDestroy(s.done);
    s = Slot();
}

size_t slot_device_bytes(const pv_server_config &c, const pv_params &p)
{
    const size_t T = (size_t)c.max_tracks_per_batch, E = (size_t)c.max_events_per_batch;
    return T * 8 * sizeof(float) + (E + 1) * sizeof(int32_t) + sizeof(int32_t) +
           E * (size_t)p.max_vertices_per_event * sizeof(pv_vertex) + 2 * E * sizeof(int32_t) +
           T * (sizeof(int32_t) + sizeof(float)) + sizeof(pvk::WorkQueue) + 2 * E * sizeof(int32_t) +
           E * (size_t)p.max_vertices_per_event * sizeof(pv_vertex) + (E + 1) * sizeof(int32_t);
}

template <typename T>
int dev_alloc(T **p, size_t n)
{
    const hipError_t err = hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
    return err == hipSuccess ? PV_OK : pvk::set_error(PV_ENOMEM, "hipMalloc: %s", hipGetErrorString(err));
}

template <typename T>
int host_alloc(T **p, size_t n)
{
    const hipError_t err = hipHostMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault);
    return err == hipSuccess ? PV_OK : pvk::set_error(PV_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(err));
}

pvk::KArgs slot_args(const pv_server &s, const Slot &sl, pvk::WorkQueue *wq, int n_events)
{
    pvk::KArgs A;
    std::memset(&A, 0, sizeof(A));
    A.x = sl.d_trk[0];
    A.y = sl.d_trk[1];
    A.z = sl.d_trk[2];
    A.tx = sl.d_trk[3];
    A.ty = sl.d_trk[4];
    A.cxx = sl.d_trk[5];
    A.cxtx = sl.d_trk[6];
    A.ctxtx = sl.d_trk[7];
    A.offsets = sl.d_offsets;
    A.n_events = n_events;
    A.vout = sl.d_vtx;
    A.nv_out = sl.d_nv;
    A.status_out = sl.d_status;
    A.trk_vtx = sl.d_tv;
    A.trk_w = sl.d_tw;
    A.wq = wq;
    A.order = (s.sched.persistent >= 3) ? pvk::order_list(wq, s.cfg.max_events_per_batch) : nullptr;
    A.p = s.kp;
    return A;
}

int init_slot(pv_server &s, Slot &sl)
{
    const int T = s.cfg.max_tracks_per_batch, E = s.cfg.max_events_per_batch;
    const int mv = s.params.max_vertices_per_event;
    const size_t in_floats = 8 * (size_t)T + (size_t)E + 2;   // int32 and float are both 4 bytes
    int rc = dev_alloc(&sl.d_in, in_floats);
    if (rc == PV_OK)
        rc = host_alloc(&sl.h_in, in_floats);
    if (rc == PV_OK)
        rc = dev_alloc(&sl.d_vtx, (size_t)E * mv);
    if (rc == PV_OK)
        rc = host_alloc(&sl.h_vtx, (size_t)E * mv);
    if (rc == PV_OK)
        rc = dev_alloc(&sl.d_ns, 2 * (size_t)E);
    if (rc == PV_OK)
        rc = host_alloc(&sl.h_ns, 2 * (size_t)E);
    if (rc == PV_OK)
        rc = dev_alloc(&sl.d_dense, (size_t)E * mv);
    if (rc == PV_OK)
        rc = dev_alloc(&sl.d_first, (size_t)E + 1);
    if (rc == PV_OK)
        rc = host_alloc(&sl.h_first, (size_t)E + 1);
    if (rc == PV_OK)
        rc = dev_alloc(&sl.d_tout, 2 * (size_t)T);
    if (rc == PV_OK)
        rc = host_alloc(&sl.h_tout, 2 * (size_t)T);
    if (rc != PV_OK)
        return rc;
    for (int k = 0; k < 8; ++k) {
        sl.d_trk[k] = sl.d_in + (size_t)k * T;
        sl.h_trk[k] = sl.h_in + (size_t)k * T;
    }
    sl.d_offsets = reinterpret_cast<int32_t *>(sl.d_in + 8 * (size_t)T);
    sl.h_offsets = reinterpret_cast<int32_t *>(sl.h_in + 8 * (size_t)T);
    sl.d_nev = sl.d_offsets + E + 1;
    sl.d_nv = sl.d_ns;
    sl.d_status = sl.d_ns + E;
    sl.h_nv = sl.h_ns;
    sl.h_status = sl.h_ns + E;
    sl.d_tv = sl.d_tout;
    sl.d_tw = reinterpret_cast<float *>(sl.d_tout + T);
    sl.h_tv = sl.h_tout;
    sl.h_tw = reinterpret_cast<float *>(sl.h_tout + T);
    const size_t wq_bytes = sizeof(pvk::WorkQueue) + 2 * sizeof(int32_t) * (size_t)E;   // deferred list, order
    hipError_t err = hipMalloc((void **)&sl.wq, wq_bytes);
    if (err != hipSuccess)
        return pvk::set_error(PV_ENOMEM, "hipMalloc: %s", hipGetErrorString(err));
    err = hipMemset(sl.wq, 0, wq_bytes);
    if (err == hipSuccess)
        err = hipDeviceSynchronize();
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "workspace init: %s", hipGetErrorString(err));
    err = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "hipEventCreate: %s", hipGetErrorString(err));
    sl.reqs.reserve(E);
    if (!s.cfg.use_graphs)
        return PV_OK;
    pvk::KArgs A = slot_args(s, sl, sl.wq, E);
    A.n_events_dev = sl.d_nev;
    err = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(err));
    int lerr = pvk::launch_batch(A, s.sched, false, sl.stream, nullptr);
    if (lerr == (int)hipSuccess)
        lerr = pvk::launch_compact(sl.d_vtx, sl.d_nv, sl.d_nev, E, mv, sl.d_dense, sl.d_first, sl.stream);
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(sl.stream, &g);
    if (lerr != (int)hipSuccess || err != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return pvk::set_error(PV_EHIP, "graph capture: %s",
                              hipGetErrorString(lerr != (int)hipSuccess ? (hipError_t)lerr : err));
    }
    err = hipGraphInstantiate(&sl.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(err));
    return PV_OK;
}

// Enqueue copies, launch and copy-back of a sealed slot on its stream.
int dispatch(pv_server &s, Slot &sl)
{
    const int E = sl.n_events, T = sl.n_tracks;
    const size_t capE = (size_t)s.cfg.max_events_per_batch, capT = (size_t)s.cfg.max_tracks_per_batch;
    hipStream_t st = sl.stream;
    sl.h_offsets[capE + 1] = E;
    hipError_t err = hipSuccess;
    if (T > 0)   // the eight columns: 8 rows of T floats at a pitch of capT floats
        err = hipMemcpy2DAsync(sl.d_in, capT * sizeof(float), sl.h_in, capT * sizeof(float),
                               (size_t)T * sizeof(float), 8, hipMemcpyHostToDevice, st);
    if (err == hipSuccess)   // offsets and, at capE + 1, the event count
        err = hipMemcpyAsync(sl.d_offsets, sl.h_offsets, sizeof(int32_t) * (capE + 2), hipMemcpyHostToDevice, st);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "server copy-in: %s", hipGetErrorString(err));
    if (sl.graph) {
        err = hipGraphLaunch(sl.graph, st);
        if (err != hipSuccess)
            return pvk::set_error(PV_EHIP, "hipGraphLaunch: %s", hipGetErrorString(err));
    } else {
        const pvk::KArgs A = slot_args(s, sl, sl.wq, E);
        int lerr = pvk::launch_batch(A, s.sched, false, st, nullptr);
        if (lerr == (int)hipSuccess)
            lerr = pvk::launch_compact(sl.d_vtx, sl.d_nv, nullptr, E, s.params.max_vertices_per_event, sl.d_dense,
                                       sl.d_first, st);
        if (lerr != (int)hipSuccess)
            return pvk::set_error(PV_EHIP, "server launch: %s", hipGetErrorString((hipError_t)lerr));
    }
    const size_t mv = (size_t)s.params.max_vertices_per_event;
    // vertex counts and status: 2 rows of E ints at a pitch of capE
    err = hipMemcpy2DAsync(sl.h_ns, capE * sizeof(int32_t), sl.d_ns, capE * sizeof(int32_t),
                           (size_t)E * sizeof(int32_t), 2, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess)
        err = hipMemcpyAsync(sl.h_first, sl.d_first, sizeof(int32_t) * ((size_t)E + 1), hipMemcpyDeviceToHost, st);
    // the dense records, up to the budget (a batch averages about 10 per event
    // on the served mix; more are fetched on completion)
    sl.dense_copied = (int)std::min<size_t>(mv * (size_t)E, (size_t)kDenseBudget * (size_t)E);
    if (err == hipSuccess)
        err = hipMemcpyAsync(sl.h_vtx, sl.d_dense, sizeof(pv_vertex) * (size_t)sl.dense_copied,
                             hipMemcpyDeviceToHost, st);
    if (err == hipSuccess && T > 0)   // vertex ids and weights: 2 rows of T at a pitch of capT
        err = hipMemcpy2DAsync(sl.h_tout, capT * sizeof(int32_t), sl.d_tout, capT * sizeof(int32_t),
                               (size_t)T * sizeof(int32_t), 2, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess)
        err = hipEventRecord(sl.done, st);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "server copy-out: %s", hipGetErrorString(err));
    return PV_OK;
}

// Scatter a finished slot's results into the callers' buffers.
int complete(pv_server &s, Slot &sl, std::vector<pv_completion> &out)
{
    const int total = sl.h_first[sl.n_events];
    int rc = PV_OK;
    if (total > sl.dense_copied) {
        // more records than the budget: fetch the rest (not under the lock)
        const size_t rest = (size_t)(total - sl.dense_copied);
        hipError_t err = hipMemcpyAsync(sl.h_vtx + sl.dense_copied, sl.d_dense + sl.dense_copied,
                                        sizeof(pv_vertex) * rest, hipMemcpyDeviceToHost, sl.stream);
        if (err == hipSuccess)
            err = hipStreamSynchronize(sl.stream);
        if (err != hipSuccess)
            rc = pvk::set_error(PV_EHIP, "server copy-out: %s", hipGetErrorString(err));
    }
    for (int e = 0; e < sl.n_events; ++e) {
        const Request &r = sl.reqs[e];
        const int nv = sl.h_nv[e];
        if (nv > 0 && r.vertices && rc == PV_OK)
            std::memcpy(r.vertices, sl.h_vtx + sl.h_first[e], sizeof(pv_vertex) * (size_t)nv);
        if (r.n_tracks > 0) {
            std::memcpy(r.track_vertex, sl.h_tv + r.first_track, sizeof(int32_t) * (size_t)r.n_tracks);
            std::memcpy(r.track_weight, sl.h_tw + r.first_track, sizeof(float) * (size_t)r.n_tracks);
        }
        pv_completion c;
        c.tag = r.tag;
        c.status = sl.h_status[e];
        c.n_vertices = nv;
        c.t_arrival_ns = r.t_arrival;
        c.t_done_ns = now_ns();
        out.push_back(c);
    }
    return rc;
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
    (void)hipSetDevice(s.device);
    std::vector<pv_completion> done;
    std::vector<int> finished;
    // s.inflight is only touched by this thread; the lock guards the slot
    // states, the open / sealed queues and the completion list, which the
    // callers share.  No HIP call is made with the lock held.
    std::unique_lock<std::mutex> lk(s.mu);
    while (!s.stop) {
        // completions
        if (!s.inflight.empty()) {
            lk.unlock();
            finished.clear();
            for (size_t i = 0; i < s.inflight.size();) {
                const int id = s.inflight[i];
                const hipError_t q = hipEventQuery(s.slots[id].done);
                if (q == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                if (q != hipSuccess) {
                    std::lock_guard<std::mutex> g(s.mu);
                    if (s.worker_error == PV_OK)
                        s.worker_error = pvk::set_error(PV_EHIP, "server batch: %s", hipGetErrorString(q));
                }
                s.inflight.erase(s.inflight.begin() + (long)i);
                finished.push_back(id);
            }
            done.clear();
            int crc = PV_OK;
            for (int id : finished) {
                const int rc = complete(s, s.slots[id], done);
                if (rc != PV_OK)
                    crc = rc;
            }
            lk.lock();
            if (crc != PV_OK && s.worker_error == PV_OK)
                s.worker_error = crc;
            for (const auto &c : done)
                s.completed.push_back(c);
            s.n_completed += (int64_t)done.size();
            for (int id : finished) {
                Slot &sl = s.slots[id];
                sl.state = SlotState::Free;
                sl.n_events = sl.n_tracks = 0;
                sl.reqs.clear();
            }
            if (!finished.empty())
                s.cv_done.notify_all();
        }
        // continuous batching: a batch is sealed when it is full, or when a
        // stream is free and either the GPU is idle or its oldest event has
        // waited max_wait_us.  While every stream is busy the open batch keeps
        // growing, so batches grow with the load.
        if (s.open >= 0) {
            const Slot &o = s.slots[s.open];
            const int busy = (int)(s.inflight.size() + s.sealed.size());
            const bool stream_free = busy < s.cfg.n_streams;
            const bool idle = busy == 0;
            const bool waited = now_ns() - o.t_oldest >= (int64_t)s.cfg.max_wait_us * 1000;
            if (o.n_events > 0 && (o.n_events >= s.cfg.max_events_per_batch || (stream_free && (idle || waited))))
                seal_open(s);
        }
        // launches, oldest batch first, without the lock
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
            if (rc != PV_OK && s.worker_error == PV_OK)
                s.worker_error = rc;
            s.inflight.push_back(id);
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
    auto s = new pv_server();
    s->params = *params;
    s->beamline = *beamline;
    s->cfg = c;
    int rc = pvk::derive_kparams(params, beamline, s->kp);
    if (rc == PV_OK)
        rc = pvk::schedule_for(schedule, s->sched);
    const size_t per_slot = slot_device_bytes(c, *params);
    if (rc == PV_OK && (double)per_slot * c.n_slots > (double)c.device_budget_bytes)
        rc = pvk::set_error(PV_EINVAL, "server: %d slots of %zu bytes exceed the device budget of %lld bytes",
                            c.n_slots, per_slot, (long long)c.device_budget_bytes);
    if (rc == PV_OK && hipGetDevice(&s->device) != hipSuccess)
        rc = pvk::set_error(PV_EHIP, "hipGetDevice failed");
    for (int k = 0; k < c.n_streams && rc == PV_OK; ++k) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            rc = pvk::set_error(PV_EHIP, "hipStreamCreate failed");
        else
            s->streams.push_back(st);
    }
    if (rc == PV_OK) {
        s->slots.resize((size_t)c.n_slots);
        for (int k = 0; k < c.n_slots && rc == PV_OK; ++k) {
            s->slots[k].id = k;
            s->slots[k].stream = s->streams[(size_t)(k % c.n_streams)];
            rc = init_slot(*s, s->slots[k]);
        }
        s->device_bytes = (int64_t)per_slot * c.n_slots;
    }
    if (rc != PV_OK) {
        for (auto &sl : s->slots)
            free_slot(sl);
        for (auto st : s->streams)
            (void)hipStreamDestroy(st);
        delete s;
        return rc;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
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
                sl.h_offsets[0] = 0;
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
        std::memcpy(sl.h_trk[k] + sl.n_tracks, cols[k], sizeof(float) * (size_t)n);
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
    sl.h_offsets[sl.n_events] = sl.n_tracks;
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
    for (auto st : s->streams)
        (void)hipStreamSynchronize(st);
    for (auto &sl : s->slots)
        free_slot(sl);
    for (auto st : s->streams)
        (void)hipStreamDestroy(st);
    delete s;
    return PV_OK;
}

}  // extern "C"
