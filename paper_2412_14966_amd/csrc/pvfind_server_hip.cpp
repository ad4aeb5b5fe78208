// pvfind_server_hip.cpp -- device side of the continuous-batching server:
// per slot, device buffers and pinned staging in a few contiguous blocks, its
// own work queue, an optional hipGraph of the launches (the batch size read
// from device memory on replay), and a completion event; slots share a few
// non-blocking streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "pvfind_server_device.h"

namespace {

// A batch moves with six copies: the eight track columns (one 2-D copy of
// rows of cap_tracks floats), offsets and event count, vertex counts and
// status (one 2-D copy), per-event offsets of the written vertex records, the
// records themselves (gathered into one dense array on the device), and
// per-track vertex ids and weights (one 2-D copy).
struct HipSlot {
    hipStream_t stream = nullptr;
    // device
    float *d_in = nullptr;          // 8 columns of cap_tracks floats, then cap_events + 2 ints
    float *d_trk[8] = {};
    int32_t *d_offsets = nullptr;   // cap_events + 1 offsets, then the event count
    int32_t *d_nev = nullptr;
    pv_vertex *d_vtx = nullptr;     // max_vertices slots per event, as pv_find writes them
    int32_t *d_ns = nullptr;        // vertex counts, then status: 2 rows of cap_events
    int32_t *d_nv = nullptr, *d_status = nullptr;
    int32_t *d_tout = nullptr;      // vertex ids, then weights: 2 rows of cap_tracks
    int32_t *d_tv = nullptr;
    float *d_tw = nullptr;
    pv_vertex *d_dense = nullptr;   // written vertex records, event after event
    int32_t *d_first = nullptr;     // cap_events + 1: offsets of each event's records, then the total
    pvk::WorkQueue *wq = nullptr;   // this slot's own queue counters (baked into its graph)
    // pinned host, same layouts
    float *h_in = nullptr;
    int32_t *h_ns = nullptr;
    int32_t *h_tout = nullptr;
    pvk::SlotHost h;
    hipGraphExec_t graph = nullptr;
    hipEvent_t done = nullptr;
};

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

class HipServerDevice final : public pvk::ServerDevice {
public:
    HipServerDevice(const pv_server_config &c, const pv_params &p, const pvk::KParams &kp, const pv_schedule &s)
        : cfg_(c), params_(p), kp_(kp), sched_(s)
    {
    }

    ~HipServerDevice() override
    {
        for (auto &sl : slots_)
            free_slot(sl);
        for (auto st : streams_)
            (void)hipStreamDestroy(st);
    }

    int init()
    {
        if (hipGetDevice(&device_) != hipSuccess)
            return pvk::set_error(PV_EHIP, "hipGetDevice failed");
        for (int k = 0; k < cfg_.n_streams; ++k) {
            hipStream_t st;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
                return pvk::set_error(PV_EHIP, "hipStreamCreate failed");
            streams_.push_back(st);
        }
        slots_.resize((size_t)cfg_.n_slots);
        for (int k = 0; k < cfg_.n_slots; ++k) {
            slots_[k].stream = streams_[(size_t)(k % cfg_.n_streams)];
            const int rc = init_slot(slots_[k]);
            if (rc != PV_OK)
                return rc;
        }
        return PV_OK;
    }

    int64_t device_bytes() const override
    {
        return (int64_t)pvk::server_slot_bytes(cfg_, params_) * cfg_.n_slots;
    }

    const pvk::SlotHost &host(int slot) const override { return slots_[(size_t)slot].h; }

    void bind_thread() override { (void)hipSetDevice(device_); }

    int dispatch(int slot, int E, int T, int records) override
    {
        HipSlot &sl = slots_[(size_t)slot];
        const size_t capE = (size_t)cfg_.max_events_per_batch, capT = (size_t)cfg_.max_tracks_per_batch;
        hipStream_t st = sl.stream;
        sl.h.offsets[capE + 1] = E;
        hipError_t err = hipSuccess;
        if (T > 0)   // the eight columns: 8 rows of T floats at a pitch of capT floats
            err = hipMemcpy2DAsync(sl.d_in, capT * sizeof(float), sl.h_in, capT * sizeof(float),
                                   (size_t)T * sizeof(float), 8, hipMemcpyHostToDevice, st);
        if (err == hipSuccess)   // offsets and, at capE + 1, the event count
            err = hipMemcpyAsync(sl.d_offsets, sl.h.offsets, sizeof(int32_t) * (capE + 2), hipMemcpyHostToDevice,
                                 st);
        if (err != hipSuccess)
            return pvk::set_error(PV_EHIP, "server copy-in: %s", hipGetErrorString(err));
        if (sl.graph) {
            err = hipGraphLaunch(sl.graph, st);
            if (err != hipSuccess)
                return pvk::set_error(PV_EHIP, "hipGraphLaunch: %s", hipGetErrorString(err));
        } else {
            const pvk::KArgs A = slot_args(sl, E);
            int lerr = pvk::launch_batch(A, sched_, false, st, nullptr);
            if (lerr == (int)hipSuccess)
                lerr = pvk::launch_compact(sl.d_vtx, sl.d_nv, nullptr, E, params_.max_vertices_per_event, sl.d_dense,
                                           sl.d_first, st);
            if (lerr != (int)hipSuccess)
                return pvk::set_error(PV_EHIP, "server launch: %s", hipGetErrorString((hipError_t)lerr));
        }
        // vertex counts and status: 2 rows of E ints at a pitch of capE
        err = hipMemcpy2DAsync(sl.h_ns, capE * sizeof(int32_t), sl.d_ns, capE * sizeof(int32_t),
                               (size_t)E * sizeof(int32_t), 2, hipMemcpyDeviceToHost, st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(sl.h.first, sl.d_first, sizeof(int32_t) * ((size_t)E + 1), hipMemcpyDeviceToHost,
                                 st);
        if (err == hipSuccess && records > 0)
            err = hipMemcpyAsync(sl.h.vtx, sl.d_dense, sizeof(pv_vertex) * (size_t)records, hipMemcpyDeviceToHost,
                                 st);
        if (err == hipSuccess && T > 0)   // vertex ids and weights: 2 rows of T at a pitch of capT
            err = hipMemcpy2DAsync(sl.h_tout, capT * sizeof(int32_t), sl.d_tout, capT * sizeof(int32_t),
                                   (size_t)T * sizeof(int32_t), 2, hipMemcpyDeviceToHost, st);
        if (err == hipSuccess)
            err = hipEventRecord(sl.done, st);
        if (err != hipSuccess)
            return pvk::set_error(PV_EHIP, "server copy-out: %s", hipGetErrorString(err));
        return PV_OK;
    }

    int query(int slot) override
    {
        const hipError_t q = hipEventQuery(slots_[(size_t)slot].done);
        if (q == hipErrorNotReady)
            return 1;
        if (q != hipSuccess)
            return pvk::set_error(PV_EHIP, "server batch: %s", hipGetErrorString(q));
        return PV_OK;
    }

    int fetch(int slot, int from, int count) override
    {
        HipSlot &sl = slots_[(size_t)slot];
        hipError_t err = hipMemcpyAsync(sl.h.vtx + from, sl.d_dense + from, sizeof(pv_vertex) * (size_t)count,
                                        hipMemcpyDeviceToHost, sl.stream);
        if (err == hipSuccess)
            err = hipEventRecord(sl.done, sl.stream);
        if (err != hipSuccess)
            return pvk::set_error(PV_EHIP, "server copy-out: %s", hipGetErrorString(err));
        return PV_OK;
    }

    void synchronize() override
    {
        for (auto st : streams_)
            (void)hipStreamSynchronize(st);
    }

private:
    pvk::KArgs slot_args(const HipSlot &sl, int n_events) const
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
        A.wq = sl.wq;
        A.order = (sched_.persistent >= 3) ? pvk::order_list(sl.wq, cfg_.max_events_per_batch) : nullptr;
        A.p = kp_;
        return A;
    }

    int init_slot(HipSlot &sl)
    {
        const int T = cfg_.max_tracks_per_batch, E = cfg_.max_events_per_batch;
        const int mv = params_.max_vertices_per_event;
        const size_t in_floats = 8 * (size_t)T + (size_t)E + 2;   // int32 and float are both 4 bytes
        int rc = dev_alloc(&sl.d_in, in_floats);
        if (rc == PV_OK)
            rc = host_alloc(&sl.h_in, in_floats);
        if (rc == PV_OK)
            rc = dev_alloc(&sl.d_vtx, (size_t)E * mv);
        if (rc == PV_OK)
            rc = host_alloc(&sl.h.vtx, (size_t)E * mv);
        if (rc == PV_OK)
            rc = dev_alloc(&sl.d_ns, 2 * (size_t)E);
        if (rc == PV_OK)
            rc = host_alloc(&sl.h_ns, 2 * (size_t)E);
        if (rc == PV_OK)
            rc = dev_alloc(&sl.d_dense, (size_t)E * mv);
        if (rc == PV_OK)
            rc = dev_alloc(&sl.d_first, (size_t)E + 1);
        if (rc == PV_OK)
            rc = host_alloc(&sl.h.first, (size_t)E + 1);
        if (rc == PV_OK)
            rc = dev_alloc(&sl.d_tout, 2 * (size_t)T);
        if (rc == PV_OK)
            rc = host_alloc(&sl.h_tout, 2 * (size_t)T);
        if (rc != PV_OK)
            return rc;
        for (int k = 0; k < 8; ++k) {
            sl.d_trk[k] = sl.d_in + (size_t)k * T;
            sl.h.trk[k] = sl.h_in + (size_t)k * T;
        }
        sl.d_offsets = reinterpret_cast<int32_t *>(sl.d_in + 8 * (size_t)T);
        sl.h.offsets = reinterpret_cast<int32_t *>(sl.h_in + 8 * (size_t)T);
        sl.d_nev = sl.d_offsets + E + 1;
        sl.d_nv = sl.d_ns;
        sl.d_status = sl.d_ns + E;
        sl.h.nv = sl.h_ns;
        sl.h.status = sl.h_ns + E;
        sl.d_tv = sl.d_tout;
        sl.d_tw = reinterpret_cast<float *>(sl.d_tout + T);
        sl.h.tv = sl.h_tout;
        sl.h.tw = reinterpret_cast<float *>(sl.h_tout + T);
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
        if (!cfg_.use_graphs)
            return PV_OK;
        pvk::KArgs A = slot_args(sl, E);
        A.n_events_dev = sl.d_nev;
        err = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
        if (err != hipSuccess)
            return pvk::set_error(PV_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(err));
        int lerr = pvk::launch_batch(A, sched_, false, sl.stream, nullptr);
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

    static void free_slot(HipSlot &s)
    {
        for (void *p : {(void *)s.d_in, (void *)s.d_vtx, (void *)s.d_ns, (void *)s.d_tout, (void *)s.wq,
                        (void *)s.d_dense, (void *)s.d_first})
            if (p)
                (void)hipFree(p);
        for (void *p : {(void *)s.h_in, (void *)s.h.vtx, (void *)s.h_ns, (void *)s.h_tout, (void *)s.h.first})
            if (p)
                (void)hipHostFree(p);
        if (s.graph)
            (void)hipGraphExecDestroy(s.graph);
        if (s.done)
            (void)hipEventDestroy(s.done);
        s = HipSlot();
    }

    pv_server_config cfg_;
    pv_params params_;
    pvk::KParams kp_;
    pv_schedule sched_;
    int device_ = 0;
    std::vector<hipStream_t> streams_;
    std::vector<HipSlot> slots_;
};

}  // namespace

namespace pvk {

int make_server_device(const pv_server_config &config, const pv_params &params, const KParams &kp,
                       const pv_schedule &sched, std::unique_ptr<ServerDevice> *out)
{
    std::unique_ptr<HipServerDevice> d(new HipServerDevice(config, params, kp, sched));
    const int rc = d->init();
    if (rc != PV_OK)
        return rc;   // the destructor frees what init allocated
    *out = std::move(d);
    return PV_OK;
}

}  // namespace pvk
