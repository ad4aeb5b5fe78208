// fake_server_device.cpp -- CPU stand-in for pvk::ServerDevice.  A dispatch
// computes the batch's results at once into "device" arrays and poisons the
// host outputs; the copies back to the host staging happen when query first
// sees the batch's run time elapsed, and only for what a real copy would
// move (the first `records` records; fetch moves the rest), so the server
// reading anything early or unfetched reads poison.  The inputs are read
// again at completion: a server that changed the staging of a running batch
// is counted.
#include "fake_server_device.h"

#include <chrono>
#include <cstring>
#include <vector>

#include "pvfind_server_device.h"

namespace fake {

Knobs &knobs()
{
    static Knobs k;
    return k;
}

void event_result(const float *const trk[8], int first, int n, int max_v, int32_t *nv, int32_t *status,
                  pv_vertex *vtx, int32_t *tv, float *tw)
{
    const int k_n = n / 3 < max_v ? n / 3 : max_v;
    *nv = k_n;
    *status = (n % 5 == 0) ? PV_EV_FIT_FAILED : 0;
    for (int k = 0; k < k_n; ++k) {
        pv_vertex v;
        std::memset(&v, 0, sizeof(v));
        v.x = trk[0][first + k % n];
        v.y = trk[1][first + k % n];
        v.z = trk[2][first] + (float)k;
        v.chi2 = trk[3][first + (k * 7) % n];
        v.ndof = (float)(2 * k + 1);
        v.n_tracks = k + 1;
        v.flags = (uint8_t)(k & 3);
        vtx[k] = v;
    }
    for (int i = 0; i < n; ++i) {
        tv[i] = k_n > 0 ? i % k_n : -1;
        tw[i] = trk[3][first + i] * 0.5f + trk[5][first + i];
    }
}

}  // namespace fake

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct FakeSlot {
    std::vector<float> trk;          // 8 columns of capT
    std::vector<int32_t> offsets;    // capE + 2
    std::vector<int32_t> nv, status, first, tv;
    std::vector<float> tw;
    std::vector<pv_vertex> vtx;      // capE * max_v
    // "device" side
    std::vector<int32_t> d_nv, d_status, d_first, d_tv;
    std::vector<float> d_tw;
    std::vector<pv_vertex> d_vtx;
    std::vector<float> in_copy;      // the inputs as dispatched
    pvk::SlotHost h;
    int64_t done_at = 0;
    int pending = 0;                 // 0 none, 1 dispatch copies, 2 fetch copies
    int E = 0, T = 0, records = 0, from = 0, count = 0;
};

class FakeServerDevice final : public pvk::ServerDevice {
public:
    FakeServerDevice(const pv_server_config &c, const pv_params &p) : cfg_(c), max_v_(p.max_vertices_per_event)
    {
        ++fake::knobs().live_devices;
        const size_t T = (size_t)c.max_tracks_per_batch, E = (size_t)c.max_events_per_batch;
        slots_.resize((size_t)c.n_slots);
        for (auto &s : slots_) {
            s.trk.assign(8 * T, 0.0f);
            s.offsets.assign(E + 2, 0);
            s.nv.assign(E, 0);
            s.status.assign(E, 0);
            s.first.assign(E + 1, 0);
            s.tv.assign(T, 0);
            s.tw.assign(T, 0.0f);
            s.vtx.assign(E * (size_t)max_v_, pv_vertex());
            for (int k = 0; k < 8; ++k)
                s.h.trk[k] = s.trk.data() + (size_t)k * T;
            s.h.offsets = s.offsets.data();
            s.h.nv = s.nv.data();
            s.h.status = s.status.data();
            s.h.first = s.first.data();
            s.h.vtx = s.vtx.data();
            s.h.tv = s.tv.data();
            s.h.tw = s.tw.data();
        }
        bytes_ = (int64_t)pvk::server_slot_bytes(c, p) * c.n_slots;
    }
    ~FakeServerDevice() override { --fake::knobs().live_devices; }

    int64_t device_bytes() const override { return bytes_; }
    const pvk::SlotHost &host(int slot) const override { return slots_[(size_t)slot].h; }
    void bind_thread() override {}

    int dispatch(int slot, int E, int T, int records) override
    {
        const int n = fake::knobs().dispatches++;
        if (n == fake::knobs().fail_dispatch_at.load())
            return pvk::set_error(PV_EHIP, "fake device: dispatch %d refused", n);
        FakeSlot &s = slots_[(size_t)slot];
        if (s.pending != 0)
            return pvk::set_error(PV_EHIP, "fake device: slot %d dispatched while busy", slot);
        if (E < 1 || E > cfg_.max_events_per_batch || T < 0 || T > cfg_.max_tracks_per_batch || records < 0 ||
            records > E * max_v_ || s.offsets[0] != 0 || s.offsets[(size_t)E] != T)
            return pvk::set_error(PV_EINVAL, "fake device: inconsistent batch (E %d, T %d, records %d)", E, T,
                                  records);
        s.E = E;
        s.T = T;
        s.records = records;
        s.in_copy = snapshot(s);
        compute(s);
        // poison the host outputs until the copies land
        std::memset(s.nv.data(), 0xA5, sizeof(int32_t) * (size_t)E);
        std::memset(s.status.data(), 0xA5, sizeof(int32_t) * (size_t)E);
        std::memset(s.first.data(), 0xA5, sizeof(int32_t) * ((size_t)E + 1));
        std::memset(s.vtx.data(), 0xA5, sizeof(pv_vertex) * s.vtx.size());
        std::memset(s.tv.data(), 0xA5, sizeof(int32_t) * (size_t)T);
        std::memset(s.tw.data(), 0xA5, sizeof(float) * (size_t)T);
        s.pending = 1;
        s.done_at = now_ns() + 1000ll * fake::knobs().latency_us.load();
        return PV_OK;
    }

    int query(int slot) override
    {
        FakeSlot &s = slots_[(size_t)slot];
        if (s.pending == 0)
            return PV_OK;
        if (now_ns() < s.done_at)
            return 1;
        if (s.pending == 1 && fake::knobs().batches_done++ == fake::knobs().fail_batch_at.load()) {
            s.pending = 0;
            return pvk::set_error(PV_EHIP, "fake device: batch of slot %d failed", slot);
        }
        if (s.pending == 1) {
            if (snapshot(s) != s.in_copy)
                ++fake::knobs().staging_violations;
            std::memcpy(s.nv.data(), s.d_nv.data(), sizeof(int32_t) * (size_t)s.E);
            std::memcpy(s.status.data(), s.d_status.data(), sizeof(int32_t) * (size_t)s.E);
            std::memcpy(s.first.data(), s.d_first.data(), sizeof(int32_t) * ((size_t)s.E + 1));
            std::memcpy(s.vtx.data(), s.d_vtx.data(), sizeof(pv_vertex) * (size_t)s.records);
            std::memcpy(s.tv.data(), s.d_tv.data(), sizeof(int32_t) * (size_t)s.T);
            std::memcpy(s.tw.data(), s.d_tw.data(), sizeof(float) * (size_t)s.T);
        } else {
            std::memcpy(s.vtx.data() + s.from, s.d_vtx.data() + s.from, sizeof(pv_vertex) * (size_t)s.count);
        }
        s.pending = 0;
        return PV_OK;
    }

    int fetch(int slot, int from, int count) override
    {
        FakeSlot &s = slots_[(size_t)slot];
        if (s.pending != 0 || from < 0 || count < 1 || from + count > s.d_first[(size_t)s.E])
            return pvk::set_error(PV_EINVAL, "fake device: bad fetch [%d, %d) of slot %d", from, from + count, slot);
        ++fake::knobs().fetches;
        s.from = from;
        s.count = count;
        s.pending = 2;
        s.done_at = now_ns() + 250ll * fake::knobs().latency_us.load();
        return PV_OK;
    }

    void synchronize() override
    {
        for (size_t k = 0; k < slots_.size(); ++k)
            while (query((int)k) == 1) {
            }
    }

private:
    std::vector<float> snapshot(const FakeSlot &s) const
    {
        std::vector<float> v;
        for (int k = 0; k < 8; ++k)
            v.insert(v.end(), s.h.trk[k], s.h.trk[k] + s.T);
        for (int e = 0; e <= s.E; ++e)
            v.push_back((float)s.offsets[(size_t)e]);
        return v;
    }

    void compute(FakeSlot &s)
    {
        s.d_nv.assign((size_t)s.E, 0);
        s.d_status.assign((size_t)s.E, 0);
        s.d_first.assign((size_t)s.E + 1, 0);
        s.d_tv.assign((size_t)s.T, 0);
        s.d_tw.assign((size_t)s.T, 0.0f);
        s.d_vtx.assign((size_t)s.E * (size_t)max_v_, pv_vertex());
        std::vector<pv_vertex> ev((size_t)max_v_);
        int total = 0;
        for (int e = 0; e < s.E; ++e) {
            const int a = s.offsets[(size_t)e], b = s.offsets[(size_t)e + 1];
            fake::event_result(s.h.trk, a, b - a, max_v_, &s.d_nv[(size_t)e], &s.d_status[(size_t)e], ev.data(),
                               s.d_tv.data() + a, s.d_tw.data() + a);
            s.d_first[(size_t)e] = total;
            std::memcpy(s.d_vtx.data() + total, ev.data(), sizeof(pv_vertex) * (size_t)s.d_nv[(size_t)e]);
            total += s.d_nv[(size_t)e];
        }
        s.d_first[(size_t)s.E] = total;
    }

    pv_server_config cfg_;
    int max_v_;
    int64_t bytes_ = 0;
    std::vector<FakeSlot> slots_;
};

}  // namespace

namespace pvk {

int make_server_device(const pv_server_config &config, const pv_params &params, const KParams &,
                       const pv_schedule &, std::unique_ptr<ServerDevice> *out)
{
    if (fake::knobs().fail_create.load())
        return set_error(PV_ENOMEM, "fake device: allocation refused");
    out->reset(new FakeServerDevice(config, params));
    return PV_OK;
}

}  // namespace pvk
