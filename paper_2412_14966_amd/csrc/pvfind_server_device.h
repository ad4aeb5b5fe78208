// pvfind_server_device.h -- what the continuous-batching server asks of the
// device: batch slots, each with host staging buffers, that run one batch at
// a time, asynchronously.  pvfind_server_hip.cpp implements it with the
// pv_find kernels on HIP streams; the server's own logic (pvfind_server.cpp)
// holds no device code, so that it also runs against a CPU stand-in.
#pragma once

#include <stdint.h>

#include <memory>

#include "pvfind_internal.h"

namespace pvk {

// Host staging of one slot (pinned memory on the device implementation).
// The server writes a batch's track columns (the batch's tracks one after
// another in each) and offsets[0 .. n_events] before dispatch, and reads the
// results once the slot reports the batch finished.
struct SlotHost {
    float *trk[8] = {};         // x, y, z, tx, ty, cov_xx, cov_xtx, cov_txtx: max_tracks_per_batch each
    int32_t *offsets = nullptr; // max_events_per_batch + 1
    int32_t *nv = nullptr;      // vertices written per event
    int32_t *status = nullptr;  // PV_EV_* bits per event
    int32_t *first = nullptr;   // max_events_per_batch + 1: each event's first record in vtx, then the total
    pv_vertex *vtx = nullptr;   // the written vertex records, event after event
    int32_t *tv = nullptr;      // per-track vertex index (pv_track_out.vertex)
    float *tw = nullptr;        // per-track weight
};

class ServerDevice {
public:
    virtual ~ServerDevice() = default;
    // Device memory the slots hold, in bytes.
    virtual int64_t device_bytes() const = 0;
    virtual const SlotHost &host(int slot) const = 0;
    // Make the calling thread's device calls go to the server's device.
    virtual void bind_thread() = 0;
    // Start the batch held in the slot's staging (n_events events, n_tracks
    // tracks): copies in, the find and the record compaction, then copies of
    // the counts, statuses, record offsets, the first `records` records and the
    // per-track outputs back.  Returns PV_OK or an error code (message set).
    virtual int dispatch(int slot, int n_events, int n_tracks, int records) = 0;
    // 0 when the slot's last dispatch or fetch has completed, 1 while it runs,
    // an error code (message set) when it failed.
    virtual int query(int slot) = 0;
    // Copy records [from, from + count) of the slot's finished batch back,
    // asynchronously (query reports its completion).
    virtual int fetch(int slot, int from, int count) = 0;
    // Wait until every slot is idle.
    virtual void synchronize() = 0;
};

// Create the device side of a server on the current device: config.n_slots
// slots over config.n_streams streams.  Returns PV_OK, PV_ENOMEM or PV_EHIP.
int make_server_device(const pv_server_config &config, const pv_params &params, const KParams &kp,
                       const pv_schedule &sched, std::unique_ptr<ServerDevice> *out);

// Device bytes of one slot (inputs, outputs, dense records, workspace).
size_t server_slot_bytes(const pv_server_config &c, const pv_params &p);

}  // namespace pvk
