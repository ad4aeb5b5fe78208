// fake_server_device.h -- a CPU stand-in for the server's device side
// (pvk::ServerDevice), for host-only tests of the server's batching,
// completion and error logic under sanitizers.  Its "find" is a cheap
// deterministic function of each event's tracks, not the method.
#pragma once

#include <atomic>
#include <cstdint>

#include "pvfind.h"

namespace fake {

struct Knobs {
    std::atomic<int> latency_us{30};        // how long a dispatched batch runs
    std::atomic<int> fail_create{0};        // make_server_device returns PV_ENOMEM
    std::atomic<int> fail_dispatch_at{-1};  // the n-th dispatch (from 0) fails
    std::atomic<int> fail_batch_at{-1};     // the n-th batch to finish (from 0) reports a device error
    std::atomic<int> batches_done{0};
    std::atomic<int> dispatches{0};
    std::atomic<int> fetches{0};            // second copies of vertex records
    std::atomic<int> staging_violations{0}; // staging changed while its batch ran
    std::atomic<int> live_devices{0};
};

Knobs &knobs();

// The stand-in's result for one event of n tracks (columns trk[0..7], rows
// first .. first + n - 1): vertex count (at most max_v), status, records and
// per-track outputs (tv, tw indexed from 0).
void event_result(const float *const trk[8], int first, int n, int max_v, int32_t *nv, int32_t *status,
                  pv_vertex *vtx, int32_t *tv, float *tw);

}  // namespace fake
