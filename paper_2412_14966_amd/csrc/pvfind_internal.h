// pvfind_internal.h -- definitions shared by the host API and the gfx950 kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "pvfind.h"

namespace pvk {

constexpr int kMaxBins = 4096;      // histogram bins held in LDS
constexpr int kMaxVertices = 128;   // seed clusters / vertices per event
constexpr int kMaxTracks = 4096;    // tracks per event
constexpr int kBigWaves = 8;        // wavefronts of a large-event team
constexpr int kBigCapacity = 4096;  // tracks held in LDS by a large-event team

// per-track flags packed into the LDS track word
constexpr int kTrHist = 1;
constexpr int kTrAssoc = 2;
constexpr int kTrNonfinite = 4;

// Parameters as the kernels use them, derived once on the host.
struct KParams {
    float z_min, z_max, dz, u0, inv_dz;
    float sigma_max_pp, sigma_max_gas;
    float unit;                 // 2^frac_bits
    int nb, gas_bin;
    int proto_thr, dip_prom, min_int_pp, min_int_gas;
    int part_min_pp, part_min_gas, pv_min_pp, pv_min_gas;
    int max_iter;
    float chi2_max, inv_chi2_max, conv_dchi2, conv_dz, max_rho2_pp, cond_fp64, sing_ratio;
    int max_tracks, max_vertices;
    float bx, by, btx, bty;
    // multi-vertex variant (Eq. 18)
    int mv;
    float e_max_mv;             // exp(-chi2_max_mv / 2)
    float chi2_window_mv, conv_dz_mv, dup_ratio, w_count_mv;
    int peak_rec;               // x86 splitting of proto-clusters (Sec. 3.3)
    int dz_pow2;                // dz is a power of two: x / dz == x * inv_dz exactly
    int edges_exact;            // every bin edge z_min + j dz (0 <= j <= nb) is exact in binary32
};

// Device workspace of one stream: work-queue counters, the list of events
// deferred to the large-team launch and, behind it, the processing order of
// the sorted mode (each list holds `capacity` entries).  Counters
// return to zero at the end of every launch (the last workgroup to finish
// resets them).
struct WorkQueue {
    unsigned int next;          // next event index of the main launch
    unsigned int done;          // workgroups of the main launch that finished
    unsigned int n_big;         // events deferred to the large-team launch
    unsigned int next_big;      // next deferred event
    unsigned int done_big;      // workgroups of the large-team launch that finished
    unsigned int pad[11];
    int big[1];                 // capacity entries, then the order list
};

struct KArgs {
    const float *x, *y, *z, *tx, *ty, *cxx, *cxtx, *ctxtx;
    const int32_t *offsets;
    int32_t n_events;               // events of the batch, or the capacity when n_events_dev is set
    const int32_t *n_events_dev;    // when set, the batch size is read from device memory (graph replay)
    pv_vertex *vout;
    int32_t *nv_out;
    int32_t *status_out;
    int32_t *trk_vtx;
    float *trk_w;
    int32_t *dbg_hist;
    pv_cluster *dbg_cl;
    int32_t *dbg_ncl;
    float *dbg_zp, *dbg_sg;
    int32_t *dbg_bin;
    uint32_t *dbg_cycles;
    WorkQueue *wq;
    int32_t *order;                 // persistent launches: event order (largest first), or null
    KParams p;
};

// Events recorded around the launches of one call (benchmark timing).
struct LaunchEvents {
    void *main_begin = nullptr, *main_end = nullptr;    // hipEvent_t
    void *large_begin = nullptr, *large_end = nullptr;  // hipEvent_t, unused when no large launch
    bool large = false;
};

// Host helpers shared by the C ABI files (pvfind_params.cpp, which needs no
// device, defines the first six).
// Record the calling thread's error message (pv_last_error) and return code.
int set_error(int code, const char *fmt, ...);
// Validate params and beamline and derive the kernels' parameters.
int derive_kparams(const pv_params *p, const pv_beamline *bl, KParams &k);
// A requested schedule with its zero fields taken from the process default.
pv_schedule resolve_schedule(const pv_schedule *requested);
int validate_schedule(const pv_schedule &s);
// resolve_schedule, then validate_schedule.
int schedule_for(const pv_schedule *requested, pv_schedule &out);
// Null and count checks of the find calls' arguments.
int check_find_args(const pv_tracks *tracks, const int32_t *offsets, int32_t n_events, const pv_beamline *beamline,
                    const pv_params *params, const pv_vertices_out *ov, const pv_track_out *ot);
int workspace_for(void *stream, int n_events, WorkQueue **out, int32_t **order);

// Device address of the order list of a workspace with `capacity` entries per list.
inline int32_t *order_list(WorkQueue *wq, int capacity)
{
    return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(wq) + offsetof(WorkQueue, big)) + capacity;
}

// Workspace of the allocation-free entry point on the current device (a
// file-scope device array of the kernel file, PV_NOALLOC_MAX_EVENTS events),
// and a launch that zeroes its counters on `stream`.  Return hipError_t values.
int noalloc_workspace(WorkQueue **wq, int32_t **order);
int clear_queue(WorkQueue *wq, void *stream);

// Gather the written vertex records of n_events events (read from
// n_events_dev when set, n_events its upper bound) into `dense`, with the
// per-event offsets and total in first[0 .. n_events].  Returns a hipError_t.
int launch_compact(const pv_vertex *slots, const int32_t *nv, const int32_t *n_events_dev, int n_events, int max_v,
                   pv_vertex *dense, int32_t *first, void *stream);

// Launch one batch on `stream` with schedule `s` (already validated).  With
// `ev`, events are recorded around the launches.  Returns a hipError_t value.
int launch_batch(const KArgs &args, const pv_schedule &s, bool debug, void *stream, LaunchEvents *ev);

}  // namespace pvk
