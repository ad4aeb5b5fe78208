// pvfind_api.cpp -- host side of the libpvfind C ABI that drives the device:
// per-stream device workspace, the find calls' launches, autotuning and the
// benchmark timing records (validation and parameters: pvfind_params.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "pvfind_internal.h"

namespace {

// benchmark timing records
std::mutex g_tmu;
bool g_timing = false;
std::vector<pvk::LaunchEvents> g_records;

void destroy_events(pvk::LaunchEvents &e)
{
    for (void *p : {e.main_begin, e.main_end, e.large_begin, e.large_end})
        if (p)
            (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(p));
    e = pvk::LaunchEvents();
}

int create_events(pvk::LaunchEvents &e)
{
    void **slots[4] = {&e.main_begin, &e.main_end, &e.large_begin, &e.large_end};
    for (void **s : slots) {
        hipEvent_t h;
        const hipError_t err = hipEventCreate(&h);
        if (err != hipSuccess) {
            destroy_events(e);
            return pvk::set_error(PV_EHIP, "hipEventCreate: %s", hipGetErrorString(err));
        }
        *s = h;
    }
    return PV_OK;
}

struct Workspace {
    pvk::WorkQueue *wq = nullptr;
    int capacity = 0;   // events the deferred list can hold
};
// keyed by (device, stream)
std::mutex g_wsmu;
std::map<std::pair<int, void *>, Workspace> g_ws;

// Workspace of (current device, stream), grown to hold n_events deferred events.
int get_workspace(void *stream, int n_events, pvk::WorkQueue **out, int32_t **order)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "hipGetDevice: %s", hipGetErrorString(err));
    std::lock_guard<std::mutex> lk(g_wsmu);
    Workspace &w = g_ws[std::make_pair(dev, stream)];
    const int need = n_events > 1024 ? n_events : 1024;
    if (w.wq == nullptr || w.capacity < need) {
        if (w.wq != nullptr) {
            // work already queued on this stream may still use the old block
            err = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
            if (err != hipSuccess)
                return pvk::set_error(PV_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(err));
            (void)hipFree(w.wq);
            w.wq = nullptr;
            w.capacity = 0;
        }
        const size_t bytes = sizeof(pvk::WorkQueue) + 2 * sizeof(int) * (size_t)need;   // deferred list, order
        void *ptr = nullptr;
        err = hipMalloc(&ptr, bytes);
        if (err != hipSuccess)
            return pvk::set_error(PV_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(err));
        err = hipMemset(ptr, 0, bytes);
        if (err != hipSuccess) {
            (void)hipFree(ptr);
            return pvk::set_error(PV_EHIP, "hipMemset: %s", hipGetErrorString(err));
        }
        w.wq = static_cast<pvk::WorkQueue *>(ptr);
        w.capacity = need;
    }
    *out = w.wq;
    *order = pvk::order_list(w.wq, w.capacity);
    return PV_OK;
}

int find_impl(const pv_tracks *tracks, const int32_t *offsets, int32_t n_events, const pv_beamline *beamline,
              const pv_params *params, pv_vertices_out *ov, pv_track_out *ot, const pv_debug_out *dbg,
              const pv_schedule *schedule, void *stream, bool noalloc = false)
{
    int rc = pvk::check_find_args(tracks, offsets, n_events, beamline, params, ov, ot);
    if (rc != PV_OK)
        return rc;
    pvk::KArgs A;
    std::memset(&A, 0, sizeof(A));
    rc = pvk::derive_kparams(params, beamline, A.p);
    if (rc != PV_OK)
        return rc;
    const pv_schedule s = pvk::resolve_schedule(schedule);
    rc = pvk::validate_schedule(s);
    if (rc != PV_OK)
        return rc;
    if (noalloc && n_events > PV_NOALLOC_MAX_EVENTS)
        return pvk::set_error(PV_EINVAL, "pv_find_noalloc: n_events %d exceeds PV_NOALLOC_MAX_EVENTS (%d)", n_events,
                    PV_NOALLOC_MAX_EVENTS);
    if (n_events == 0)
        return PV_OK;
    int32_t *order = nullptr;
    if (noalloc) {
        int herr = pvk::noalloc_workspace(&A.wq, &order);
        if (herr == (int)hipSuccess)
            herr = pvk::clear_queue(A.wq, stream);
        if (herr != (int)hipSuccess)
            return pvk::set_error(PV_EHIP, "pv_find_noalloc workspace: %s", hipGetErrorString((hipError_t)herr));
    } else {
        rc = get_workspace(stream, n_events, &A.wq, &order);
        if (rc != PV_OK)
            return rc;
    }
    A.order = (s.persistent >= 3) ? order : nullptr;
    A.x = tracks->x;
    A.y = tracks->y;
    A.z = tracks->z;
    A.tx = tracks->tx;
    A.ty = tracks->ty;
    A.cxx = tracks->cov_xx;
    A.cxtx = tracks->cov_xtx;
    A.ctxtx = tracks->cov_txtx;
    A.offsets = offsets;
    A.n_events = n_events;
    A.vout = ov->vertices;
    A.nv_out = ov->n_vertices;
    A.status_out = ov->status;
    A.trk_vtx = ot->vertex;
    A.trk_w = ot->weight;
    const bool debug = dbg != nullptr;
    if (debug) {
        A.dbg_hist = dbg->hist;
        A.dbg_cl = dbg->clusters;
        A.dbg_ncl = dbg->n_clusters;
        A.dbg_zp = dbg->zpoca;
        A.dbg_sg = dbg->sigma;
        A.dbg_bin = dbg->bin;
        A.dbg_cycles = dbg->stage_cycles;
    }
    bool timing = false;
    if (!noalloc) {
        std::lock_guard<std::mutex> lk(g_tmu);
        timing = g_timing;
    }
    pvk::LaunchEvents ev;
    if (timing) {
        rc = create_events(ev);
        if (rc != PV_OK)
            return rc;
    }
    const int err = pvk::launch_batch(A, s, debug, stream, timing ? &ev : nullptr);
    if (timing) {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_records.push_back(ev);
    }
    if (err != (int)hipSuccess)
        return pvk::set_error(PV_EHIP, "kernel launch: %s", hipGetErrorString((hipError_t)err));
    return PV_OK;
}

}  // namespace

namespace pvk {

int workspace_for(void *stream, int n_events, WorkQueue **out, int32_t **order)
{
    return get_workspace(stream, n_events, out, order);
}

}  // namespace pvk

extern "C" {

int pv_find(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events, const pv_beamline *beamline,
            const pv_params *params, pv_vertices_out *out_vertices, pv_track_out *out_track_weights, void *stream)
{
    return find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights, nullptr,
                     nullptr, stream);
}

int pv_find_noalloc(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                    const pv_beamline *beamline, const pv_params *params, pv_vertices_out *out_vertices,
                    pv_track_out *out_track_weights, void *stream)
{
    return find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights, nullptr,
                     nullptr, stream, true);
}

int pv_find_sched(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                  const pv_beamline *beamline, const pv_params *params, pv_vertices_out *out_vertices,
                  pv_track_out *out_track_weights, const pv_schedule *schedule, void *stream)
{
    return find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights, nullptr,
                     schedule, stream);
}

int pv_find_debug(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                  const pv_beamline *beamline, const pv_params *params, pv_vertices_out *out_vertices,
                  pv_track_out *out_track_weights, const pv_debug_out *debug, const pv_schedule *schedule,
                  void *stream)
{
    if (!debug)
        return pvk::set_error(PV_EINVAL, "null debug argument");
    return find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights, debug,
                     schedule, stream);
}

}  // extern "C"

namespace {

std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string s = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    for (char &c : s)
        if (c == '\t' || c == '\n' || c == ' ')
            c = '_';
    return s;
}

bool read_cache(const char *path, const std::string &dev, const std::string &key, pv_schedule &out)
{
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream ls(line);
        std::string d, k;
        pv_schedule s;
        double us;
        if (std::getline(ls, d, '\t') && std::getline(ls, k, '\t') &&
            (ls >> s.waves_per_team >> s.track_capacity >> s.persistent >> s.teams_per_cu >> us) && d == dev &&
            k == key && pvk::validate_schedule(s) == PV_OK) {
            out = s;   // the last matching line wins
            found = true;
        }
    }
    return found;
}

// Shape of a batch for the autotuner's cache: the event count and the
// track-count distribution (median, 90th and 99th percentiles, maximum), each
// in quarter-octave buckets (about 19 % wide), and the association and
// splitting variants, which select different kernels.  Batches of one shape
// share a cache entry; another pile-up or batch size gets its own.
int workload_shape(const int32_t *offsets, int n_events, const pv_params *p, hipStream_t st, std::string &out)
{
    std::vector<int32_t> off((size_t)n_events + 1);
    hipError_t err = hipMemcpyAsync(off.data(), offsets, sizeof(int32_t) * off.size(), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess)
        err = hipStreamSynchronize(st);
    if (err != hipSuccess)
        return pvk::set_error(PV_EHIP, "autotune: reading the offsets: %s", hipGetErrorString(err));
    std::vector<int> n((size_t)n_events);
    for (int e = 0; e < n_events; ++e) {
        const int a = off[(size_t)e], b = off[(size_t)e + 1];
        n[(size_t)e] = (a >= 0 && b >= a) ? b - a : 0;
    }
    std::sort(n.begin(), n.end());
    auto bucket = [](double x) { return x < 1.0 ? 0 : 1 + (int)std::floor(4.0 * std::log2(x)); };
    auto q = [&](double f) { return n.empty() ? 0.0 : (double)n[(size_t)std::min<double>(f * n.size(), n.size() - 1)]; };
    std::ostringstream o;
    o << "E" << bucket((double)n_events) << ".p50_" << bucket(q(0.5)) << ".p90_" << bucket(q(0.9)) << ".p99_"
      << bucket(q(0.99)) << ".max" << bucket(n.empty() ? 0.0 : (double)n.back()) << ".a" << p->assoc_mode << "p"
      << p->peak_mode;
    out = o.str();
    return PV_OK;
}

}  // namespace

extern "C" {

int pv_autotune(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                const pv_beamline *beamline, const pv_params *params, pv_vertices_out *out_vertices,
                pv_track_out *out_track_weights, int32_t reps, const char *cache_path, const char *key,
                int32_t force, pv_schedule *best, double *best_us, void *stream)
{
    if (reps < 1)
        return pvk::set_error(PV_EINVAL, "autotune: reps must be >= 1");
    if (key && (std::strchr(key, '\t') || std::strchr(key, '\n')))
        return pvk::set_error(PV_EINVAL, "autotune: key must not contain tabs or newlines");
    int rc = pvk::check_find_args(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights);
    if (rc != PV_OK)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const std::string dev = device_tag();
    std::string entry;   // the cache key: the caller's key and the batch's shape
    if (cache_path) {
        std::string shape;
        rc = workload_shape(event_offsets, n_events, params, st, shape);
        if (rc != PV_OK)
            return rc;
        entry = std::string(key ? key : "") + "|" + shape;
    }
    pv_schedule chosen{};
    double chosen_us = 0.0;
    if (cache_path && !force && read_cache(cache_path, dev, entry, chosen)) {
        int rc = pv_set_schedule(&chosen);
        if (rc == PV_OK) {
            if (best)
                *best = chosen;
            if (best_us)
                *best_us = 0.0;
        }
        return rc;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return pvk::set_error(PV_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return pvk::set_error(PV_EHIP, "hipEventCreate failed");
    }
    bool have = false;
    const int waves[4] = {1, 2, 4, 8}, caps[5] = {256, 512, 1024, 1536, 2048}, modes[2] = {2, 4};
    for (int w : waves)
        for (int c : caps)
            for (int m : modes) {
                if (rc != PV_OK)
                    break;
                const pv_schedule s = {w, c, m, 0};
                if (w == 8 && c < 1024)
                    continue;   // not a schedule (pvk::validate_schedule)
                rc = find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights,
                               nullptr, &s, stream);   // warm-up, also validates the arguments
                if (rc != PV_OK)
                    break;
                hipError_t err = hipEventRecord(e0, st);
                for (int r = 0; r < reps && rc == PV_OK && err == hipSuccess; ++r)
                    rc = find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices,
                                   out_track_weights, nullptr, &s, stream);
                if (rc != PV_OK)
                    break;
                if (err == hipSuccess)
                    err = hipEventRecord(e1, st);
                if (err == hipSuccess)
                    err = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (err == hipSuccess)
                    err = hipEventElapsedTime(&ms, e0, e1);
                if (err != hipSuccess) {
                    rc = pvk::set_error(PV_EHIP, "autotune timing: %s", hipGetErrorString(err));
                    break;
                }
                const double us = 1e3 * (double)ms / reps;
                if (!have || us < chosen_us) {
                    chosen = s;
                    chosen_us = us;
                    have = true;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PV_OK || !have)
        return rc != PV_OK ? rc : pvk::set_error(PV_EINVAL, "autotune: nothing timed");
    // leave the winner's results in the outputs
    rc = find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights, nullptr,
                   &chosen, stream);
    if (rc == PV_OK) {
        const hipError_t err = hipStreamSynchronize(st);
        if (err != hipSuccess)
            rc = pvk::set_error(PV_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(err));
    }
    if (rc != PV_OK)
        return rc;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (!f)
            return pvk::set_error(PV_EINVAL, "autotune: cannot append to %s", cache_path);
        f << dev << '\t' << entry << '\t' << chosen.waves_per_team << ' ' << chosen.track_capacity << ' '
          << chosen.persistent << ' ' << chosen.teams_per_cu << ' ' << chosen_us << '\n';
    }
    rc = pv_set_schedule(&chosen);
    if (rc == PV_OK) {
        if (best)
            *best = chosen;
        if (best_us)
            *best_us = chosen_us;
    }
    return rc;
}

int pv_timing_start(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &r : g_records)
        destroy_events(r);
    g_records.clear();
    g_timing = true;
    return PV_OK;
}

int pv_timing_stop(double *main_ms, double *large_ms, int64_t *n_calls)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = false;
    double tm = 0.0, tl = 0.0;
    int rc = PV_OK;
    for (auto &r : g_records) {
        float ms = 0.0f;
        hipError_t err = hipEventSynchronize(reinterpret_cast<hipEvent_t>(r.large ? r.large_end : r.main_end));
        if (err == hipSuccess)
            err = hipEventElapsedTime(&ms, reinterpret_cast<hipEvent_t>(r.main_begin),
                                      reinterpret_cast<hipEvent_t>(r.main_end));
        if (err == hipSuccess) {
            tm += ms;
            if (r.large) {
                err = hipEventElapsedTime(&ms, reinterpret_cast<hipEvent_t>(r.large_begin),
                                          reinterpret_cast<hipEvent_t>(r.large_end));
                if (err == hipSuccess)
                    tl += ms;
            }
        }
        if (err != hipSuccess && rc == PV_OK)
            rc = pvk::set_error(PV_EHIP, "timing events: %s", hipGetErrorString(err));
    }
    if (n_calls)
        *n_calls = (int64_t)g_records.size();
    for (auto &r : g_records)
        destroy_events(r);
    g_records.clear();
    if (main_ms)
        *main_ms = tm;
    if (large_ms)
        *large_ms = tl;
    return rc;
}

}  // extern "C"
