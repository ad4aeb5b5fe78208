// pvfind_api.cpp -- host side of the libpvfind C ABI: argument validation,
// parameter derivation, per-stream device workspace, error reporting.
#include <hip/hip_runtime.h>

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

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

std::mutex g_mu;
pv_schedule g_sched = {2, 512, 4, 0};   // fastest measured at mu = 5 before pv_autotune runs

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
            return fail(PV_EHIP, "hipEventCreate: %s", hipGetErrorString(err));
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
std::map<std::pair<int, void *>, Workspace> g_ws;

int nbins_of(const pv_params *p)
{
    const double span = ((double)p->z_max - (double)p->z_min) / (double)p->dz;
    if (!(p->dz > 0.0f) || !std::isfinite(span))
        return -1;
    const long nb = std::lround(span);
    if (nb < 1 || nb > pvk::kMaxBins || std::fabs(span - (double)nb) > 1e-6 * (double)nb)
        return -1;
    return (int)nb;
}

int validate_schedule(const pv_schedule &s)
{
    if (s.waves_per_team != 1 && s.waves_per_team != 2 && s.waves_per_team != 4)
        return fail(PV_EINVAL, "schedule: waves_per_team must be 1, 2 or 4 (got %d)", s.waves_per_team);
    if (s.track_capacity != 256 && s.track_capacity != 512 && s.track_capacity != 1024 && s.track_capacity != 1536 &&
        s.track_capacity != 2048)
        return fail(PV_EINVAL, "schedule: track_capacity must be 256, 512, 1024, 1536 or 2048 (got %d)",
                    s.track_capacity);
    if (s.persistent < 1 || s.persistent > 4)
        return fail(PV_EINVAL, "schedule: persistent must be 1, 2, 3 or 4 (got %d)", s.persistent);
    if (s.persistent == 1 || s.persistent == 3)
        return fail(PV_EINVAL, "schedule: persistent small-team launches (modes 1 and 3) are disabled; "
                               "use 2 or 4");
    if (s.teams_per_cu < 0 || s.teams_per_cu > 64)
        return fail(PV_EINVAL, "schedule: teams_per_cu out of range (got %d)", s.teams_per_cu);
    return PV_OK;
}

pv_schedule resolve_schedule(const pv_schedule *s)
{
    pv_schedule d;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        d = g_sched;
    }
    if (!s)
        return d;
    pv_schedule r = *s;
    if (r.waves_per_team == 0)
        r.waves_per_team = d.waves_per_team;
    if (r.track_capacity == 0)
        r.track_capacity = d.track_capacity;
    if (r.persistent == 0)
        r.persistent = d.persistent;
    return r;
}

int derive_params(const pv_params *p, const pv_beamline *bl, pvk::KParams &k)
{
    const int nb = nbins_of(p);
    if (nb < 0)
        return fail(PV_EINVAL, "params: (z_max - z_min) / dz must be a whole number of bins in [1, %d]",
                    pvk::kMaxBins);
    if (!std::isfinite(p->z_min) || !std::isfinite(p->z_max) || !std::isfinite(p->z_gas))
        return fail(PV_EINVAL, "params: non-finite histogram range");
    if (!(p->sigma_max_pp > 0.0f) || !(p->sigma_max_gas > 0.0f) || !(p->u0 > 0.0f) ||
        !std::isfinite(p->sigma_max_pp) || !std::isfinite(p->sigma_max_gas) || !std::isfinite(p->u0))
        return fail(PV_EINVAL, "params: sigma_max_pp, sigma_max_gas and u0 must be positive and finite");
    if (p->frac_bits < 1 || p->frac_bits > 18)
        return fail(PV_EINVAL, "params: frac_bits must be in [1, 18] (int32 histogram for 4096 tracks)");
    if (p->proto_thr < 0 || p->dip_prom < 1 || p->min_int_pp < 0 || p->min_int_gas < 0)
        return fail(PV_EINVAL, "params: proto_thr >= 0, dip_prom >= 1, min_int_* >= 0 required");
    if (p->part_min_pp < 0 || p->part_min_gas < 0 || p->pv_min_pp < 0 || p->pv_min_gas < 0)
        return fail(PV_EINVAL, "params: minimum track counts must be >= 0");
    if (p->max_iter < 1 || p->max_iter > 255)
        return fail(PV_EINVAL, "params: max_iter must be in [1, 255]");
    if (!(p->chi2_max > 0.0f) || !(p->conv_dchi2 > 0.0f) || !(p->conv_dz > 0.0f) || !(p->max_rho_pp >= 0.0f) ||
        !(p->cond_fp64 > 0.0f) || !(p->sing_ratio >= 0.0f) || !(p->sing_ratio < 1.0f))
        return fail(PV_EINVAL, "params: chi2_max, conv_dchi2, conv_dz, cond_fp64 > 0, max_rho_pp >= 0 and "
                               "sing_ratio in [0, 1) required");
    if (p->max_tracks_per_event < 0 || p->max_tracks_per_event > pvk::kMaxTracks)
        return fail(PV_EINVAL, "params: max_tracks_per_event must be in [0, %d]", pvk::kMaxTracks);
    if (p->max_vertices_per_event < 1 || p->max_vertices_per_event > pvk::kMaxVertices)
        return fail(PV_EINVAL, "params: max_vertices_per_event must be in [1, %d]", pvk::kMaxVertices);
    if (p->assoc_mode != PV_ASSOC_PARTITION && p->assoc_mode != PV_ASSOC_MULTIVERTEX)
        return fail(PV_EINVAL, "params: assoc_mode must be PV_ASSOC_PARTITION or PV_ASSOC_MULTIVERTEX");
    if (p->assoc_mode == PV_ASSOC_MULTIVERTEX &&
        (!(p->chi2_max_mv > 0.0f) || !(p->chi2_max_mv < 170.0f) || !(p->chi2_window_mv >= 0.0f) ||
         !(p->conv_dz_mv > 0.0f) || !(p->dup_ratio >= 0.0f) || !std::isfinite(p->dup_ratio) ||
         !(p->w_count_mv >= 0.0f) || !(p->w_count_mv <= 1.0f)))
        return fail(PV_EINVAL, "params: chi2_max_mv in (0, 170), chi2_window_mv >= 0, conv_dz_mv > 0, finite "
                               "dup_ratio >= 0 and w_count_mv in [0, 1] required");
    if (p->peak_mode != PV_PEAK_Z_ORDERED && p->peak_mode != PV_PEAK_RECURSIVE)
        return fail(PV_EINVAL, "params: peak_mode must be PV_PEAK_Z_ORDERED or PV_PEAK_RECURSIVE");
    if (!std::isfinite(bl->x) || !std::isfinite(bl->y) || !std::isfinite(bl->tx) || !std::isfinite(bl->ty))
        return fail(PV_EINVAL, "beamline: non-finite value");
    k.z_min = p->z_min;
    k.z_max = p->z_max;
    k.dz = p->dz;
    k.inv_dz = 1.0f / p->dz;
    {
        int ex = 0;
        k.dz_pow2 = (std::frexp(p->dz, &ex) == 0.5f) ? 1 : 0;
    }
    k.edges_exact = 1;
    for (int j = 0; j <= nb && k.edges_exact; ++j) {
        const double jd = (double)j * (double)p->dz, e = (double)p->z_min + jd;
        if ((double)(float)jd != jd || (double)(float)e != e)
            k.edges_exact = 0;
    }
    k.u0 = p->u0;
    k.sigma_max_pp = p->sigma_max_pp;
    k.sigma_max_gas = p->sigma_max_gas;
    k.unit = (float)(1 << p->frac_bits);
    k.nb = nb;
    const double gb = std::floor(((double)p->z_gas - (double)p->z_min) / (double)p->dz);
    k.gas_bin = (int)std::fmax(-1.0, std::fmin((double)nb + 1.0, gb));
    k.proto_thr = p->proto_thr;
    k.dip_prom = p->dip_prom;
    k.min_int_pp = p->min_int_pp;
    k.min_int_gas = p->min_int_gas;
    k.part_min_pp = p->part_min_pp;
    k.part_min_gas = p->part_min_gas;
    k.pv_min_pp = p->pv_min_pp;
    k.pv_min_gas = p->pv_min_gas;
    k.max_iter = p->max_iter;
    k.chi2_max = p->chi2_max;
    k.inv_chi2_max = 1.0f / p->chi2_max;
    k.conv_dchi2 = p->conv_dchi2;
    k.conv_dz = p->conv_dz;
    k.max_rho2_pp = p->max_rho_pp * p->max_rho_pp;
    k.cond_fp64 = p->cond_fp64;
    k.sing_ratio = p->sing_ratio;
    k.max_tracks = p->max_tracks_per_event;
    k.max_vertices = p->max_vertices_per_event;
    k.bx = bl->x;
    k.by = bl->y;
    k.btx = bl->tx;
    k.bty = bl->ty;
    k.mv = p->assoc_mode == PV_ASSOC_MULTIVERTEX ? 1 : 0;
    k.e_max_mv = (float)std::exp(-0.5 * (double)p->chi2_max_mv);
    k.chi2_window_mv = p->chi2_window_mv;
    k.conv_dz_mv = p->conv_dz_mv;
    k.dup_ratio = p->dup_ratio;
    k.w_count_mv = p->w_count_mv;
    k.peak_rec = p->peak_mode == PV_PEAK_RECURSIVE ? 1 : 0;
    return PV_OK;
}

// Workspace of (current device, stream), grown to hold n_events deferred events.
int get_workspace(void *stream, int n_events, pvk::WorkQueue **out, int32_t **order)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return fail(PV_EHIP, "hipGetDevice: %s", hipGetErrorString(err));
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &w = g_ws[std::make_pair(dev, stream)];
    const int need = n_events > 1024 ? n_events : 1024;
    if (w.wq == nullptr || w.capacity < need) {
        if (w.wq != nullptr) {
            // work already queued on this stream may still use the old block
            err = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
            if (err != hipSuccess)
                return fail(PV_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(err));
            (void)hipFree(w.wq);
            w.wq = nullptr;
            w.capacity = 0;
        }
        const size_t bytes = sizeof(pvk::WorkQueue) + 2 * sizeof(int) * (size_t)need;   // deferred list, order
        void *ptr = nullptr;
        err = hipMalloc(&ptr, bytes);
        if (err != hipSuccess)
            return fail(PV_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(err));
        err = hipMemset(ptr, 0, bytes);
        if (err != hipSuccess) {
            (void)hipFree(ptr);
            return fail(PV_EHIP, "hipMemset: %s", hipGetErrorString(err));
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
    if (!tracks || !offsets || !beamline || !params || !ov || !ot)
        return fail(PV_EINVAL, "null argument");
    if (n_events < 0)
        return fail(PV_EINVAL, "n_events < 0");
    if (!tracks->x || !tracks->y || !tracks->z || !tracks->tx || !tracks->ty || !tracks->cov_xx ||
        !tracks->cov_xtx || !tracks->cov_txtx)
        return fail(PV_EINVAL, "null track array");
    if (!ov->vertices || !ov->n_vertices || !ov->status || !ot->vertex || !ot->weight)
        return fail(PV_EINVAL, "null output array");
    pvk::KArgs A;
    std::memset(&A, 0, sizeof(A));
    int rc = derive_params(params, beamline, A.p);
    if (rc != PV_OK)
        return rc;
    const pv_schedule s = resolve_schedule(schedule);
    rc = validate_schedule(s);
    if (rc != PV_OK)
        return rc;
    if (noalloc && n_events > PV_NOALLOC_MAX_EVENTS)
        return fail(PV_EINVAL, "pv_find_noalloc: n_events %d exceeds PV_NOALLOC_MAX_EVENTS (%d)", n_events,
                    PV_NOALLOC_MAX_EVENTS);
    if (n_events == 0)
        return PV_OK;
    int32_t *order = nullptr;
    if (noalloc) {
        int herr = pvk::noalloc_workspace(&A.wq, &order);
        if (herr == (int)hipSuccess)
            herr = pvk::clear_queue(A.wq, stream);
        if (herr != (int)hipSuccess)
            return fail(PV_EHIP, "pv_find_noalloc workspace: %s", hipGetErrorString((hipError_t)herr));
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
        return fail(PV_EHIP, "kernel launch: %s", hipGetErrorString((hipError_t)err));
    return PV_OK;
}

}  // namespace

namespace pvk {

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int derive_kparams(const pv_params *p, const pv_beamline *bl, KParams &k)
{
    if (!p || !bl)
        return fail(PV_EINVAL, "null params or beamline");
    return derive_params(p, bl, k);
}

int schedule_for(const pv_schedule *requested, pv_schedule &out)
{
    out = resolve_schedule(requested);
    return validate_schedule(out);
}

int workspace_for(void *stream, int n_events, WorkQueue **out, int32_t **order)
{
    return get_workspace(stream, n_events, out, order);
}

}  // namespace pvk

extern "C" {

void pv_params_default(pv_params *p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    p->z_min = -600.0f;            // benchmark histogram range; the paper uses [-550, 300] mm
    p->z_max = 400.0f;
    p->dz = 0.25f;                 // Sec. 3.2
    p->z_gas = -300.0f;            // Table 2
    p->sigma_max_pp = 1.5f;        // Sec. 3.2, Table 2
    p->sigma_max_gas = 10.0f;
    p->u0 = 2.13f;                 // parabolic kernel closest to the Gaussian cumulative
    p->frac_bits = 16;
    p->proto_thr = 6554;           // 0.1 track / bin
    p->dip_prom = 131072;          // 2 tracks / bin
    p->min_int_pp = 163840;        // Table 2: 2.5 tracks
    p->min_int_gas = 114688;       // Table 2: 1.75 tracks
    p->part_min_pp = 3;            // Sec. 3.4
    p->part_min_gas = 2;
    p->pv_min_pp = 4;              // Table 2
    p->pv_min_gas = 3;
    p->max_iter = 10;              // Sec. 3.5
    p->chi2_max = 12.0f;           // Eq. 17
    p->conv_dchi2 = 0.01f;         // Sec. 3.5 (x86 criterion)
    p->conv_dz = 0.001f;
    p->max_rho_pp = 0.3f;          // end of Sec. 3.5
    p->cond_fp64 = 1.0e6f;
    p->sing_ratio = 1.0e-4f;       // normal matrix singular below det / prod(diag) = 1e-4
    p->max_tracks_per_event = pvk::kMaxTracks;
    p->max_vertices_per_event = pvk::kMaxVertices;
    // GPU variant (Sec. 3.5, Sec. 5).  The paper's illustration of Eq. 18 uses
    // a cut-off of 4, with which an uncontested weight follows the Tukey weight
    // at 12 as the text says; it gives no value for the chi2 pre-cut (25
    // leaves out tracks of uncontested weight below 3e-5 at the seed); the
    // duplicate test reads as dz^2 / (Czz_1 + Czz_2) < 25.
    p->assoc_mode = PV_ASSOC_PARTITION;
    p->chi2_max_mv = 4.0f;
    p->chi2_window_mv = 25.0f;
    p->conv_dz_mv = 0.0005f;       // Sec. 3.5, GPU criterion: 0.5 micrometre
    p->dup_ratio = 25.0f;
    p->w_count_mv = 0.5f;
    p->peak_mode = PV_PEAK_Z_ORDERED;
}

int32_t pv_nbins(const pv_params *p)
{
    if (!p)
        return -1;
    return nbins_of(p);
}

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
        return fail(PV_EINVAL, "null debug argument");
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
            k == key && validate_schedule(s) == PV_OK) {
            out = s;   // the last matching line wins
            found = true;
        }
    }
    return found;
}

}  // namespace

extern "C" {

int pv_autotune(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                const pv_beamline *beamline, const pv_params *params, pv_vertices_out *out_vertices,
                pv_track_out *out_track_weights, int32_t reps, const char *cache_path, const char *key,
                int32_t force, pv_schedule *best, double *best_us, void *stream)
{
    if (reps < 1)
        return fail(PV_EINVAL, "autotune: reps must be >= 1");
    if (cache_path && !key)
        return fail(PV_EINVAL, "autotune: a cache needs a key");
    if (key && (std::strchr(key, '\t') || std::strchr(key, '\n')))
        return fail(PV_EINVAL, "autotune: key must not contain tabs or newlines");
    const std::string dev = device_tag();
    pv_schedule chosen{};
    double chosen_us = 0.0;
    if (cache_path && !force && read_cache(cache_path, dev, key, chosen)) {
        int rc = pv_set_schedule(&chosen);
        if (rc == PV_OK) {
            if (best)
                *best = chosen;
            if (best_us)
                *best_us = 0.0;
        }
        return rc;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return fail(PV_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PV_EHIP, "hipEventCreate failed");
    }
    int rc = PV_OK;
    bool have = false;
    const int waves[3] = {1, 2, 4}, caps[5] = {256, 512, 1024, 1536, 2048}, modes[2] = {2, 4};
    for (int w : waves)
        for (int c : caps)
            for (int m : modes) {
                if (rc != PV_OK)
                    break;
                const pv_schedule s = {w, c, m, 0};
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
                    rc = fail(PV_EHIP, "autotune timing: %s", hipGetErrorString(err));
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
        return rc != PV_OK ? rc : fail(PV_EINVAL, "autotune: nothing timed");
    // leave the winner's results in the outputs
    rc = find_impl(tracks, event_offsets, n_events, beamline, params, out_vertices, out_track_weights, nullptr,
                   &chosen, stream);
    if (rc == PV_OK) {
        const hipError_t err = hipStreamSynchronize(st);
        if (err != hipSuccess)
            rc = fail(PV_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(err));
    }
    if (rc != PV_OK)
        return rc;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (!f)
            return fail(PV_EINVAL, "autotune: cannot append to %s", cache_path);
        f << dev << '\t' << key << '\t' << chosen.waves_per_team << ' ' << chosen.track_capacity << ' '
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

int pv_set_schedule(const pv_schedule *schedule)
{
    if (!schedule)
        return fail(PV_EINVAL, "null schedule");
    const int rc = validate_schedule(*schedule);
    if (rc != PV_OK)
        return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_sched = *schedule;
    return PV_OK;
}

int pv_get_schedule(pv_schedule *schedule)
{
    if (!schedule)
        return fail(PV_EINVAL, "null schedule");
    std::lock_guard<std::mutex> lk(g_mu);
    *schedule = g_sched;
    return PV_OK;
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
            rc = fail(PV_EHIP, "timing events: %s", hipGetErrorString(err));
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

const char *pv_last_error(void)
{
    return g_err;
}

const char *pv_version(void)
{
    return "pvfind 0.1 (gfx950)";
}

}  // extern "C"
