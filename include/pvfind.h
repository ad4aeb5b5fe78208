/*
 * pvfind.h -- C ABI of libpvfind, primary-vertex finding on AMD Instinct
 * MI355X (gfx950) after "A parallel algorithm for fast reconstruction of
 * primary vertices on heterogeneous architectures" (LHCb, arXiv:2412.14966).
 *
 * Per event the library runs the five steps of the paper's Sec. 3:
 *   1. project every track to its point of closest approach to the beamline
 *      (z_poca, Eq. 1) with uncertainty sigma_poca (Eq. 3);
 *   2. fill a z histogram in which each track spreads one unit of mass over
 *      the bins around z_poca (Sec. 3.2);
 *   3. find proto-clusters, split them at significant minima and place one
 *      seed per cluster (Sec. 3.3, Eq. 4-5);
 *   4. associate every track to one cluster through partition points,
 *      removing clusters with too few tracks (Sec. 3.4);
 *   5. fit each cluster's vertex with the Tukey-weighted Newton-Raphson fit
 *      (Sec. 3.5, Eq. 6-17) and apply the final selection (Table 2, end of
 *      Sec. 3.5).
 *
 * Conventions for every entry point:
 *  - Track, offset and output pointers are DEVICE pointers (HIP device
 *    memory of the current device).  Structs passed by pointer to an entry
 *    point (pv_tracks, pv_params, ...) are HOST memory and are read before
 *    the call returns.
 *  - The caller owns every buffer.  The library owns only its internal
 *    workspace (a few KiB per stream, plus 4 bytes per event of the largest
 *    batch seen) and never frees caller memory.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    default stream); outputs are valid once the caller synchronises it.
 *    Calls on different streams are independent.  Calls that share a stream
 *    are serialised by it.
 *  - Return value: PV_OK (0) or a negative PV_E* code; pv_last_error()
 *    describes the last failure of the calling thread.  No C++ exception
 *    crosses this interface.  Problems found on the device in one event
 *    never abort the batch: they set that event's status bits.
 */
#ifndef PVFIND_H
#define PVFIND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PV_OK        0
#define PV_EINVAL  (-1)   /* null pointer, negative count, inconsistent parameters */
#define PV_EHIP    (-2)   /* a HIP runtime call failed                               */
#define PV_ENOMEM  (-3)   /* workspace allocation failed                             */
#define PV_EBUSY   (-4)   /* server: no admission possible right now                 */

/* per-event status bits */
#define PV_EV_NONFINITE_INPUT  1  /* some track had a NaN/Inf field; it was skipped     */
#define PV_EV_TOO_MANY_TRACKS  2  /* more than max_tracks_per_event; event skipped      */
#define PV_EV_VERTEX_OVERFLOW  4  /* more seed clusters than max_vertices_per_event;
                                     the first ones in z were kept                      */
#define PV_EV_OFFSETS_INVALID  8  /* offsets of this event out of order or range;
                                     event skipped, its track outputs left untouched    */
#define PV_EV_FIT_FAILED      16  /* a candidate's fit failed and the candidate was
                                     dropped: no track kept weight, or the normal
                                     matrix of the Newton step (Eq. 15) was singular    */

/* per-vertex flag bits */
#define PV_VX_NOT_CONVERGED    1  /* stopped at max_iter (Sec. 3.5 caps the iterations) */
#define PV_VX_FP64_INVERSION   2  /* covariance inverted in binary64 (ill-conditioned)  */

/* Track states at z_trk (Sec. 2: straight VELO tracks with state x, y,
 * tx = dx/dz, ty = dy/dz and covariance V).  Structure of arrays, float32,
 * one entry per track, tracks of event e at [offsets[e], offsets[e+1]).
 * x and y errors are uncorrelated and of identical magnitude (Sec. 3.1), so
 * one set (Vxx, Vxtx, Vtxtx) serves both projections. */
typedef struct {
    const float *x, *y, *z, *tx, *ty;
    const float *cov_xx, *cov_xtx, *cov_txtx;
} pv_tracks;

/* Beamline at z = 0 (Sec. 3: average transverse position and direction). */
typedef struct {
    float x, y, tx, ty;
} pv_beamline;

/* Algorithm parameters; pv_params_default() fills the paper's values where it
 * gives them (Sec. 3.2, 3.4, 3.5, Table 2) and documented choices elsewhere. */
typedef struct {
    float   z_min, z_max, dz;          /* histogram range and bin width (mm)          */
    float   z_gas;                     /* bins below this z use the p-gas settings     */
    float   sigma_max_pp, sigma_max_gas; /* max sigma_poca to enter the histogram (mm)  */
    float   u0;                        /* kernel half-width in units of sigma_poca     */
    int32_t frac_bits;                 /* one track = 2^frac_bits histogram units      */
    int32_t proto_thr;                 /* proto-cluster threshold (units, bin > thr)   */
    int32_t dip_prom;                  /* significance of a minimum/maximum (units)    */
    int32_t min_int_pp, min_int_gas;   /* min cluster integral (units, Table 2)        */
    int32_t part_min_pp, part_min_gas; /* min tracks of a partition (Sec. 3.4)         */
    int32_t pv_min_pp, pv_min_gas;     /* min tracks of a final vertex (Table 2)       */
    int32_t max_iter;                  /* fit iteration cap (Sec. 3.5)                 */
    float   chi2_max;                  /* Tukey cut-off (Eq. 17)                       */
    float   conv_dchi2, conv_dz;       /* convergence: |dchi2| and |dz_vtx| (mm)       */
    float   max_rho_pp;                /* pp vertices within this distance of the beam */
    float   cond_fp64;                 /* covariance inverted in binary64 above this
                                          1-norm condition number                      */
    float   sing_ratio;                /* the fit fails when the normal matrix has
                                          det <= sing_ratio * product of its diagonal
                                          (e.g. a single weighted track)               */
    int32_t max_tracks_per_event;      /* <= 4096                                      */
    int32_t max_vertices_per_event;    /* <= 128; output slots per event               */
    /* Association and fit variant.  PV_ASSOC_PARTITION (default): each track
     * goes to the candidate owning its bin (Sec. 3.4), Tukey-weighted fit
     * (Eq. 17), the x86 convergence criterion.  PV_ASSOC_MULTIVERTEX: the GPU
     * variant of Sec. 3.5 and Sec. 5, every track weighted to every candidate
     * with Eq. 18, the other candidates held at their seeds; a candidate fits
     * the tracks whose chi2 at its seed (in binary32) is below chi2_window_mv;
     * converged when |dz| < conv_dz_mv; duplicates (dz^2 / (Czz_1 + Czz_2) <
     * dup_ratio) lose the one with fewer tracks; a vertex's n_tracks counts
     * the tracks with final weight >= w_count_mv; all candidates' track lists
     * together hold at most max_tracks_per_event entries (else the event is
     * flagged PV_EV_TOO_MANY_TRACKS).                                           */
    int32_t assoc_mode;
    float   chi2_max_mv;               /* Eq. 18 cut-off: uncontested weight 1/2 here  */
    float   chi2_window_mv;            /* pre-cut at the seed                          */
    float   conv_dz_mv;                /* mm                                           */
    float   dup_ratio;
    float   w_count_mv;
    /* Splitting of proto-clusters (Sec. 3.3).  PV_PEAK_Z_ORDERED (default, the
     * GPU variant): significant minima taken in z order.  PV_PEAK_RECURSIVE
     * (the x86 variant): the smallest significant minimum between the two
     * largest maxima, then each part the same way; ties go to the lower z, a
     * cut needs both parts to reach their integral threshold.                */
    int32_t peak_mode;
} pv_params;

#define PV_ASSOC_PARTITION   0
#define PV_ASSOC_MULTIVERTEX 1
#define PV_PEAK_Z_ORDERED    0
#define PV_PEAK_RECURSIVE    1

/* One fitted vertex, 64 bytes. */
typedef struct {
    float   x, y, z;                   /* mm */
    float   cov[6];                    /* xx, xy, yy, xz, yz, zz (Eq. 14)              */
    float   chi2;                      /* sum_i w_i chi2_i at the final position      */
    float   ndof;                      /* 2 sum_i w_i - 3                              */
    float   z_seed;                    /* Eq. 4                                        */
    int32_t n_tracks;                  /* tracks associated through the partition;
                                          multi-vertex: tracks of weight >= w_count_mv */
    int16_t bin_lo, bin_hi;            /* seed cluster bin range                      */
    int16_t peak_bin;                  /* highest bin of the seed cluster             */
    uint8_t n_iter;                    /* fit iterations                               */
    uint8_t flags;                     /* PV_VX_* bits                                 */
    int32_t reserved;
} pv_vertex;

typedef struct {
    pv_vertex *vertices;               /* n_events * max_vertices_per_event slots;
                                          event e's vertices at e * max_vertices, in z
                                          order of their seeds                         */
    int32_t   *n_vertices;             /* n_events                                      */
    int32_t   *status;                 /* n_events, PV_EV_* bits                        */
} pv_vertices_out;

/* Per input track: index of its vertex within the event (-1 if none) and its
 * final weight (0 if none).  Multi-vertex: the written vertex that gives the
 * track its largest weight (the earlier one when equal to 2^-16). */
typedef struct {
    int32_t *vertex;
    float   *weight;
} pv_track_out;

/* Seed cluster as found by step 3 and treated by step 4 (debug output). */
typedef struct {
    int32_t lo, hi, peak;              /* bin range and first highest bin              */
    float   z_seed;
    int32_t kept;                      /* 1 if it survived the association step        */
    int32_t n_assoc;                   /* its tracks after the association step
                                          (multi-vertex: tracks passing its pre-cut)   */
    int32_t own_lo, own_hi;            /* bins it owns after the association step
                                          (multi-vertex: -1)                           */
} pv_cluster;

/* Optional intermediate results of pv_find_debug; any member may be NULL. */
typedef struct {
    int32_t    *hist;                  /* n_events * n_bins fixed-point histogram      */
    pv_cluster *clusters;              /* n_events * max_vertices_per_event            */
    int32_t    *n_clusters;            /* n_events: clusters written for the event     */
    float      *zpoca, *sigma;         /* per track, Eq. 1 and Eq. 3                   */
    int32_t    *bin;                   /* per track central bin, -1 outside            */
    uint32_t   *stage_cycles;          /* n_events * 8 shader-clock cycles spent by the
                                          event's team in: clear, project+fill, peak
                                          search, association, gather, fit, selection,
                                          final weights and outputs                    */
} pv_debug_out;

/* How a batch is mapped onto the GPU.  Zero fields mean "library choice". */
typedef struct {
    int32_t waves_per_team;            /* wavefronts cooperating on one event: 1, 2, 4,
                                          or 8 with a track_capacity of 1024 or more  */
    int32_t track_capacity;            /* tracks per event held in LDS by small teams:
                                          256, 512, 1024, 1536 or 2048; larger events go to
                                          a second launch with 4096-track teams       */
    int32_t persistent;                /* 2: one team per event, hardware-scheduled;
                                          4: as 2, teams launched in the order of a
                                          counting sort by decreasing track count
                                          (one small launch first, sorting slices of
                                          up to 1024 events, interleaved).  1 and 3 (a
                                          persistent grid popping a device work queue,
                                          unsorted / sorted) are rejected: with events
                                          handed to the large-team launch part-way
                                          they did not finish on the GPU, for a reason
                                          not found.  Large-event teams always run
                                          persistent.                                 */
    int32_t teams_per_cu;              /* 0..64, not used by modes 2 and 4 (it sized the
                                          persistent grids of modes 1 and 3)           */
} pv_schedule;

/* Fill *p with the defaults described above. */
void pv_params_default(pv_params *p);

/* Number of histogram bins for *p, or -1 if (z_max - z_min) / dz is not a
 * whole number between 1 and 4096. */
int32_t pv_nbins(const pv_params *p);

/* The whole path over a batch of events (Sec. 3.1-3.5).
 *  tracks        : device SoA arrays of offsets[n_events] tracks (float32).
 *                  Every pointer must be non-null, also for a batch without
 *                  tracks (the host cannot see offsets[n_events]); a null one
 *                  returns PV_EINVAL.  The same holds for every output array.
 *  event_offsets : device int32[n_events + 1]; event e owns tracks
 *                  [offsets[e], offsets[e+1]); offsets[n_events] is the number
 *                  of tracks in the arrays.  Events whose offsets are negative,
 *                  decreasing or beyond offsets[n_events] are flagged
 *                  PV_EV_OFFSETS_INVALID.
 *  n_events      : >= 0; 0 enqueues nothing.
 *  beamline, params : host structs.
 *  out_vertices  : device outputs, see pv_vertices_out.
 *  out_track_weights : device outputs, one entry per track.
 *  stream        : hipStream_t.
 * The schedule is the library's current default (see pv_set_schedule). */
int pv_find(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
            const pv_beamline *beamline, const pv_params *params,
            pv_vertices_out *out_vertices, pv_track_out *out_track_weights, void *stream);

/* pv_find for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, work and outputs as pv_find (default schedule), but the
 * workspace is a fixed device array inside the library (one per device,
 * about 2 MiB, held until the process ends) instead of memory the library
 * allocates: no hipMalloc, hipFree or other allocating call is made.
 *  n_events      : 0 .. PV_NOALLOC_MAX_EVENTS; more returns PV_EINVAL.
 * All calls on one device share that array: calls that may overlap on one
 * device (different streams, or different threads without ordering) race
 * and give undefined results; calls on one stream are ordered by it.  Each
 * call first zeroes the array's counters with a small kernel on `stream`
 * (no memset), so a call may be captured into a graph.  The first call on a
 * device looks the array's address up (hipGetSymbolAddress).  Calls made
 * while pv_timing_start() is active are not timed. */
#define PV_NOALLOC_MAX_EVENTS 262144
int pv_find_noalloc(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                    const pv_beamline *beamline, const pv_params *params,
                    pv_vertices_out *out_vertices, pv_track_out *out_track_weights, void *stream);

/* pv_find with an explicit schedule (NULL = default).  Integer outputs (vertex
 * counts, track-to-vertex indices, histograms, clusters) do not depend on
 * the schedule; floating-point outputs are reproducible bit for bit for a
 * fixed schedule and agree across schedules to rounding. */
int pv_find_sched(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                  const pv_beamline *beamline, const pv_params *params,
                  pv_vertices_out *out_vertices, pv_track_out *out_track_weights,
                  const pv_schedule *schedule, void *stream);

/* pv_find that also writes the intermediate results named in *debug
 * (device pointers, NULL members skipped).  Same outputs as pv_find. */
int pv_find_debug(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                  const pv_beamline *beamline, const pv_params *params,
                  pv_vertices_out *out_vertices, pv_track_out *out_track_weights,
                  const pv_debug_out *debug, const pv_schedule *schedule, void *stream);

/* Autotuner for the batched form: runs pv_find on the caller's batch with
 * every schedule (waves_per_team x track_capacity x persistent), times
 * `reps` launches of each with HIP events on `stream`, and makes the fastest
 * the process-wide default.  Arguments as for pv_find; the outputs are
 * overwritten (they end up holding the result of the winning schedule, which
 * equals every other schedule's in its integer outputs).
 *  reps       : timed launches per schedule, >= 1.
 *  cache_path : text file keeping one line per (device, key, batch shape);
 *               NULL for none.  The shape is read from the batch: its event
 *               count and the median, 90th and 99th percentile and maximum
 *               of its track counts, each in quarter-octave buckets, and the
 *               association and splitting variants.  With an entry for
 *               (device, key, shape) and force == 0 nothing is timed: the
 *               cached schedule becomes the default.
 *  key        : caller's name for the workload (no tabs/newlines); may be
 *               NULL, the shape alone then keys the cache.
 *  best       : receives the chosen schedule; may be NULL.
 *  best_us    : receives its time per launch in microseconds (0 when read
 *               from the cache); may be NULL.
 * Synchronises `stream`. */
int pv_autotune(const pv_tracks *tracks, const int32_t *event_offsets, int32_t n_events,
                const pv_beamline *beamline, const pv_params *params,
                pv_vertices_out *out_vertices, pv_track_out *out_track_weights, int32_t reps,
                const char *cache_path, const char *key, int32_t force, pv_schedule *best,
                double *best_us, void *stream);

/* Output compaction for transfers.  pv_find writes each event's vertices
 * into max_vertices slots; most stay unused (about 5 vertices per event at
 * mu = 5 against 128 slots).  This gathers the written records of a batch
 * into one dense array so that only they need to cross PCIe:
 *  slots, n_vertices : device outputs of pv_find for n_events events with
 *                      max_vertices (1..128) slots each (counts are clamped
 *                      to [0, max_vertices]).
 *  dense             : device, room for first[n_events] records (at most
 *                      n_events * max_vertices); event e's records land at
 *                      dense[first[e] .. first[e + 1]).
 *  first             : device int32[n_events + 1], written: exclusive prefix of
 *                      the counts, first[n_events] = total.
 * Two launches on `stream` (a one-workgroup scan, then the copy); no
 * allocation.  The caller reads first[n_events] back to size its copy. */
int pv_compact_vertices(const pv_vertex *slots, const int32_t *n_vertices, int32_t n_events,
                        int32_t max_vertices, pv_vertex *dense, int32_t *first, void *stream);

/* Replace / read the default schedule used by pv_find (process-wide). */
int pv_set_schedule(const pv_schedule *schedule);
int pv_get_schedule(pv_schedule *schedule);

/* Benchmark support: time the library's own kernels with HIP events
 * recorded on the caller's stream around each launch.
 * pv_timing_start() drops earlier records and makes every later pv_find*
 * call record events; pv_timing_stop() stops recording, waits for the
 * recorded events and returns the total milliseconds spent in the main fused
 * kernel and in the large-event kernel, and the number of calls timed (any
 * output pointer may be NULL). */
int pv_timing_start(void);
int pv_timing_stop(double *main_ms, double *large_ms, int64_t *n_calls);

/* Benchmark support: the LDS read bandwidth of the current device, the peak
 * the kernels' LDS traffic is compared with.  Two workgroups per compute unit
 * (64 KiB of LDS each) read 16 bytes per lane per step, without bank
 * conflicts, 4096 steps; the best of three timed launches (HIP events on
 * `stream`, after one warm-up) gives *bytes_per_s; *workgroups (may be NULL)
 * receives the grid size.  Allocates and frees a small device buffer;
 * synchronises `stream`. */
int pv_measure_lds_peak(double *bytes_per_s, int32_t *workgroups, void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of events that arrive one at a time.
 *
 * The paper processes batches of events on several streams so that
 * transfers overlap compute (Sec. 6).  A server owns a fixed pool of batch
 * slots, each with pinned host staging, device buffers and (optionally) an
 * instantiated hipGraph of the pv_find launches; the graphs read the batch
 * size from device memory, so one graph serves every batch of its slot.
 * pv_server_submit copies an event into the slot that is open for
 * admission; a worker thread seals the open batch when it is full, or when
 * a stream is free and either the device is idle or the oldest event has
 * waited max_wait_us; it copies the batch in, launches, copies the results
 * out and scatters them into the caller's host buffers.
 * Events that arrive while others are on the GPU join the next batch.
 * Admission is bounded by the slot pool (sized against the device-memory
 * budget): when every slot is busy, submit returns PV_EBUSY.
 * A server with max_events_per_batch = 1 is the plain one-launch-per-event
 * form on the same machinery.  Every event's result does not depend on the
 * batch it was processed in.
 * ------------------------------------------------------------------------ */
typedef struct pv_server pv_server;

typedef struct {
    int32_t max_events_per_batch;   /* events per batch slot, >= 1                   */
    int32_t max_tracks_per_batch;   /* tracks per batch slot; also the largest event  */
    int32_t n_slots;                /* batch slots (staging + device buffers), >= 2   */
    int32_t n_streams;              /* HIP streams, >= 1; batches in flight <= this   */
    int64_t device_budget_bytes;    /* the slots' device memory must fit in this      */
    int32_t max_wait_us;            /* with a stream free while other batches run,
                                       seal the open batch once its oldest event has
                                       waited this long (at once when the device is
                                       idle); while every stream is busy it grows     */
    int32_t use_graphs;             /* 1: launch batches as hipGraphs; 0: launches    */
} pv_server_config;

typedef struct {
    const float *x, *y, *z, *tx, *ty, *cov_xx, *cov_xtx, *cov_txtx;   /* HOST, n_tracks each;
                                       read before pv_server_submit returns            */
    int32_t n_tracks;
    pv_vertex *vertices;            /* HOST, max_vertices_per_event records           */
    int32_t *track_vertex;          /* HOST, n_tracks                                 */
    float *track_weight;            /* HOST, n_tracks                                 */
} pv_request;                       /* output buffers stay the caller's; they are
                                       written before the event is reported complete  */

typedef struct {
    uint64_t tag;
    int32_t status;                 /* PV_EV_* bits                                   */
    int32_t n_vertices;
    int64_t t_arrival_ns;           /* steady clock, see pv_clock_ns                  */
    int64_t t_done_ns;              /* when the results were in the caller's buffers  */
} pv_completion;

typedef struct {
    int64_t submitted, completed, rejected_busy, batches;
    double mean_batch_events;
    int64_t device_bytes;           /* device memory held by the slots               */
} pv_server_stats;

/* Steady-clock nanoseconds used for arrival and completion stamps. */
int64_t pv_clock_ns(void);

void pv_server_config_default(pv_server_config *c);

/* Create a server on the current device.  schedule may be NULL (default).
 * Returns PV_EINVAL for bad arguments or when the slots do not fit in the
 * budget, PV_ENOMEM / PV_EHIP on allocation or capture failures. */
int pv_server_create(pv_server **out, const pv_params *params, const pv_beamline *beamline,
                     const pv_server_config *config, const pv_schedule *schedule);

/* Admit one event.  t_arrival_ns = 0 stamps the current time.
 * PV_EBUSY: no batch slot can take it now (retry later); PV_EINVAL: the
 * event has more tracks than a slot holds or a null pointer. */
int pv_server_submit(pv_server *s, const pv_request *req, uint64_t tag, int64_t t_arrival_ns);

/* Move up to max_out completions into out, waiting up to timeout_us for the
 * first one.  Returns the number moved (>= 0) or a negative PV_E* code. */
int pv_server_poll(pv_server *s, pv_completion *out, int32_t max_out, int32_t timeout_us);

/* Wait until every admitted event is complete (timeout_ms < 0: no limit).
 * Returns PV_OK, or PV_EBUSY on timeout. */
int pv_server_drain(pv_server *s, int32_t timeout_ms);

/* Submit reqs[k] at arrival time t0 + t_offset_ns[k] (t0 = call time),
 * retrying while the server is busy, and collect every completion:
 * out[k] is the completion of reqs[k] (tag = k).  Returns when all n are
 * complete. */
int pv_server_replay(pv_server *s, const pv_request *reqs, const int64_t *t_offset_ns, int32_t n,
                     pv_completion *out);

int pv_server_get_stats(pv_server *s, pv_server_stats *stats);
int pv_server_destroy(pv_server *s);

/* Thread-local description of the last non-zero return of this thread. */
const char *pv_last_error(void);

/* Library version string. */
const char *pv_version(void);

#ifdef __cplusplus
}
#endif
#endif
