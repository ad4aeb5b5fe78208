/*
 * pv_oracle.h -- plain CPU reference of the primary-vertex finding path of
 * "A parallel algorithm for fast reconstruction of primary vertices on
 * heterogeneous architectures" (LHCb, arXiv:2412.14966).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the HIP path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * Precision.  The projection (Eq. 1, Eq. 3) and the histogram kernel
 * (Sec. 3.2) are defined here in binary32 arithmetic: every operation is
 * evaluated in binary64 and rounded once to binary32, which equals plain
 * binary32 arithmetic for +, -, *, /, sqrt (double rounding is innocuous when
 * the wide format has at least 2p+2 bits; S. Figueroa, ACM SIGNUM Newsletter
 * 30(3), 1995).  This is what makes an integer histogram reproducible across
 * implementations.  Everything after the integer histogram (seeds, fit,
 * selection) is binary64.
 *
 * Parity pins: every function below is checked by the CPU test suite against
 * closed forms, invariants, brute force or library routines (see the header
 * comment of each function for the passage it follows).
 */
#ifndef PV_ORACLE_H
#define PV_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Per-event status bits. */
#define ORC_EV_NONFINITE_INPUT  1
#define ORC_EV_TOO_MANY_TRACKS  2
#define ORC_EV_VERTEX_OVERFLOW  4
#define ORC_EV_OFFSETS_INVALID  8
#define ORC_EV_FIT_FAILED      16   /* a candidate's fit failed (no weight left, or a
                                       singular normal matrix) and it was dropped */

/* Per-vertex flag bits. */
#define ORC_VX_NOT_CONVERGED    1

/* Per-track projection flags. */
#define ORC_TR_HIST       1   /* enters the histogram                     */
#define ORC_TR_ASSOC      2   /* may be associated to a vertex            */
#define ORC_TR_NONFINITE  4   /* some input field is NaN or infinite      */

typedef struct {
    /* histogram stage (binary32 values) */
    float z_min, z_max, dz, z_gas;
    float sigma_max_pp, sigma_max_gas;   /* Sec. 3.2 and Table 2: 1.5 / 10 mm   */
    float u0;                            /* half-width of the cubic kernel / sigma */
    int   frac_bits;                     /* fixed-point unit 2^frac_bits per track */
    /* peak search, in fixed-point units */
    int   proto_thr, dip_prom, min_int_pp, min_int_gas;
    /* association (Sec. 3.4) and final selection (Table 2) */
    int   part_min_pp, part_min_gas, pv_min_pp, pv_min_gas;
    /* fit (Sec. 3.5) */
    int   max_iter;
    double chi2_max, conv_dchi2, conv_dz, max_rho_pp;
    double sing_ratio;         /* normal matrix singular below this det / prod(diag) */
    /* capacities */
    int   max_tracks, max_vertices;
    /* GPU variant of the association and fit (Sec. 3.5, Eq. 18, Sec. 5) */
    int    assoc_mode;        /* 0: partition association, Tukey fit (Sec. 3.4-3.5);
                                 1: every track weighted to every candidate (Eq. 18) */
    double chi2_max_mv;       /* chi2 at which an uncontested weight is 1/2 (Eq. 18) */
    double chi2_window_mv;    /* tracks enter a candidate's fit below this chi2 at its seed */
    double conv_dz_mv;        /* GPU convergence: |dz| below this, no dchi2 requirement */
    double dup_ratio;         /* duplicates: dz^2 / (Czz_1 + Czz_2) below this */
    double w_count_mv;        /* a track counts for a vertex with final weight >= this */
    /* splitting of proto-clusters (Sec. 3.3) */
    int    peak_mode;         /* 0: minima in z order (GPU variant); 1: the smallest minimum
                                 between the two largest maxima, recursively (x86 variant) */
    /* reporting only (no effect on the results): a threshold decision whose
       deciding quantity lies within tie_rel (relative) of its threshold is
       counted as one that an evaluation in another precision may take the
       other way */
    double tie_rel;
    /* test hook: the fit of the cluster whose highest bin is
       iter_override_bin runs exactly iter_override_n iterations (stopping
       early only if it fails); -1 / 0 leave every fit alone */
    int    iter_override_bin, iter_override_n;
} orc_params;

#define ORC_PEAK_Z_ORDERED 0
#define ORC_PEAK_RECURSIVE 1

#define ORC_ASSOC_PARTITION   0
#define ORC_ASSOC_MULTIVERTEX 1

typedef struct {
    int lo, hi, peak;          /* seed cluster bin range and its first highest bin */
    double z_seed;             /* Eq. 4-5 */
    int kept;                  /* survives the association step            */
    int n_assoc;               /* tracks owned after the association step  */
    int own_lo, own_hi;        /* bins owned after the association step    */
    int n_near_cut;            /* multi-vertex: associable tracks whose chi2 at
                                  the seed lies within tie_rel of the pre-cut */
} orc_cluster;

typedef struct {
    double x, y, z;
    double cov[6];             /* xx, xy, yy, xz, yz, zz (Eq. 14) */
    double chi2, ndof, z_seed;
    double conv_margin;        /* smallest relative distance of a convergence
                                  decision quantity from its threshold      */
    double dchi2;              /* predicted chi2 change of the last step (Eq. 16) */
    int n_tracks, bin_lo, bin_hi, peak_bin, n_iter, flags;
    /* multi-vertex decisions a binary32 evaluation may take the other way:
       tracks whose final weight is within 1e-4 of w_count_mv, and the
       smallest |dz^2 / (R (Czz_1 + Czz_2)) - 1| of a duplicate test this
       vertex took part in (INFINITY if none) */
    int n_near;
    double dup_margin;
} orc_vertex;

void orc_params_default(orc_params *p);
/* number of histogram bins, or -1 if the range is not a whole number of bins */
int  orc_nbins(const orc_params *p);
/* first pp bin: bins below it belong to the beam-gas region */
int  orc_gas_bin(const orc_params *p);

/* Eq. 1 and Eq. 3 for one track; trk = x, y, z, tx, ty, Vxx, Vxtx, Vtxtx;
   beam = xb, yb, txb, tyb.  Returns the ORC_TR_* flags. */
int  orc_project(const float trk[8], const float beam[4], const orc_params *p,
                 float *zpoca, float *sigma, int *bin);

/* fixed-point cumulative kernel mass left of edge e for a track at zp with
   half-width sw (Sec. 3.2, cubic approximation of the Gaussian CDF);
   s = (e - zp) * fl(1 / sw) in binary32 */
int  orc_edge_code(float e, float zp, float sw, int frac_bits);

/* histogram and per-bin associable-track counts of one event */
void orc_hist_event(const float *const trk[8], int n, const float beam[4],
                    const orc_params *p, int *h, int *c);

/* proto-clusters, dip splitting and seeds (Sec. 3.3); returns the number of
   clusters written (at most max_out); *overflow is set if more existed */
int  orc_peak_search(const int *h, const orc_params *p, orc_cluster *out,
                     int max_out, int *overflow);

/* seed position of a cluster whose highest bin is i (Eq. 4-5) */
double orc_seed_z(const int *h, int nb, int i, const orc_params *p);

/* explicit track association with iterative removal (Sec. 3.4); fills
   kept / n_assoc / own_lo / own_hi; returns the number kept */
int  orc_partition(orc_cluster *cl, int n_cl, const int *c, const orc_params *p);

/* adaptive vertex fit (Sec. 3.5) of the tracks idx[0..n-1] from the seed;
   w_out[k] receives the final weight of track idx[k].  Returns 0 on
   success, 1 if the fit failed (no weight left or singular matrix). */
int  orc_fit(const float *const trk[8], const int *idx, int n,
             double x_seed, double y_seed, double z_seed, const orc_params *p,
             orc_vertex *v, double *w_out);

/* Eq. 18: weight of a track with chi2 relative to this candidate, when its
   terms exp(-chi2_k / 2) for the other candidates sum to `others` */
double orc_mv_weight(double chi2, double others, double chi2_max);

/* the fit of orc_fit with the weights of Eq. 18: others[k] is the sum of
   exp(-chi2 / 2) of track idx[k] relative to the other candidates at their
   seeds; converged when |dz| < conv_dz_mv (the GPU criterion of Sec. 3.5) */
int  orc_fit_mv(const float *const trk[8], const int *idx, const double *others, int n,
                double x_seed, double y_seed, double z_seed, const orc_params *p,
                orc_vertex *v, double *w_out);

/* Whole path over a batch.  trk: 8 arrays of offsets[n_events] tracks.
   vtx: n_events * max_vertices records; trk_vtx / trk_w per input track.
   Optional (NULL to skip): hist (n_events * nbins), clusters
   (n_events * max_vertices) with n_clusters (n_events), and per-track
   zpoca / sigma / bin.  n_threads <= 0 uses every available thread.
   Returns 0, or -1 on bad arguments. */
int  orc_find(const float *const trk[8], const int *offsets, int n_events,
              const float beam[4], const orc_params *p,
              int *n_vtx, int *status, orc_vertex *vtx, int *trk_vtx, double *trk_w,
              int *hist, orc_cluster *clusters, int *n_clusters,
              float *trk_zpoca, float *trk_sigma, int *trk_bin, int n_threads);

/* threads orc_find would use for n_threads <= 0 */
int  orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
