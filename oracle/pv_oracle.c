/*
 * pv_oracle.c -- plain, sequential CPU reference of the primary-vertex
 * finding path of arXiv:2412.14966 (LHCb).  TEST INFRASTRUCTURE ONLY: used by
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark;
 * never by the product path.
 *
 * The five steps of Sec. 3 are written out in the paper's order and notation:
 *   Sec. 3.1  projection to the point of closest approach (Eq. 1, Eq. 3)
 *   Sec. 3.2  histogram of z_poca with a finite-support kernel whose
 *             cumulative is a cubic approximation of the Gaussian CDF
 *   Sec. 3.3  proto-clusters, dip search, z-ordered splitting, seeds (Eq. 4-5)
 *   Sec. 3.4  explicit association through partition points, iterative
 *             removal of clusters with too few tracks
 *   Sec. 3.5  Newton-Raphson vertex fit with Tukey weights (Eq. 6-17),
 *             followed by the final selection (end of Sec. 3.5, Table 2)
 * Readings of points the paper leaves open are stated where they are used.
 *
 * Nothing here is blocked, fused or reordered for speed: one event at a time,
 * one track at a time, general 3x3 matrix algebra for the fit.
 */
#include "pv_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* binary32 operations: evaluate in binary64, round once to binary32        */
/* ------------------------------------------------------------------------ */
static float add32(float a, float b) { return (float)((double)a + (double)b); }
static float sub32(float a, float b) { return (float)((double)a - (double)b); }
static float mul32(float a, float b) { return (float)((double)a * (double)b); }
static float div32(float a, float b) { return (float)((double)a / (double)b); }
static float sqrt32(float a) { return (float)sqrt((double)a); }

void orc_params_default(orc_params *p)
{
    memset(p, 0, sizeof(*p));
    /* histogram range of the benchmark workloads; the paper's own range is
       [-550, 300] mm with the same 0.25 mm bins (Sec. 3.2) */
    p->z_min = -600.0f;
    p->z_max = 400.0f;
    p->dz = 0.25f;
    p->z_gas = -300.0f;              /* Table 2: p-gas region below -300 mm */
    p->sigma_max_pp = 1.5f;          /* Sec. 3.2, Table 2 */
    p->sigma_max_gas = 10.0f;
    p->u0 = 2.13f;                   /* kernel half-width in units of sigma */
    p->frac_bits = 16;
    p->proto_thr = 6554;             /* 0.1 track per bin */
    p->dip_prom = 131072;            /* 2 tracks per bin */
    p->min_int_pp = 163840;          /* Table 2: 2.5 tracks */
    p->min_int_gas = 114688;         /* Table 2: 1.75 tracks */
    p->part_min_pp = 3;              /* Sec. 3.4 */
    p->part_min_gas = 2;
    p->pv_min_pp = 4;                /* Table 2 */
    p->pv_min_gas = 3;
    p->max_iter = 10;                /* Sec. 3.5 */
    p->chi2_max = 12.0;              /* Eq. 17 */
    p->conv_dchi2 = 0.01;            /* Sec. 3.5, x86 criterion */
    p->conv_dz = 0.001;              /* 1 micrometre */
    p->max_rho_pp = 0.3;             /* end of Sec. 3.5 */
    p->sing_ratio = 1e-4;
    p->max_tracks = 4096;
    p->max_vertices = 128;
    /* GPU variant (Sec. 3.5, Eq. 18).  The paper gives no default for the
       cut-off of Eq. 18; 4 is the value of its illustration, with which an
       uncontested weight is close to the Tukey weight at 12, as the text
       says it should be.  The chi2 pre-cut (Sec. 5) has no value either: 25
       leaves out tracks whose uncontested weight at the seed is below 3e-5.
       The duplicate test reads "difference over the sum of the variances
       below 25" as dz^2 / (Czz_1 + Czz_2) < 25, i.e. closer than five
       combined standard deviations. */
    p->assoc_mode = ORC_ASSOC_PARTITION;
    p->chi2_max_mv = 4.0;
    p->chi2_window_mv = 25.0;
    p->conv_dz_mv = 0.0005;          /* Sec. 3.5, GPU criterion: 0.5 micrometre */
    p->dup_ratio = 25.0;
    p->w_count_mv = 0.5;
    p->peak_mode = ORC_PEAK_Z_ORDERED;
    p->tie_rel = 1e-5;
    p->iter_override_bin = -1;
    p->iter_override_n = 0;
}

int orc_nbins(const orc_params *p)
{
    double span = ((double)p->z_max - (double)p->z_min) / (double)p->dz;
    long nb = lround(span);
    if (!(p->dz > 0.0f) || nb < 1 || fabs(span - (double)nb) > 1e-6 * (double)nb)
        return -1;
    return (int)nb;
}

int orc_gas_bin(const orc_params *p)
{
    return (int)floor(((double)p->z_gas - (double)p->z_min) / (double)p->dz);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: projection to the point of closest approach                    */
/* ------------------------------------------------------------------------ */
/*
 * Eq. 1: z_poca = z_trk + [(tx - txb)(xb - x) + (ty - tyb)(yb - y)]
 *                         / [(tx - txb)^2 + (ty - tyb)^2]
 * Eq. 3: sigma_poca = sqrt(Vxx / [(tx - txb)^2 + (ty - tyb)^2])
 * Eq. 1 is used as printed, with the beamline's transverse position at z = 0.
 * The central bin is floor((z_poca - z_min) / dz).  A track enters the
 * histogram if its inputs are finite, Vxx > 0, the slope difference is
 * nonzero, z_poca lies in [z_min, z_max) and sigma_poca is at most the
 * region's maximum (Sec. 3.2); the region is that of the central bin.  It may
 * be associated to a vertex under the same conditions without the sigma cut
 * (the paper applies that cut to histogram filling only).
 */
int orc_project(const float trk[8], const float beam[4], const orc_params *p,
                float *zpoca, float *sigma, int *bin)
{
    const float x = trk[0], y = trk[1], z = trk[2], tx = trk[3], ty = trk[4], vxx = trk[5];
    const float xb = beam[0], yb = beam[1], txb = beam[2], tyb = beam[3];
    int k, flags = 0;
    *zpoca = 0.0f;
    *sigma = 0.0f;
    *bin = -1;
    for (k = 0; k < 8; ++k)
        if (!isfinite(trk[k]))
            return ORC_TR_NONFINITE;

    const float dtx = sub32(tx, txb);
    const float dty = sub32(ty, tyb);
    const float dx = sub32(xb, x);
    const float dy = sub32(yb, y);
    const float num = add32(mul32(dtx, dx), mul32(dty, dy));
    const float den = add32(mul32(dtx, dtx), mul32(dty, dty));
    if (!(den > 0.0f) || !(vxx > 0.0f))
        return 0;
    const float zp = add32(z, div32(num, den));
    const float s2 = div32(vxx, den);
    const float sg = sqrt32(s2);
    *zpoca = zp;
    *sigma = sg;
    if (!(zp >= p->z_min && zp < p->z_max))
        return 0;
    const int nb = orc_nbins(p);
    int b = (int)floorf(div32(sub32(zp, p->z_min), p->dz));
    if (b > nb - 1)
        b = nb - 1;
    if (b < 0)
        b = 0;
    *bin = b;
    flags |= ORC_TR_ASSOC;
    const float smax = (b < orc_gas_bin(p)) ? p->sigma_max_gas : p->sigma_max_pp;
    const float sw = mul32(p->u0, sg);
    if (s2 <= mul32(smax, smax) && sw > 0.0f)
        flags |= ORC_TR_HIST;
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2: histogram filling                                              */
/* ------------------------------------------------------------------------ */
/*
 * The paper fills each track as the integral of a Gaussian N(z_poca, sigma)
 * over every bin near the central one, with a cubic polynomial standing in
 * for the Gaussian cumulative on the GPU.  Reading: the cubic is
 *   P(s) = 1/2 + s (3/4 - s^2 / 4),  s = clamp((e - z_poca) / (u0 sigma), -1, 1),
 * the cumulative of a parabolic kernel of half-width u0 sigma (u0 = 2.13
 * minimises the largest deviation from the Gaussian cumulative).  Bin j gets
 * P(e_{j+1}) - P(e_j), in integer units of 2^-frac_bits track, so every
 * histogrammed track adds exactly 2^frac_bits; the first edge of the
 * histogram counts as P = 0 and the last as P = 1, so mass beyond the range
 * lands in the end bins.  In binary32 the division by u0 sigma is a product
 * with its rounded reciprocal, taken once per track: s = (e - z_poca) r with
 * r = 1 / (u0 sigma).
 */
int orc_edge_code(float e, float zp, float sw, int frac_bits)
{
    const float r = div32(1.0f, sw);
    float s = mul32(sub32(e, zp), r);
    if (s < -1.0f)
        s = -1.0f;
    if (s > 1.0f)
        s = 1.0f;
    const float P = add32(0.5f, mul32(s, sub32(0.75f, mul32(0.25f, mul32(s, s)))));
    /* P * 2^frac_bits is exact; round half to even */
    return (int)nearbyint((double)P * ldexp(1.0, frac_bits));
}

static float edge_z(const orc_params *p, int j)
{
    return add32(p->z_min, mul32((float)j, p->dz));
}

void orc_hist_event(const float *const trk[8], int n, const float beam[4],
                    const orc_params *p, int *h, int *c)
{
    const int nb = orc_nbins(p);
    const int full = 1 << p->frac_bits;
    int i, j, k;
    memset(h, 0, sizeof(int) * (size_t)nb);
    memset(c, 0, sizeof(int) * (size_t)nb);
    for (i = 0; i < n; ++i) {
        float t[8], zp, sg;
        int b;
        for (k = 0; k < 8; ++k)
            t[k] = trk[k][i];
        const int fl = orc_project(t, beam, p, &zp, &sg, &b);
        if (fl & ORC_TR_ASSOC)
            c[b] += 1;
        if (!(fl & ORC_TR_HIST))
            continue;
        const float sw = mul32(p->u0, sg);
        /* edges with nonzero, non-full code lie strictly inside (zp - sw, zp + sw);
           widen by one edge each side so the end codes are 0 and 'full' */
        int jl = (int)floor(((double)zp - (double)sw - (double)p->z_min) / (double)p->dz) - 1;
        int jh = (int)ceil(((double)zp + (double)sw - (double)p->z_min) / (double)p->dz) + 1;
        if (jl < 0)
            jl = 0;
        if (jh > nb)
            jh = nb;
        int prev = (jl == 0) ? 0 : orc_edge_code(edge_z(p, jl), zp, sw, p->frac_bits);
        for (j = jl; j < jh; ++j) {
            const int next = (j + 1 == nb) ? full : orc_edge_code(edge_z(p, j + 1), zp, sw, p->frac_bits);
            h[j] += next - prev;
            prev = next;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.3: peak search                                                    */
/* ------------------------------------------------------------------------ */
static int first_argmax(const int *h, int a, int b)
{
    int i = a, j;
    for (j = a + 1; j <= b; ++j)
        if (h[j] > h[i])
            i = j;
    return i;
}

static int64_t range_sum(const int *h, int a, int b)
{
    int64_t s = 0;
    int j;
    for (j = a; j <= b; ++j)
        s += h[j];
    return s;
}

/* cluster-integral threshold for the region of the candidate's highest bin
   (Table 2: 2.5 tracks pp, 1.75 tracks p-gas) */
static int64_t integral_threshold(const int *h, int a, int b, const orc_params *p)
{
    return (first_argmax(h, a, b) < orc_gas_bin(p)) ? p->min_int_gas : p->min_int_pp;
}

/* Eq. 4-5: z_seed = z_i + delta dz with
   delta = 1/2 (N_{i+1} - N_{i-1}) / (2 N_i - N_{i+1} - N_{i-1}), in [-1/2, 1/2] */
double orc_seed_z(const int *h, int nb, int i, const orc_params *p)
{
    const double Ni = h[i];
    const double Nm = (i > 0) ? h[i - 1] : 0.0;
    const double Np = (i + 1 < nb) ? h[i + 1] : 0.0;
    const double den = 2.0 * Ni - Np - Nm;
    double delta = (den > 0.0) ? 0.5 * (Np - Nm) / den : 0.0;
    if (delta > 0.5)
        delta = 0.5;
    if (delta < -0.5)
        delta = -0.5;
    const double zi = (double)p->z_min + ((double)i + 0.5) * (double)p->dz;
    return zi + delta * (double)p->dz;
}

/*
 * Proto-clusters are maximal runs of bins with content above proto_thr.
 * Inside each, a walk with hysteresis dip_prom records the significant
 * minima: a minimum is recorded once the content has fallen by at least
 * dip_prom below the preceding maximum and risen again by at least dip_prom
 * above it (so each recorded minimum has a maximum on either side); of a flat
 * minimum the lowest-z bin is kept.  The minima are then taken in z order
 * (the paper's GPU variant): the proto-cluster is cut after minimum m if the
 * part left of the cut (from the previous cut) and everything right of it up
 * to the proto-cluster's end both reach the cluster-integral threshold of
 * their region.  The remainder is a cluster if it reaches the threshold.
 */
/* significant minima of bins [s, e] in z order (reading: a minimum counts
   after a fall of at least D below the preceding maximum and a rise of at
   least D above it; of a flat minimum the lowest-z bin is kept) */
static int dip_minima(const int *h, int s, int e, int D, int *minima)
{
    int n_min = 0, up = 1, M = h[s], m = 0, mj = -1, k;
    for (k = s + 1; k <= e; ++k) {
        if (up) {
            if (h[k] > M) {
                M = h[k];
            } else if (h[k] <= M - D) {
                up = 0;
                m = h[k];
                mj = k;
            }
        } else {
            if (h[k] < m) {
                m = h[k];
                mj = k;
            } else if (h[k] >= m + D) {
                minima[n_min++] = mj;
                up = 1;
                M = h[k];
            }
        }
    }
    return n_min;
}

static void emit_cluster(const int *h, int lo, int hi, const orc_params *p, int nb, orc_cluster *out, int max_out,
                         int *n_out, int *overflow)
{
    if (*n_out < max_out) {
        orc_cluster *cl = &out[*n_out];
        memset(cl, 0, sizeof(*cl));
        cl->lo = lo;
        cl->hi = hi;
        cl->peak = first_argmax(h, lo, hi);
        cl->z_seed = orc_seed_z(h, nb, cl->peak, p);
        cl->kept = 1;
        ++*n_out;
    } else {
        *overflow = 1;
    }
}

/*
 * x86 variant of the splitting (Sec. 3.3): the range [s, e] is cut at the
 * smallest significant minimum between its two largest maxima, and each part
 * is treated the same way, recursively (its significant extrema found anew
 * within the part).  Readings: the maxima are the highest bins of the
 * segments between consecutive significant minima; of equal maxima the lower
 * z counts as larger, of equal minima the lower z is taken; the cut bin stays
 * with the left part; a cut is made only when both parts reach the integral
 * threshold of their region (Table 2), otherwise the range is one cluster if
 * it reaches its own.  Clusters come out in z order.
 */
static void split_recursive(const int *h, int s, int e, const orc_params *p, int nb, orc_cluster *out,
                            int max_out, int *n_out, int *overflow)
{
    int *minima = (int *)malloc(sizeof(int) * (size_t)(e - s + 1));
    const int n_min = dip_minima(h, s, e, p->dip_prom, minima);
    int cut = -1;
    if (n_min > 0) {
        /* the two largest segment maxima */
        int b1 = -1, b2 = -1, q;
        for (q = 0; q <= n_min; ++q) {
            const int a = (q == 0) ? s : minima[q - 1] + 1;
            const int b = (q == n_min) ? e : minima[q] - 1;
            const int i = first_argmax(h, a, b);
            if (b1 < 0 || h[i] > h[b1]) {
                b2 = b1;
                b1 = i;
            } else if (b2 < 0 || h[i] > h[b2]) {
                b2 = i;
            }
        }
        const int p1 = b1 < b2 ? b1 : b2, p2 = b1 < b2 ? b2 : b1;
        for (q = 0; q < n_min; ++q)
            if (minima[q] > p1 && minima[q] < p2 && (cut < 0 || h[minima[q]] < h[cut]))
                cut = minima[q];
        if (cut >= 0 && !(range_sum(h, s, cut) >= integral_threshold(h, s, cut, p) &&
                          range_sum(h, cut + 1, e) >= integral_threshold(h, cut + 1, e, p)))
            cut = -1;
    }
    free(minima);
    if (cut >= 0) {
        split_recursive(h, s, cut, p, nb, out, max_out, n_out, overflow);
        split_recursive(h, cut + 1, e, p, nb, out, max_out, n_out, overflow);
    } else if (range_sum(h, s, e) >= integral_threshold(h, s, e, p)) {
        emit_cluster(h, s, e, p, nb, out, max_out, n_out, overflow);
    }
}

int orc_peak_search(const int *h, const orc_params *p, orc_cluster *out,
                    int max_out, int *overflow)
{
    const int nb = orc_nbins(p);
    const int T = p->proto_thr, D = p->dip_prom;
    int n_out = 0, j = 0;
    int *minima = (int *)malloc(sizeof(int) * (size_t)nb);
    *overflow = 0;
    while (j < nb) {
        if (h[j] <= T) {
            ++j;
            continue;
        }
        const int s = j;
        while (j + 1 < nb && h[j + 1] > T)
            ++j;
        const int e = j;
        ++j;

        if (p->peak_mode == ORC_PEAK_RECURSIVE) {
            split_recursive(h, s, e, p, nb, out, max_out, &n_out, overflow);
            continue;
        }
        const int n_min = dip_minima(h, s, e, D, minima);

        /* z-ordered splitting (GPU variant) */
        int cs = s, q, lo = 0, hi = 0;
        for (q = 0; q <= n_min; ++q) {
            int emit = 0;
            if (q < n_min) {
                const int cut = minima[q];
                if (range_sum(h, cs, cut) >= integral_threshold(h, cs, cut, p) &&
                    range_sum(h, cut + 1, e) >= integral_threshold(h, cut + 1, e, p)) {
                    lo = cs;
                    hi = cut;
                    emit = 1;
                    cs = cut + 1;
                }
            } else if (range_sum(h, cs, e) >= integral_threshold(h, cs, e, p)) {
                lo = cs;
                hi = e;
                emit = 1;
            }
            if (emit)
                emit_cluster(h, lo, hi, p, nb, out, max_out, &n_out, overflow);
        }
    }
    free(minima);
    return n_out;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.4: explicit track association                                     */
/* ------------------------------------------------------------------------ */
/*
 * The partition point between consecutive clusters is the bin halfway
 * between the first one's upper bound and the next one's lower bound
 * (rounded down); a cluster owns the bins above the previous partition point
 * up to and including its own, the first from bin 0 and the last to the end.
 * Its track count is the number of associable tracks whose central bin it
 * owns.  While some cluster has fewer tracks than its region's minimum (3 pp,
 * 2 p-gas), the one with the fewest tracks (lowest z on ties) is removed and
 * the partition is redone; the paper removes one cluster per round.
 */
int orc_partition(orc_cluster *cl, int n_cl, const int *c, const orc_params *p)
{
    const int nb = orc_nbins(p);
    const int gas_bin = orc_gas_bin(p);
    int *live = (int *)malloc(sizeof(int) * (size_t)(n_cl > 0 ? n_cl : 1));
    int i, k, b;
    for (i = 0; i < n_cl; ++i) {
        cl[i].kept = 1;
        cl[i].n_assoc = 0;
        cl[i].own_lo = -1;
        cl[i].own_hi = -1;
    }
    for (;;) {
        int n_live = 0;
        for (i = 0; i < n_cl; ++i)
            if (cl[i].kept)
                live[n_live++] = i;
        int prev_p = -1;
        for (k = 0; k < n_live; ++k) {
            orc_cluster *a = &cl[live[k]];
            const int pk = (k + 1 < n_live) ? (a->hi + cl[live[k + 1]].lo) / 2 : nb - 1;
            a->own_lo = prev_p + 1;
            a->own_hi = pk;
            a->n_assoc = 0;
            for (b = a->own_lo; b <= a->own_hi; ++b)
                a->n_assoc += c[b];
            prev_p = pk;
        }
        int worst = -1;
        for (k = 0; k < n_live; ++k) {
            orc_cluster *a = &cl[live[k]];
            const int need = (a->peak < gas_bin) ? p->part_min_gas : p->part_min_pp;
            if (a->n_assoc < need && (worst < 0 || a->n_assoc < cl[worst].n_assoc))
                worst = live[k];
        }
        if (worst < 0) {
            free(live);
            return n_live;
        }
        cl[worst].kept = 0;
        cl[worst].n_assoc = 0;
        cl[worst].own_lo = -1;
        cl[worst].own_hi = -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.5: adaptive vertex fit                                            */
/* ------------------------------------------------------------------------ */
/* Eq. 17 */
static double tukey(double chi2, double chi2_max)
{
    if (chi2 < chi2_max) {
        const double t = 1.0 - chi2 / chi2_max;
        return t * t;
    }
    return 0.0;
}

/* general 3x3 inverse by the adjugate.  Returns 0 if the matrix counts as
   singular: the paper does not say what happens when the normal matrix is
   singular (for instance when a single track keeps a nonzero weight, which
   leaves z undetermined); the reading here is that the fit fails when
   det(A) <= sing_ratio * A00 A11 A22.  For a symmetric positive semi-definite
   matrix that ratio lies in [0, 1] (Hadamard's inequality) and does not
   depend on the scale of A. */
static int inverse3(const double a[3][3], double inv[3][3], double sing_ratio)
{
    const double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
    const double c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
    const double c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    const double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
    const double diag = a[0][0] * a[1][1] * a[2][2];
    if (!(det > 0.0) || !isfinite(det) || !(det > sing_ratio * diag))
        return 0;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
    inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
    inv[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
    inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
    inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
    inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
    return 1;
}

/* residual of track i at vertex alpha (Eq. 9) and its chi2 (Eq. 7) */
static double track_chi2(const float *const trk[8], int i, const double W[2][2],
                         const double alpha[3], double r[2])
{
    const double x = trk[0][i], y = trk[1][i], z = trk[2][i], tx = trk[3][i], ty = trk[4][i];
    r[0] = x + (alpha[2] - z) * tx - alpha[0];
    r[1] = y + (alpha[2] - z) * ty - alpha[1];
    double Wr[2];
    Wr[0] = W[0][0] * r[0] + W[0][1] * r[1];
    Wr[1] = W[1][0] * r[0] + W[1][1] * r[1];
    return r[0] * Wr[0] + r[1] * Wr[1];
}

static double rel_dist(double q, double t)
{
    return fabs(q - t) / t;
}

/*
 * Newton-Raphson fit of alpha = (x, y, z) (Eq. 10-16).  W_i = V_i^-1 with
 * V_i from Eq. 2 evaluated once at the seed z; with x and y uncorrelated and
 * of identical magnitude, V_i = diag(Vx, Vx) with
 * Vx = Vxx + 2 dz Vxtx + dz^2 Vtxtx, dz = z_seed - z_trk (a track with
 * Vx <= 0 keeps weight 0).  Each iteration evaluates residuals, chi2_i and
 * Tukey weights at the current alpha, forms the gradient and Hessian,
 * steps alpha_1 = alpha_0 - Hess^-1 grad and predicts
 * dchi2 = 1/2 (alpha_1 - alpha_0) . grad.  It stops when |dchi2| < conv_dchi2
 * and |dz_vtx| < conv_dz (x86 criterion), or after max_iter iterations
 * (flagged as not converged, result kept).  C = (Hess / 2)^-1 of the last
 * iteration (Eq. 14); the reported weights and chi2 = sum w_i chi2_i are
 * evaluated at the final alpha, and ndof = 2 sum w - 3.  The fit fails when
 * no weight is left or the Hessian counts as singular (see inverse3).
 */
/* Eq. 18 */
double orc_mv_weight(double chi2, double others, double chi2_max)
{
    const double e = exp(-0.5 * chi2);
    return e / (exp(-0.5 * chi2_max) + e + others);
}

static double fit_weight(double chi2, const double *others, int k, const orc_params *p)
{
    return others ? orc_mv_weight(chi2, others[k], p->chi2_max_mv) : tukey(chi2, p->chi2_max);
}

/* others == NULL: Tukey weights and the x86 criterion; otherwise the weights
   of Eq. 18 and the GPU criterion */
static int fit_core(const float *const trk[8], const int *idx, const double *others, int n,
                    double x_seed, double y_seed, double z_seed, const orc_params *p, int force_iter,
                    orc_vertex *v, double *w_out)
{
    double alpha[3] = {x_seed, y_seed, z_seed};
    double hess_last[3][3];
    double *Wd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int k, it, a, b, converged = 0, n_iter = 0, failed = 0;
    double margin = INFINITY;

    memset(v, 0, sizeof(*v));
    memset(hess_last, 0, sizeof(hess_last));
    v->z_seed = z_seed;

    for (k = 0; k < n; ++k) {
        const int i = idx[k];
        const double dz = z_seed - (double)trk[2][i];
        const double Vx = (double)trk[5][i] + 2.0 * dz * (double)trk[6][i] + dz * dz * (double)trk[7][i];
        Wd[k] = (Vx > 0.0 && isfinite(Vx)) ? 1.0 / Vx : 0.0;   /* 0 marks an unusable track */
    }

    const int n_max = force_iter > 0 ? force_iter : p->max_iter;
    for (it = 1; it <= n_max; ++it) {
        double grad[3] = {0, 0, 0}, hess[3][3], sumw = 0.0;
        memset(hess, 0, sizeof(hess));
        for (k = 0; k < n; ++k) {
            if (Wd[k] == 0.0)
                continue;
            const int i = idx[k];
            const double W[2][2] = {{Wd[k], 0.0}, {0.0, Wd[k]}};
            const double H[2][3] = {{-1.0, 0.0, (double)trk[3][i]}, {0.0, -1.0, (double)trk[4][i]}};
            double r[2];
            const double chi2 = track_chi2(trk, i, W, alpha, r);
            const double w = fit_weight(chi2, others, k, p);
            sumw += w;
            /* grad += 2 w H^T W r ; hess += 2 w H^T W H  (Eq. 10-11) */
            double WH[2][3];
            for (a = 0; a < 2; ++a)
                for (b = 0; b < 3; ++b)
                    WH[a][b] = W[a][0] * H[0][b] + W[a][1] * H[1][b];
            const double Wr[2] = {W[0][0] * r[0] + W[0][1] * r[1], W[1][0] * r[0] + W[1][1] * r[1]};
            for (a = 0; a < 3; ++a) {
                grad[a] += 2.0 * w * (H[0][a] * Wr[0] + H[1][a] * Wr[1]);
                for (b = 0; b < 3; ++b)
                    hess[a][b] += 2.0 * w * (H[0][a] * WH[0][b] + H[1][a] * WH[1][b]);
            }
        }
        double hinv[3][3];
        if (!(sumw > 0.0) || !inverse3(hess, hinv, p->sing_ratio)) {
            failed = 1;
            break;
        }
        double d[3];
        for (a = 0; a < 3; ++a)
            d[a] = -(hinv[a][0] * grad[0] + hinv[a][1] * grad[1] + hinv[a][2] * grad[2]);
        const double dchi2 = 0.5 * (d[0] * grad[0] + d[1] * grad[1] + d[2] * grad[2]);   /* Eq. 16 */
        for (a = 0; a < 3; ++a)
            alpha[a] += d[a];
        memcpy(hess_last, hess, sizeof(hess));
        n_iter = it;
        v->dchi2 = dchi2;

        /* how close this stop/continue decision came to flipping */
        const double q1 = fabs(dchi2), q2 = fabs(d[2]);
        const double tz = others ? p->conv_dz_mv : p->conv_dz;
        const double r1 = others ? INFINITY : rel_dist(q1, p->conv_dchi2), r2 = rel_dist(q2, tz);
        const int below1 = others ? 1 : q1 < p->conv_dchi2, below2 = q2 < tz;
        double frag;
        if (below1 && below2)
            frag = (r1 < r2) ? r1 : r2;
        else if (!below1 && !below2)
            frag = (r1 > r2) ? r1 : r2;
        else
            frag = below1 ? r2 : r1;
        if (frag < margin)
            margin = frag;

        converged = below1 && below2;
        if (converged && force_iter <= 0)
            break;
    }

    if (failed || n_iter == 0) {
        free(Wd);
        v->x = alpha[0];
        v->y = alpha[1];
        v->z = alpha[2];
        v->n_iter = n_iter;
        v->conv_margin = margin;
        for (k = 0; k < n; ++k)
            w_out[k] = 0.0;
        return 1;
    }

    /* Eq. 14: C = (1/2 Hess)^-1 */
    double half[3][3], C[3][3];
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b)
            half[a][b] = 0.5 * hess_last[a][b];
    if (!inverse3(half, C, p->sing_ratio)) {
        free(Wd);
        for (k = 0; k < n; ++k)
            w_out[k] = 0.0;
        return 1;
    }

    double chi2_tot = 0.0, sumw = 0.0;
    for (k = 0; k < n; ++k) {
        if (Wd[k] == 0.0) {
            w_out[k] = 0.0;
            continue;
        }
        const double W[2][2] = {{Wd[k], 0.0}, {0.0, Wd[k]}};
        double r[2];
        const double chi2 = track_chi2(trk, idx[k], W, alpha, r);
        const double w = fit_weight(chi2, others, k, p);
        w_out[k] = w;
        chi2_tot += w * chi2;
        sumw += w;
    }
    free(Wd);

    v->x = alpha[0];
    v->y = alpha[1];
    v->z = alpha[2];
    v->cov[0] = C[0][0];
    v->cov[1] = C[0][1];
    v->cov[2] = C[1][1];
    v->cov[3] = C[0][2];
    v->cov[4] = C[1][2];
    v->cov[5] = C[2][2];
    v->chi2 = chi2_tot;
    v->ndof = 2.0 * sumw - 3.0;
    v->n_iter = n_iter;
    v->flags = converged ? 0 : ORC_VX_NOT_CONVERGED;
    v->conv_margin = margin;
    return 0;
}

int orc_fit(const float *const trk[8], const int *idx, int n,
            double x_seed, double y_seed, double z_seed, const orc_params *p,
            orc_vertex *v, double *w_out)
{
    return fit_core(trk, idx, NULL, n, x_seed, y_seed, z_seed, p, 0, v, w_out);
}

int orc_fit_mv(const float *const trk[8], const int *idx, const double *others, int n,
               double x_seed, double y_seed, double z_seed, const orc_params *p,
               orc_vertex *v, double *w_out)
{
    return fit_core(trk, idx, others, n, x_seed, y_seed, z_seed, p, 0, v, w_out);
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.5 and Sec. 5, GPU variant: implicit association (Eq. 18)          */
/* ------------------------------------------------------------------------ */
/*
 * Every associable track is weighted to every candidate.  Candidate j fits
 * the tracks whose chi2 at its seed is below chi2_window_mv (the pre-cut of
 * Sec. 5, as below; the lists of all candidates together hold at most
 * max_tracks entries, else the event is flagged as too large), with
 * W_ij = 1 / Vx at its seed as in the partition fit, and the
 * weights of Eq. 18, in which the other candidates enter at their seeds
 * (their terms exp(-chi2_ik / 2) are summed over the candidates whose
 * pre-cut the track passes).  Convergence is the GPU criterion |dz| <
 * conv_dz_mv.  A vertex's track count is the number of tracks whose final
 * weight to it is at least w_count_mv (1/2: at chi2 = chi2_max_mv an
 * uncontested track has exactly that weight).  Duplicates: among the
 * successful fits, taken by decreasing track count (lower z first on ties),
 * a vertex is dropped when dz^2 / (Czz_1 + Czz_2) < dup_ratio to one already
 * kept.  Then the selection of the partition path applies (track count,
 * distance to the beamline in the pp region) and the kept vertices are
 * written in z order.  Each track reports the written vertex that gives it
 * the largest final weight (the earlier one on ties), or (-1, 0).
 */
/*
 * Pre-cut (Sec. 5, GPU variant): candidate j fits only the tracks within a
 * chi2 window of its seed.  The chi2 is that of Eq. 7 with the residual of
 * Eq. 9 taken at the seed position alpha_j = (x_b + t_x,b z_seed,
 * y_b + t_y,b z_seed, z_seed) (Sec. 3.3: the seed lies on the beamline) and
 * W = 1 / V_x with V_x from Eq. 2 at the seed, as the fit itself starts
 * (Sec. 3.5), all in binary64.  Returns W (0: unusable track) and the chi2.
 * The same chi2 gives the terms exp(-chi2 / 2) by which candidate j enters
 * the other candidates' weights in Eq. 18.
 */
static double mv_seed_chi2(const float *const ev[8], int i, const double seed[3], double *W)
{
    const double x = ev[0][i], y = ev[1][i], z = ev[2][i], tx = ev[3][i], ty = ev[4][i];
    const double dz = seed[2] - z;
    const double Vx = (double)ev[5][i] + 2.0 * dz * (double)ev[6][i] + dz * dz * (double)ev[7][i];
    *W = (Vx > 0.0 && isfinite(Vx)) ? 1.0 / Vx : 0.0;
    const double rx = x + dz * tx - seed[0];
    const double ry = y + dz * ty - seed[1];
    return *W * (rx * rx + ry * ry);
}

static int forced_iters(const orc_params *p, int peak)
{
    return (p->iter_override_bin >= 0 && peak == p->iter_override_bin) ? p->iter_override_n : 0;
}

static void mv_event(const float *const ev[8], int n, const float beam[4], const orc_params *p, const int *fl,
                     orc_cluster *cl, int ncl, int a, int *status, int *n_vtx,
                     orc_vertex *vtx, int *trk_vtx, double *trk_w)
{
    const int gas_bin = orc_gas_bin(p);
    const int nn = n > 0 ? n : 1, nc = ncl > 0 ? ncl : 1;
    double *e0 = (double *)calloc((size_t)nc * (size_t)nn, sizeof(double));   /* e0[j n + i] */
    char *in = (char *)calloc((size_t)nc * (size_t)nn, 1);
    int *idx = (int *)malloc(sizeof(int) * (size_t)nn);
    double *oth = (double *)malloc(sizeof(double) * (size_t)nn);
    double *w = (double *)malloc(sizeof(double) * (size_t)nn);
    double *wall = (double *)calloc((size_t)nc * (size_t)nn, sizeof(double)); /* final weights */
    orc_vertex *cand = (orc_vertex *)calloc((size_t)nc, sizeof(orc_vertex));
    int *ok = (int *)calloc((size_t)nc, sizeof(int));
    int *keep = (int *)calloc((size_t)nc, sizeof(int));
    int i, j, k;

    /* pre-cut and the terms of Eq. 18 at the seeds */
    long total = 0;
    for (j = 0; j < ncl; ++j) {
        const double zs = cl[j].z_seed;
        const double seed[3] = {(double)beam[0] + (double)beam[2] * zs, (double)beam[1] + (double)beam[3] * zs, zs};
        int m = 0, near = 0;
        for (i = 0; i < n; ++i) {
            if (!(fl[i] & ORC_TR_ASSOC))
                continue;
            double W;
            const double chi2 = mv_seed_chi2(ev, i, seed, &W);
            if (!(W > 0.0))
                continue;
            if (chi2 < p->chi2_window_mv) {
                in[(size_t)j * nn + i] = 1;
                e0[(size_t)j * nn + i] = exp(-0.5 * chi2);
                ++m;
            }
            if (fabs(chi2 - p->chi2_window_mv) <= p->tie_rel * p->chi2_window_mv)
                ++near;
        }
        cl[j].kept = 1;
        cl[j].n_assoc = m;
        cl[j].n_near_cut = near;
        cl[j].own_lo = cl[j].own_hi = -1;
        total += m;
    }
    /* the candidates' track lists share the event's track capacity */
    if (total > p->max_tracks) {
        *status |= ORC_EV_TOO_MANY_TRACKS;
        ncl = 0;
    }

    /* one fit per candidate */
    for (j = 0; j < ncl; ++j) {
        int m = 0;
        for (i = 0; i < n; ++i) {
            if (!in[(size_t)j * nn + i])
                continue;
            double o = 0.0;
            for (k = 0; k < ncl; ++k)
                if (k != j)
                    o += e0[(size_t)k * nn + i];
            idx[m] = i;
            oth[m] = o;
            ++m;
        }
        const double zs = cl[j].z_seed;
        const double xs = (double)beam[0] + (double)beam[2] * zs;
        const double ys = (double)beam[1] + (double)beam[3] * zs;
        ok[j] = !fit_core(ev, idx, oth, m, xs, ys, zs, p, forced_iters(p, cl[j].peak), &cand[j], w);
        if (!ok[j])
            *status |= ORC_EV_FIT_FAILED;
        int cnt = 0, near = 0;
        for (k = 0; k < m; ++k) {
            wall[(size_t)j * nn + idx[k]] = w[k];
            if (w[k] >= p->w_count_mv)
                ++cnt;
            if (fabs(w[k] - p->w_count_mv) < 1e-4)
                ++near;
        }
        cand[j].n_tracks = cnt;
        cand[j].n_near = near;
        cand[j].dup_margin = INFINITY;
        cand[j].bin_lo = cl[j].lo;
        cand[j].bin_hi = cl[j].hi;
        cand[j].peak_bin = cl[j].peak;
    }

    /* duplicates: the successful fits by decreasing track count, lower z
       first on ties; each is kept unless it duplicates one kept before it */
    for (;;) {
        int best = -1;
        for (j = 0; j < ncl; ++j)   /* ok[j]: fitted and not yet decided */
            if (ok[j] && (best < 0 || cand[j].n_tracks > cand[best].n_tracks))
                best = j;
        if (best < 0)
            break;
        int dup = 0;
        for (k = 0; k < ncl; ++k) {
            if (!keep[k])
                continue;
            const double d = cand[best].z - cand[k].z;
            const double lim = p->dup_ratio * (cand[best].cov[5] + cand[k].cov[5]);
            if (d * d < lim)
                dup = 1;
            const double mg = lim > 0.0 ? fabs(d * d / lim - 1.0) : INFINITY;
            if (mg < cand[best].dup_margin)
                cand[best].dup_margin = mg;
            if (mg < cand[k].dup_margin)
                cand[k].dup_margin = mg;
        }
        ok[best] = 0;
        keep[best] = !dup;
    }

    /* selection, output in z order */
    int *out_of = (int *)malloc(sizeof(int) * (size_t)nc);
    for (j = 0; j < ncl; ++j) {
        out_of[j] = -1;
        if (!keep[j])
            continue;
        const int gas = cl[j].peak < gas_bin;
        int sel = cand[j].n_tracks >= (gas ? p->pv_min_gas : p->pv_min_pp);
        if (sel && !gas) {
            const double bx = cand[j].x - ((double)beam[0] + (double)beam[2] * cand[j].z);
            const double by = cand[j].y - ((double)beam[1] + (double)beam[3] * cand[j].z);
            sel = sqrt(bx * bx + by * by) <= p->max_rho_pp;
        }
        if (!sel)
            continue;
        out_of[j] = (*n_vtx)++;
        vtx[out_of[j]] = cand[j];
    }
    for (i = 0; i < n; ++i) {
        int bv = -1;
        double bw = 0.0;
        for (j = 0; j < ncl; ++j) {
            if (out_of[j] < 0 || !in[(size_t)j * nn + i])
                continue;
            const double wij = wall[(size_t)j * nn + i];
            if (bv < 0 || wij > bw) {
                bv = out_of[j];
                bw = wij;
            }
        }
        trk_vtx[a + i] = bv;
        trk_w[a + i] = bv >= 0 ? bw : 0.0;
    }
    free(out_of);
    free(e0);
    free(in);
    free(idx);
    free(oth);
    free(w);
    free(wall);
    free(cand);
    free(ok);
    free(keep);
}

/* ------------------------------------------------------------------------ */
/* the whole path                                                           */
/* ------------------------------------------------------------------------ */
/*
 * Per event: project, histogram, peak search (clusters beyond max_vertices,
 * counted in z order, are dropped and flagged), association, one fit per
 * surviving cluster, then the final selection: a vertex is kept if its fit
 * succeeded, its cluster owns at least 4 (pp) / 3 (p-gas) tracks (Table 2),
 * and, in the pp region, it lies within max_rho_pp of the beamline (end of
 * Sec. 3.5).  Regions are decided by the cluster's highest bin.  Kept
 * vertices are written in z (cluster) order; their tracks get the vertex
 * index and final weight, every other track (-1, 0).  With assoc_mode
 * ORC_ASSOC_MULTIVERTEX the association, fit and selection are those of the
 * GPU variant (mv_event).
 */
static void find_event(const float *const trk[8], int a, int n, const float beam[4],
                       const orc_params *p, int nb, int *n_vtx, int *status, orc_vertex *vtx,
                       int *trk_vtx, double *trk_w, int *hist, orc_cluster *clusters,
                       int *n_clusters, float *trk_zpoca, float *trk_sigma, int *trk_bin)
{
    const int maxv = p->max_vertices;
    const int gas_bin = orc_gas_bin(p);
    const float *ev[8];
    int i, k, q;
    for (k = 0; k < 8; ++k)
        ev[k] = trk[k] + a;
    *n_vtx = 0;
    if (n_clusters)
        *n_clusters = 0;
    for (i = 0; i < n; ++i) {
        trk_vtx[a + i] = -1;
        trk_w[a + i] = 0.0;
    }
    if (n > p->max_tracks) {
        *status |= ORC_EV_TOO_MANY_TRACKS;
        if (hist)
            memset(hist, 0, sizeof(int) * (size_t)nb);
        return;
    }

    int *bin = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *fl = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (i = 0; i < n; ++i) {
        float t[8], zp, sg;
        for (k = 0; k < 8; ++k)
            t[k] = ev[k][i];
        fl[i] = orc_project(t, beam, p, &zp, &sg, &bin[i]);
        if (fl[i] & ORC_TR_NONFINITE)
            *status |= ORC_EV_NONFINITE_INPUT;
        if (trk_zpoca)
            trk_zpoca[a + i] = zp;
        if (trk_sigma)
            trk_sigma[a + i] = sg;
        if (trk_bin)
            trk_bin[a + i] = bin[i];
    }

    int *h = (int *)malloc(sizeof(int) * (size_t)nb);
    int *c = (int *)malloc(sizeof(int) * (size_t)nb);
    orc_hist_event(ev, n, beam, p, h, c);
    if (hist)
        memcpy(hist, h, sizeof(int) * (size_t)nb);

    orc_cluster *cl = (orc_cluster *)calloc((size_t)(maxv > 0 ? maxv : 1), sizeof(orc_cluster));
    int overflow = 0;
    const int ncl = orc_peak_search(h, p, cl, maxv, &overflow);
    if (overflow)
        *status |= ORC_EV_VERTEX_OVERFLOW;
    if (p->assoc_mode == ORC_ASSOC_MULTIVERTEX) {
        mv_event(ev, n, beam, p, fl, cl, ncl, a, status, n_vtx, vtx, trk_vtx, trk_w);
        if (clusters) {
            memcpy(clusters, cl, sizeof(orc_cluster) * (size_t)ncl);
            *n_clusters = ncl;
        }
        free(cl);
        free(h);
        free(c);
        free(bin);
        free(fl);
        return;
    }
    orc_partition(cl, ncl, c, p);
    if (clusters) {
        memcpy(clusters, cl, sizeof(orc_cluster) * (size_t)ncl);
        *n_clusters = ncl;
    }

    int *idx = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (q = 0; q < ncl; ++q) {
        if (!cl[q].kept)
            continue;
        int m = 0;
        for (i = 0; i < n; ++i)
            if ((fl[i] & ORC_TR_ASSOC) && bin[i] >= cl[q].own_lo && bin[i] <= cl[q].own_hi)
                idx[m++] = i;
        const double zs = cl[q].z_seed;
        const double xs = (double)beam[0] + (double)beam[2] * zs;
        const double ys = (double)beam[1] + (double)beam[3] * zs;
        orc_vertex v;
        const int bad = fit_core(ev, idx, NULL, m, xs, ys, zs, p, forced_iters(p, cl[q].peak), &v, w);
        if (bad)
            *status |= ORC_EV_FIT_FAILED;
        const int gas = cl[q].peak < gas_bin;
        int keep = !bad && cl[q].n_assoc >= (gas ? p->pv_min_gas : p->pv_min_pp);
        if (keep && !gas) {
            const double bx = v.x - ((double)beam[0] + (double)beam[2] * v.z);
            const double by = v.y - ((double)beam[1] + (double)beam[3] * v.z);
            keep = sqrt(bx * bx + by * by) <= p->max_rho_pp;
        }
        if (!keep)
            continue;
        v.n_tracks = cl[q].n_assoc;
        v.bin_lo = cl[q].lo;
        v.bin_hi = cl[q].hi;
        v.peak_bin = cl[q].peak;
        const int out = (*n_vtx)++;
        vtx[out] = v;
        for (k = 0; k < m; ++k) {
            trk_vtx[a + idx[k]] = out;
            trk_w[a + idx[k]] = w[k];
        }
    }
    free(idx);
    free(w);
    free(cl);
    free(h);
    free(c);
    free(bin);
    free(fl);
}

int orc_find(const float *const trk[8], const int *offsets, int n_events,
             const float beam[4], const orc_params *p,
             int *n_vtx, int *status, orc_vertex *vtx, int *trk_vtx, double *trk_w,
             int *hist, orc_cluster *clusters, int *n_clusters,
             float *trk_zpoca, float *trk_sigma, int *trk_bin, int n_threads)
{
    const int nb = orc_nbins(p);
    int e;
    if (nb < 0 || n_events < 0 || !offsets || !p || p->max_vertices < 1 || p->frac_bits < 1 ||
        p->frac_bits > 20)
        return -1;
    if (n_threads <= 0)
        n_threads = orc_max_threads();
    const int total = offsets[n_events];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(n_threads)
#endif
    for (e = 0; e < n_events; ++e) {
        const int a = offsets[e], b = offsets[e + 1];
        status[e] = 0;
        n_vtx[e] = 0;
        if (n_clusters)
            n_clusters[e] = 0;
        if (a < 0 || b < a || b > total) {
            status[e] = ORC_EV_OFFSETS_INVALID;
            if (hist)
                memset(hist + (size_t)e * nb, 0, sizeof(int) * (size_t)nb);
            continue;
        }
        find_event(trk, a, b - a, beam, p, nb, &n_vtx[e], &status[e],
                   vtx + (size_t)e * p->max_vertices, trk_vtx, trk_w,
                   hist ? hist + (size_t)e * nb : NULL,
                   clusters ? clusters + (size_t)e * p->max_vertices : NULL,
                   n_clusters ? &n_clusters[e] : NULL, trk_zpoca, trk_sigma, trk_bin);
    }
    return 0;
}
