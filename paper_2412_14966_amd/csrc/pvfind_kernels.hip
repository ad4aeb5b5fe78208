// pvfind_kernels.hip -- gfx950 kernels of the primary-vertex finding path
// (arXiv:2412.14966, Sec. 3 and Sec. 5).
//
// One fused kernel runs the five steps of Sec. 3 for one event per team of W
// wavefronts.  In persistent mode a grid sized to the chip pops events from a
// device work queue; otherwise one workgroup per event is hardware-scheduled.
// Per event:
//   clear     the LDS histogram (16 KiB for 4000 bins)
//   project   coalesced SoA loads, one lane per track, Eq. 1 / Eq. 3 in
//             binary32 with correctly rounded division and square root and
//             no contraction (the file is built with -ffp-contract=off), so
//             z_poca, sigma_poca and the central bin are bit-reproducible
//   fill      integer fixed-point kernel masses added with LDS atomics: the
//             histogram does not depend on the order of the adds; a 64-bit
//             mask records which 64-bin words were touched
//   peaks     wavefront ballots over the touched words give the proto-cluster
//             runs (bit tricks on the masks), then one lane per proto-cluster
//             walks the dip search and z-ordered splitting; clusters are
//             compacted in z order with a wavefront scan
//   associate partition points, per-track owner by binary search, LDS
//             counters, removal of the weakest cluster until all pass
//   gather    stable compaction of the tracks by vertex into LDS arrays that
//             reuse the histogram's space; positions are stored relative to
//             the beamline point at the centre of the seed's peak bin (exact
//             in binary32), so the fit works on small numbers and starts at
//             the seed offset delta dz without rounding the seed itself
//   fit       a power-of-two group of lanes per vertex, sums reduced with
//             butterflies; the 3x3 Newton step is solved by eliminating x and
//             y (the normal matrix has zeros at (x, y)); covariance inverted
//             in binary64 only when its 1-norm condition number is large
//   select    Table 2 minimum tracks and the beamline-distance cut, prefix
//             compaction of the kept vertices, final weights per track
// Events with more tracks than a small team holds go to a second launch with
// eight-wavefront teams holding 4096 tracks.
#include "pvfind_device.h"

#include <map>
#include <mutex>
#include <type_traits>

namespace pvk {

// Fit state of the live vertices: position relative to the frame, the last
// normal matrix (a, b, c, d as in Eq. 14, of the slopes relative to the
// reference slope tx, ty) and n_iter | not_converged << 8 | failed << 9.
template <int V>
struct VertexFit {
    float dx[V], dy[V], dz[V];
    float a[V], b[V], c[V], d[V];
    float tx[V], ty[V];   // reference slope of the fit (normal matrix a..d is that of the shifted slopes)
    int info[V];
};

constexpr int kPages = 20;          // touched 64-bin histogram words a small team holds
constexpr int kSmallVertices = 48;  // clusters a small team of up to 512 tracks holds (64 above)
constexpr int kMvSortMin = 16;      // candidates from which the multi-vertex pre-cut takes tracks in z order

// LDS of one team.  Large-event teams hold the whole histogram.  Small teams
// hold only the touched 64-bin words ("pages"): word w lives in page
// popcount(touched words below w), so touched words that are neighbours in z
// are neighbours in LDS and every window, run and cluster maps to LDS by one
// offset.  Events that touch more than kPages words or give more than
// kSmallVertices clusters go to the large-team launch.
template <int W, int CAP, bool BIG, bool MV>
struct __align__(16) Smem {
    static constexpr int V = BIG ? kMaxVertices : (CAP <= 512 ? kSmallVertices : 64);
    union {
        int hist[BIG ? kMaxBins : 1];
        struct {
            int pg[kPages * 64];
            float tz[CAP];   // z_poca of each histogrammed track (small teams, between the passes)
            float tr[CAP];   // its 1 / (u0 sigma)
            int tw[CAP];     // its window jl | jh << 16, 0 for none
        } pp;
        struct {
            // one slot per (vertex, track) pair of the fit, by vertex
            float X[CAP];    // track x at the seed z, relative to the seed
            float Y[CAP];
            float TX[CAP];
            float TY[CAP];
            float WT[CAP];   // 1 / V_x at the seed (Eq. 2), 0 for unusable tracks
            float OTH[MV ? CAP : 1];      // multi-vertex: the other candidates' terms of Eq. 18
            unsigned BEST[MV ? CAP : 1];  // multi-vertex, per track: best weight | vertex
            short IDX[CAP];  // track index within the event
        } f;
    } u;
    union {
        int tb[CAP];         // up to the gather: (bin + 1) | flags << 13 | (owner + 1) << 16
        VertexFit<V> vf;     // fit onwards
    };
    short clo[V], chi[V], cpk[V];
    float cd0[V];            // seed offset delta * dz from the centre of the peak bin (Eq. 4)
    short live[V];
    int pb[V];               // last bin owned by live slot k
    int cnt[V];              // tracks owned by live slot k
    int base[V];             // first gathered slot of live slot k
    union {
        int wrun[W][V];      // gather: running slot per wavefront and live slot
        struct {
            short ps[64], pe[64];   // peak search: pending proto-clusters
            int po[64];             // their LDS offsets
        };
        short lmap[64 * W];  // fit: per lane, its vertex | log2 of its group's lanes << 8, -1 for none
    };
    int vout[V];
    int ntk[MV ? V : 1];     // multi-vertex: tracks of final weight >= w_count_mv
    float czz[MV ? V : 1];   // multi-vertex: C_zz for the duplicate test
    unsigned long long occ;
    int ev, status, n_cl, n_live, done, n_keep, defer, n_slots;
    int zord;                // multi-vertex: the candidates' seeds are in z order
};

// the histogram as the team holds it: h[j + off] is bin j
template <int W, int CAP, bool BIG, bool MV>
__device__ __forceinline__ int *hist_lds(Smem<W, CAP, BIG, MV> &S)
{
    if constexpr (BIG)
        return S.u.hist;
    else
        return S.u.pp.pg;
}

// page offset of touched word w (small teams): bin j of that word, and of the
// touched words after it without a gap, is pg[j + page_off(occ, w)]
__device__ __forceinline__ int page_off(unsigned long long occ, int w)
{
    return 64 * (__popcll(occ & ((1ull << w) - 1ull)) - w);
}

template <int W, int CAP, bool BIG, bool MV>
__device__ __forceinline__ int bin_value(Smem<W, CAP, BIG, MV> &S, unsigned long long occ, int j)
{
    if constexpr (BIG) {
        return S.u.hist[j];
    } else {
        const int w = j >> 6;
        return ((occ >> w) & 1ull) ? S.u.pp.pg[j + page_off(occ, w)] : 0;
    }
}

// Whole peak search, run by wavefront 0.  Proto-cluster runs come from
// ballots of (bin > proto_thr) over the touched 64-bin words; they are queued
// and walked 32-64 at a time, one lane per proto-cluster.
template <int W, int CAP, bool BIG, bool MV>
__device__ __forceinline__ void peak_search(Smem<W, CAP, BIG, MV> &S, const KParams &p)
{
    const int lane = threadIdx.x & 63;
    int *h = hist_lds(S);
    const int cap = BIG ? p.max_vertices : min(p.max_vertices, Smem<W, CAP, BIG, MV>::V);
    int n_found = 0, npend = 0, open_s = -1, open_off = 0, prev_w = -2, pgi = 0;
    const unsigned long long occ0 = S.occ;
    unsigned long long occ = occ0;
    auto push = [&](int s, int e, int off) __attribute__((always_inline)) {
        if (lane == 0) {
            S.ps[npend] = (short)s;
            S.pe[npend] = (short)e;
            S.po[npend] = off;
        }
        ++npend;
    };
    for (;;) {
        const bool last = (occ == 0ull);
        if (!last) {
            // one word adds at most 32 runs plus the close of an open one
            const int w = __ffsll((long long)occ) - 1;
            occ &= occ - 1ull;
            const int off = BIG ? 0 : 64 * (pgi - w);
            if (open_s >= 0 && prev_w != w - 1) {
                push(open_s, 64 * prev_w + 63, open_off);
                open_s = -1;
            }
            const int j = 64 * w + lane;
            const int hv = (j < p.nb) ? h[j + off] : 0;
            const unsigned long long m = __ballot(hv > p.proto_thr);
            unsigned long long st = m & ~(m << 1);
            unsigned long long en = m & ~(m >> 1);
            int cur = -1, cur_off = off;
            if (open_s >= 0) {
                if (m & 1ull) {
                    cur = open_s;
                    cur_off = open_off;
                    st &= ~1ull;
                } else {
                    push(open_s, 64 * w - 1, open_off);
                }
                open_s = -1;
            }
            while (en) {
                const int eb = __ffsll((long long)en) - 1;
                en &= en - 1ull;
                if (cur < 0) {
                    const int sb = __ffsll((long long)st) - 1;
                    st &= st - 1ull;
                    cur = 64 * w + sb;
                    cur_off = off;
                }
                if (eb == 63) {
                    open_s = cur;
                    open_off = cur_off;
                } else {
                    push(cur, 64 * w + eb, cur_off);
                }
                cur = -1;
            }
            prev_w = w;
            ++pgi;
        } else if (open_s >= 0) {
            push(open_s, 64 * prev_w + 63, open_off);
            open_s = -1;
        }
        __builtin_amdgcn_wave_barrier();
        if (npend >= 32 || (last && npend > 0)) {
            const bool has = lane < npend;
            int s = 0, e = 0, off = 0;
            if (has) {
                s = S.ps[lane];
                e = S.pe[lane];
                off = S.po[lane];
            }
            if (p.peak_rec) {
                // x86 variant: count, then write from this lane's first index
                const int c = has ? walk_recursive<false>(h, off, p, s, e, nullptr, nullptr, nullptr, 0, 0) : 0;
                const int incl = wave_incl_scan(c, lane);
                if (has && c > 0)
                    walk_recursive<true>(h, off, p, s, e, S.clo, S.chi, S.cpk, cap, n_found + incl - c);
                n_found += __shfl(incl, 63);
            } else {
                const int tot = has ? sum_bins(h, off, s, e) : 0;
                WalkOut wo{{0u, 0u, 0u, 0u}, 0, -1};
                const int c = has ? walk_proto<false>(h, off, p, s, e, tot, wo, nullptr, nullptr, nullptr, 0, 0) : 0;
                const int incl = wave_incl_scan(c, lane);
                const int first = n_found + incl - c;
                if (has && wo.nsplit > 4)   // rare: more splits than recorded
                    walk_proto<true>(h, off, p, s, e, tot, wo, S.clo, S.chi, S.cpk, cap, first);
                else if (has)
                    write_walk(wo, s, e, S.clo, S.chi, S.cpk, cap, first);
                n_found += __shfl(incl, 63);
            }
            npend = 0;
            __builtin_amdgcn_wave_barrier();
        }
        if (last)
            break;
    }

    __builtin_amdgcn_wave_barrier();
    const int ncl = min(n_found, cap);
    // seeds (Eq. 4-5): first highest bin (found by the walk), correction from the neighbours
    for (int q = lane; q < ncl; q += 64) {
        const int im = S.cpk[q];
        const int Ni = bin_value(S, occ0, im);
        const int Nm = (im > 0) ? bin_value(S, occ0, im - 1) : 0;
        const int Np = (im + 1 < p.nb) ? bin_value(S, occ0, im + 1) : 0;
        const int den = 2 * Ni - Np - Nm;
        float delta = (den > 0) ? 0.5f * (float)(Np - Nm) / (float)den : 0.0f;
        delta = fminf(fmaxf(delta, -0.5f), 0.5f);
        S.cd0[q] = delta * p.dz;
    }
    if (lane == 0) {
        S.n_cl = ncl;
        if (n_found > p.max_vertices)
            S.status |= PV_EV_VERTEX_OVERFLOW;
        // more clusters than a small team holds, where the caller allows more
        S.defer = (!BIG && n_found > cap && p.max_vertices > cap) ? 1 : 0;
    }
}

// L = 1 << lg lanes per vertex, wavefront-uniform (scalar): one copy of the
// code serves every group size.
template <int W, int CAP, bool BIG, bool MV>
__device__ __forceinline__ void fit_vertices(Smem<W, CAP, BIG, MV> &S, const KParams &p, int nl, int lg, bool prop)
{
    const int tid = threadIdx.x;
    // uniform: L = 2^lg lanes per vertex; proportional: the lane map's groups
    const int m = prop ? (int)S.lmap[tid] : (((tid >> lg) < nl) ? ((tid >> lg) | (lg << 8)) : -1);
    const bool has = m >= 0;
    const int k = has ? (m & 0xFF) : 0;
    const int L = prop ? (1 << (has ? (m >> 8) : 0)) : (1 << lg);
    const int gl = tid & (L - 1);
    // the deepest butterfly level any group of this wavefront needs
    const int lgmax = prop ? __builtin_amdgcn_readfirstlane(-wave_min(-(has ? (m >> 8) : 0))) : lg;
    {
        const int beg = has ? S.base[k] : 0, ck = has ? S.cnt[k] : 0;
        float rX[kRegTracks], rY[kRegTracks], rTX[kRegTracks], rTY[kRegTracks], rW[kRegTracks];
        float rO[MV ? kRegTracks : 1];
#pragma unroll
        for (int u = 0; u < kRegTracks; ++u) {
            const int t = gl + u * L;
            if (t < ck) {
                const int sl = beg + t;
                rX[u] = S.u.f.X[sl];
                rY[u] = S.u.f.Y[sl];
                rTX[u] = S.u.f.TX[sl];
                rTY[u] = S.u.f.TY[sl];
                rW[u] = S.u.f.WT[sl];
                if constexpr (MV)
                    rO[u] = S.u.f.OTH[sl];
            } else {
                rX[u] = rY[u] = rTX[u] = rTY[u] = rW[u] = 0.0f;
                if constexpr (MV)
                    rO[u] = 0.0f;
            }
        }
        // Reference slope: the mean of the vertex's track slopes.  The fit's
        // unknowns are e = (dx, dy) - dz t_ref and dz, its slopes t - t_ref:
        // residuals, chi2 and the step's chi2 change are those of (dx, dy, dz),
        // but the normal matrix holds no cancellation between s0 szz and
        // sx^2 + sy^2 when the slopes are alike, which in binary32 moved
        // vertices of a few tracks by micrometres.
        float trx = 0.0f, try_ = 0.0f;
        {
            float ts[2] = {0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < kRegTracks; ++u) {
                ts[0] += rTX[u];
                ts[1] += rTY[u];
            }
            for (int t = gl + kRegTracks * L; t < ck; t += L) {
                ts[0] += S.u.f.TX[beg + t];
                ts[1] += S.u.f.TY[beg + t];
            }
            if (prop)
                group_sum_n_var_rt<2>(ts, L, lgmax);
            else
                group_sum_n_rt<2>(ts, lg);
            const float inv_n = (ck > 0) ? __builtin_amdgcn_rcpf((float)ck) : 0.0f;
            trx = ts[0] * inv_n;
            try_ = ts[1] * inv_n;
#pragma unroll
            for (int u = 0; u < kRegTracks; ++u) {
                rTX[u] -= trx;
                rTY[u] -= try_;
            }
        }

        // start at the seed: on the beamline, delta dz above the bin centre
        const float d0 = has ? S.cd0[S.live[k]] : 0.0f;
        float dx = (p.btx - trx) * d0, dy = (p.bty - try_) * d0, dz = d0, la = 0.0f, lb = 0.0f, lc = 0.0f,
              ld = 0.0f;
        int nit = 0;
        bool active = has, failed = false, conv = false;
        for (int it = 1; it <= p.max_iter; ++it) {
            if (!__any(active))
                break;
            FitSums a = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            if (active) {
#pragma unroll
                for (int u = 0; u < kRegTracks; ++u)
                    if (rW[u] > 0.0f) {
                        if constexpr (MV)
                            accumulate_mv(a, rX[u], rY[u], rTX[u], rTY[u], rW[u], rO[u], dx, dy, dz, p);
                        else
                            accumulate(a, rX[u], rY[u], rTX[u], rTY[u], rW[u], dx, dy, dz, p);
                    }
                for (int t = gl + kRegTracks * L; t < ck; t += L) {
                    const int sl = beg + t;
                    const float wt = S.u.f.WT[sl];
                    if (wt > 0.0f) {
                        if constexpr (MV)
                            accumulate_mv(a, S.u.f.X[sl], S.u.f.Y[sl], S.u.f.TX[sl] - trx, S.u.f.TY[sl] - try_, wt,
                                          S.u.f.OTH[sl], dx, dy, dz, p);
                        else
                            accumulate(a, S.u.f.X[sl], S.u.f.Y[sl], S.u.f.TX[sl] - trx, S.u.f.TY[sl] - try_, wt, dx,
                                       dy, dz, p);
                    }
                }
            }
            float r[7] = {a.s0, a.sx, a.sy, a.szz, a.gx, a.gy, a.gz};
            if (prop)
                group_sum_n_var_rt<7>(r, L, lgmax);
            else
                group_sum_n_rt<7>(r, lg);
            const float s0 = r[0], sx = r[1], sy = r[2], szz = r[3], gx = r[4], gy = r[5], gz = r[6];
            if (active) {
                // A = [[s0, 0, -sx], [0, s0, -sy], [-sx, -sy, szz]], half-gradient (-gx, -gy, gz),
                // in the shifted slopes; det(A) = s0 * D is the same for the slopes
                // themselves, singular when det <= sing_ratio * s0 * s0 * szz with szz
                // that of the slopes themselves
                const float D = fmaf(s0, szz, -fmaf(sx, sx, sy * sy));
                const float szz_t = fmaf(s0, fmaf(trx, trx, try_ * try_), fmaf(2.0f, fmaf(trx, sx, try_ * sy), szz));
                if (!(s0 > 0.0f) || !(D > p.sing_ratio * (s0 * szz_t))) {
                    failed = true;
                    active = false;
                } else {
                    // eliminate x and y: D dz = sx gx + sy gy - s0 gz, then s0 dx = gx + sx dz
                    const float rs0 = __builtin_amdgcn_rcpf(s0);
                    const float ddz = fmaf(sx, gx, fmaf(sy, gy, -s0 * gz)) * __builtin_amdgcn_rcpf(D);
                    const float ddx = fmaf(sx, ddz, gx) * rs0;
                    const float ddy = fmaf(sy, ddz, gy) * rs0;
                    const float dchi2 = fmaf(ddz, gz, -fmaf(ddx, gx, ddy * gy));   // Eq. 16
                    dx += ddx;
                    dy += ddy;
                    dz += ddz;
                    la = s0;
                    lb = sx;
                    lc = sy;
                    ld = szz;
                    nit = it;
                    // x86 criterion, or the GPU variant's |dz| alone (Sec. 3.5)
                    if (MV ? (fabsf(ddz) < p.conv_dz_mv) : (fabsf(dchi2) < p.conv_dchi2 && fabsf(ddz) < p.conv_dz)) {
                        conv = true;
                        active = false;
                    }
                }
            }
        }
        if (has && gl == 0) {
            // back to the frame's transverse offsets: (dx, dy) = e + dz t_ref
            S.vf.dx[k] = fmaf(dz, trx, dx);
            S.vf.dy[k] = fmaf(dz, try_, dy);
            S.vf.dz[k] = dz;
            S.vf.a[k] = la;
            S.vf.b[k] = lb;
            S.vf.c[k] = lc;
            S.vf.d[k] = ld;
            S.vf.tx[k] = trx;
            S.vf.ty[k] = try_;
            S.vf.info[k] = nit | (conv ? 0 : kInfoNotConv) | (failed ? kInfoFailed : 0);
            if (failed)
                atomicOr(&S.status, PV_EV_FIT_FAILED);
        }
    }
}

// Final weights at the fitted position (Tukey, or Eq. 18 for the multi-vertex
// variant), per-track outputs, chi2 and ndof (2 sum w - 3), covariance
// (Eq. 14) and the vertex record.  Multi-vertex: the weights and chi2 were
// stored by the counting pass at the same positions; a track may sit in
// several candidates' lists, and each written vertex offers it (weight, vertex) through an
// LDS maximum over keys (top 24 bits of the weight, then the lower vertex
// index), and the winning slot writes the track's outputs.
template <int W, int CAP, bool BIG, bool MV>
__device__ __forceinline__ void final_pass(Smem<W, CAP, BIG, MV> &S, const KArgs &A, int e, int a, int n, int nl,
                                           int L, int lg)
{
    constexpr int NT = 64 * W;
    const int G = NT >> lg;
    const KParams &p = A.p;
    const int tid = threadIdx.x;
    const int gid = tid >> lg, gl = tid & (L - 1);
    auto weight_at = [&](int sl, float dx, float dy, float dz, float &chi2) __attribute__((always_inline)) -> float {
        if constexpr (MV) {   // stored by the counting pass at the final position
            chi2 = S.u.f.X[sl];
            return S.u.f.OTH[sl];
        }
        const float wt = S.u.f.WT[sl];
        float w = 0.0f;
        chi2 = 0.0f;
        if (wt > 0.0f) {
            const float rx = fmaf(dz, S.u.f.TX[sl], S.u.f.X[sl]) - dx;
            const float ry = fmaf(dz, S.u.f.TY[sl], S.u.f.Y[sl]) - dy;
            chi2 = wt * fmaf(rx, rx, ry * ry);
            if (chi2 < p.chi2_max) {
                const float u = fmaf(-chi2, p.inv_chi2_max, 1.0f);
                w = u * u;
            }
        }
        return w;
    };
    for (int k0 = 0; k0 < nl; k0 += G) {
        const int k = k0 + gid;
        const bool has = k < nl;
        const int beg = has ? S.base[k] : 0, ck = has ? S.cnt[k] : 0;
        const int vo = has ? S.vout[k] : -1;
        const float dx = has ? S.vf.dx[k] : 0.0f, dy = has ? S.vf.dy[k] : 0.0f, dz = has ? S.vf.dz[k] : 0.0f;
        float schi = 0.0f, sw = 0.0f;
        for (int t = gl; t < ck; t += L) {
            const int sl = beg + t;
            float chi2;
            const float w = weight_at(sl, dx, dy, dz, chi2);
            schi = fmaf(w, chi2, schi);
            sw += w;
            if constexpr (MV) {
                if (vo >= 0)
                    atomicMax(&S.u.f.BEST[S.u.f.IDX[sl]], (__float_as_uint(w) & 0xFFFFFF00u) | (255u - (unsigned)vo));
            } else {
                const int g = a + S.u.f.IDX[sl];
                A.trk_vtx[g] = vo;
                A.trk_w[g] = (vo >= 0) ? w : 0.0f;
            }
        }
        schi = group_sum_rt(schi, L);
        sw = group_sum_rt(sw, L);
        if (has && gl == 0 && vo >= 0) {
            const int cq = S.live[k];
            const float zr = bin_centre(S.cpk[cq], p);
            float cf[6];
            int flags = (S.vf.info[k] & kInfoNotConv) ? PV_VX_NOT_CONVERGED : 0;
            if (vertex_covariance(S.vf.a[k], S.vf.b[k], S.vf.c[k], S.vf.d[k], S.vf.tx[k], S.vf.ty[k], p.cond_fp64, cf))
                flags |= PV_VX_FP64_INVERSION;
            pv_vertex v;
            v.x = (p.bx + p.btx * zr) + dx;
            v.y = (p.by + p.bty * zr) + dy;
            v.z = zr + dz;
            for (int q = 0; q < 6; ++q)
                v.cov[q] = cf[q];
            v.chi2 = schi;
            v.ndof = 2.0f * sw - 3.0f;
            v.z_seed = zr + S.cd0[cq];
            v.n_tracks = MV ? S.ntk[k] : S.cnt[k];
            v.bin_lo = S.clo[cq];
            v.bin_hi = S.chi[cq];
            v.peak_bin = S.cpk[cq];
            v.n_iter = (uint8_t)(S.vf.info[k] & 0xFF);
            v.flags = (uint8_t)flags;
            v.reserved = 0;
            A.vout[(size_t)e * p.max_vertices + vo] = v;
        }
    }
    if constexpr (MV) {
        __syncthreads();
        // tracks no written vertex took
        for (int i = tid; i < n; i += NT)
            if (S.u.f.BEST[i] == 0u) {
                A.trk_vtx[a + i] = -1;
                A.trk_w[a + i] = 0.0f;
            }
        // the winning slot of every other track
        for (int k0 = 0; k0 < nl; k0 += G) {
            const int k = k0 + gid;
            const bool has = k < nl;
            const int beg = has ? S.base[k] : 0, ck = has ? S.cnt[k] : 0;
            const int vo = has ? S.vout[k] : -1;
            if (vo < 0)
                continue;
            const float dx = S.vf.dx[k], dy = S.vf.dy[k], dz = S.vf.dz[k];
            for (int t = gl; t < ck; t += L) {
                const int sl = beg + t;
                const int i = S.u.f.IDX[sl];
                if ((S.u.f.BEST[i] & 0xFFu) == 255u - (unsigned)vo) {
                    float chi2;
                    A.trk_vtx[a + i] = vo;
                    A.trk_w[a + i] = weight_at(sl, dx, dy, dz, chi2);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// one event
// ---------------------------------------------------------------------------
template <int W, int CAP, bool BIG, bool MV, bool DEBUG>
__device__ __forceinline__ void process_event(Smem<W, CAP, BIG, MV> &S, const KArgs &A, int e, int n_events)
{
    constexpr int NT = 64 * W;
    const KParams &p = A.p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    const int a = A.offsets[e], b = A.offsets[e + 1], total = A.offsets[n_events];
    const bool bad_offsets = (a < 0) || (b < a) || (b > total);
    const int n = bad_offsets ? 0 : b - a;
    if (bad_offsets || n > p.max_tracks) {
        if (!bad_offsets) {
            for (int i = tid; i < n; i += NT) {
                A.trk_vtx[a + i] = -1;
                A.trk_w[a + i] = 0.0f;
            }
        }
        if (DEBUG && A.dbg_hist)
            for (int j = tid; j < p.nb; j += NT)
                A.dbg_hist[(size_t)e * p.nb + j] = 0;
        if (tid == 0) {
            A.status_out[e] = bad_offsets ? PV_EV_OFFSETS_INVALID : PV_EV_TOO_MANY_TRACKS;
            A.nv_out[e] = 0;
            if (DEBUG && A.dbg_ncl)
                A.dbg_ncl[e] = 0;
        }
        __syncthreads();
        return;
    }
    if (!BIG && n > CAP) {
        if (tid == 0) {
            const unsigned int k = atomicAdd(&A.wq->n_big, 1u);
            A.wq->big[k] = e;
        }
        __syncthreads();
        return;
    }

    Stamps ts;
    stamp<DEBUG>(ts, 0);
    auto defer = [&]() __attribute__((always_inline)) {
        if (tid == 0) {
            const unsigned int k = atomicAdd(&A.wq->n_big, 1u);
            A.wq->big[k] = e;
        }
    };
    int *h = hist_lds(S);
    // the first chunk of tracks is requested before the clear, whose LDS
    // stores and barrier then overlap the global loads
    float cur[8];
    if (tid < n)
        load_track(A, a + tid, cur);
    // clear (large teams: the whole histogram; small teams clear their pages
    // once the touched words are known)
    if constexpr (BIG) {
        int4 *h4 = reinterpret_cast<int4 *>(S.u.hist);
        const int n4 = (p.nb + 3) >> 2;
        for (int i = tid; i < n4; i += NT)
            h4[i] = make_int4(0, 0, 0, 0);
    }
    if (tid == 0) {
        S.occ = 0ull;
        S.status = 0;
        S.done = 0;
    }
    __syncthreads();
    stamp<DEBUG>(ts, 1);

    // Kernel windows of up to kShortWindow bins are filled by their own lane;
    // wider ones (about 1.6 % of tracks at mu = 5) by the whole wavefront, one
    // track at a time, so no lane idles through another lane's long window.
    // `off` maps a window's bins to LDS (0 for the whole histogram).
    auto fill_chunk = [&](bool has, float zp, float rinv, Window w, int off) __attribute__((always_inline)) {
        const bool wide = has && (w.jh - w.jl) > kShortWindow;
        if (has && !wide)
            fill_short(h, off, w, zp, rinv, p);
        unsigned long long wm = __ballot(wide);
        while (wm) {
            const int src = __ffsll((long long)wm) - 1;
            wm &= wm - 1ull;
            const float zs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zp), src));
            const float rs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rinv), src));
            const int jl = __builtin_amdgcn_readlane(w.jl, src);
            const int jh = __builtin_amdgcn_readlane(w.jh, src);
            const int os = __builtin_amdgcn_readlane(off, src);
            for (int j = jl + lane; j < jh; j += 64) {
                const int d = code_at(j + 1, zs, rs, p) - code_at(j, zs, rs, p);
                if (d != 0)
                    atomicAdd(&h[j + os], d);
            }
        }
    };

    // project (+ fill for large teams).  All lanes run every chunk
    // (wavefront-wide steps above); the loads of the next chunk are issued
    // before this chunk is processed.  Small teams record each histogrammed
    // track's z_poca, 1 / (u0 sigma) and window for the fill pass.
    {
        float nxt[8];
        unsigned long long words = 0ull;
        for (int i0 = 0; i0 < n; i0 += NT) {
            const int i = i0 + tid;
            const bool valid = i < n;
            if (i + NT < n)
                load_track(A, a + i + NT, nxt);
            Proj r{0.0f, 0.0f, -1, 0};
            if (valid)
                r = project(cur[0], cur[1], cur[2], cur[3], cur[4], cur[5], cur[6], cur[7], p);
            bool has = false;
            float rinv = 0.0f;
            Window w{0, 0};
            if (r.fl & kTrHist) {
                const float sw = p.u0 * r.sg;
                rinv = 1.0f / sw;
                w = track_window(r.zp, sw, p);
                if (w.jh > w.jl) {
                    words |= window_words(w);
                    has = true;
                }
            }
            if constexpr (BIG)
                fill_chunk(has, r.zp, rinv, w, 0);
            if (valid) {
                if (r.fl & kTrNonfinite)
                    atomicOr(&S.status, PV_EV_NONFINITE_INPUT);
                S.tb[i] = (r.bin + 1) | (r.fl << 13);
                if constexpr (!BIG) {
                    S.u.pp.tz[i] = r.zp;
                    S.u.pp.tr[i] = rinv;
                    S.u.pp.tw[i] = has ? (w.jl | (w.jh << 16)) : 0;
                }
                if (DEBUG) {
                    const int g = a + i;
                    if (A.dbg_zp)
                        A.dbg_zp[g] = r.zp;
                    if (A.dbg_sg)
                        A.dbg_sg[g] = r.sg;
                    if (A.dbg_bin)
                        A.dbg_bin[g] = r.bin;
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                cur[q] = nxt[q];
        }
        // one OR per wavefront into the touched-word mask
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            words |= (unsigned long long)__shfl_xor((long long)words, off);
        if (lane == 0 && words)
            atomicOr(&S.occ, words);
    }
    __syncthreads();
    if constexpr (!BIG) {
        const unsigned long long occ = S.occ;
        const int npg = __popcll(occ);
        if (npg > kPages) {
            defer();
            return;
        }
        int4 *h4 = reinterpret_cast<int4 *>(S.u.pp.pg);
        for (int k = tid; k < npg * 16; k += NT)
            h4[k] = make_int4(0, 0, 0, 0);
        __syncthreads();
        // fill: each touched word's bins sit at one offset
        for (int i0 = 0; i0 < n; i0 += NT) {
            const int i = i0 + tid;
            float zp = 0.0f, rinv = 0.0f;
            Window w{0, 0};
            int off = 0;
            bool has = false;
            if (i < n) {
                const int tw = S.u.pp.tw[i];
                if (tw != 0) {
                    w = Window{tw & 0xFFFF, tw >> 16};
                    zp = S.u.pp.tz[i];
                    rinv = S.u.pp.tr[i];
                    off = page_off(occ, w.jl >> 6);
                    has = true;
                }
            }
            fill_chunk(has, zp, rinv, w, off);
        }
        __syncthreads();
    }
    if (DEBUG && A.dbg_hist) {
        const unsigned long long occ = S.occ;
        for (int j = tid; j < p.nb; j += NT)
            A.dbg_hist[(size_t)e * p.nb + j] = bin_value(S, occ, j);
    }
    // The gather reads each wavefront's range of tracks again; its first chunk
    // is requested now, so that the loads complete during the peak search and
    // the association.
    const int R = (((n + W - 1) / W) + 63) & ~63;
    const int r0 = wave * R, r1 = min(n, r0 + R);
    float gnext[8];
    if (r0 + lane < r1)
        load_track(A, a + r0 + lane, gnext);

    stamp<DEBUG>(ts, 2);
    // peaks and seeds
    if (wave == 0)
        peak_search(S, p);
    __syncthreads();
    if (!BIG && S.defer) {
        defer();
        return;
    }
    stamp<DEBUG>(ts, 3);

    int nl;
    if constexpr (!MV) {
        // association with iterative removal (Sec. 3.4)
        if (wave == 0) {
            for (int q = lane; q < S.n_cl; q += 64)
                S.live[q] = (short)q;
            if (lane == 0)
                S.n_live = S.n_cl;
        }
        __syncthreads();
        for (;;) {
            const int nl = S.n_live;
            if (wave == 0) {
                for (int k = lane; k < nl; k += 64) {
                    const int cq = S.live[k];
                    S.pb[k] = (k + 1 < nl) ? ((S.chi[cq] + S.clo[S.live[k + 1]]) >> 1) : p.nb - 1;
                    S.cnt[k] = 0;
                }
            }
            __syncthreads();
            for (int i = tid; i < n; i += NT) {
                const int t = S.tb[i];
                int own = -1;
                if (((t >> 13) & kTrAssoc) && nl > 0) {
                    own = lower_bound_bins(S.pb, nl, (t & 0x1FFF) - 1);
                    atomicAdd(&S.cnt[own], 1);
                }
                S.tb[i] = (t & 0xFFFF) | ((own + 1) << 16);
            }
            __syncthreads();
            if (wave == 0) {
                int key = INT_MAX;
                for (int k = lane; k < nl; k += 64) {
                    const int cq = S.live[k];
                    const int need = (S.cpk[cq] < p.gas_bin) ? p.part_min_gas : p.part_min_pp;
                    const int c = S.cnt[k];
                    if (c < need)
                        key = min(key, (c << 8) | k);
                }
                key = wave_min(key);
                if (key == INT_MAX) {
                    if (lane == 0)
                        S.done = 1;
                } else {
                    const int kv = key & 0xFF;
                    const int k0 = lane, k1 = lane + 64;
                    short v0 = 0, v1 = 0;
                    if (k0 < nl - 1)
                        v0 = S.live[k0 + (k0 >= kv ? 1 : 0)];
                    if (k1 < nl - 1)
                        v1 = S.live[k1 + (k1 >= kv ? 1 : 0)];
                    __builtin_amdgcn_wave_barrier();
                    if (k0 < nl - 1)
                        S.live[k0] = v0;
                    if (k1 < nl - 1)
                        S.live[k1] = v1;
                    if (lane == 0)
                        S.n_live = nl - 1;
                }
            }
            __syncthreads();
            if (S.done)
                break;
        }
        nl = S.n_live;
        stamp<DEBUG>(ts, 4);

        if (DEBUG && A.dbg_cl && wave == 0) {
            for (int q = lane; q < S.n_cl; q += 64)
                S.vout[q] = -1;
            __builtin_amdgcn_wave_barrier();
            for (int k = lane; k < nl; k += 64)
                S.vout[S.live[k]] = k;
            __builtin_amdgcn_wave_barrier();
            for (int q = lane; q < S.n_cl; q += 64) {
                const int k = S.vout[q];
                pv_cluster c;
                c.lo = S.clo[q];
                c.hi = S.chi[q];
                c.peak = S.cpk[q];
                c.z_seed = bin_centre(S.cpk[q], p) + S.cd0[q];
                c.kept = (k >= 0) ? 1 : 0;
                c.n_assoc = (k >= 0) ? S.cnt[k] : 0;
                c.own_lo = (k > 0) ? S.pb[k - 1] + 1 : (k == 0 ? 0 : -1);
                c.own_hi = (k >= 0) ? S.pb[k] : -1;
                A.dbg_cl[(size_t)e * p.max_vertices + q] = c;
            }
        }

        // gather tracks by vertex (stable, by track index)
        if (wave == 0) {
            const int c0 = (lane < nl) ? S.cnt[lane] : 0;
            const int c1 = (lane + 64 < nl) ? S.cnt[lane + 64] : 0;
            const int i0 = wave_incl_scan(c0, lane);
            const int t0 = __shfl(i0, 63);
            const int i1 = wave_incl_scan(c1, lane);
            if (lane < nl)
                S.base[lane] = i0 - c0;
            if (lane + 64 < nl)
                S.base[lane + 64] = t0 + i1 - c1;
        }
        if (W > 1) {
            for (int k = tid; k < W * Smem<W, CAP, BIG, MV>::V; k += NT)
                (&S.wrun[0][0])[k] = 0;
            __syncthreads();
            for (int i = r0 + lane; i < r1; i += 64) {
                const int own = (S.tb[i] >> 16) - 1;
                if (own >= 0)
                    atomicAdd(&S.wrun[wave][own], 1);
            }
            __syncthreads();
            for (int k = tid; k < nl; k += NT) {
                int run = S.base[k];
                for (int w = 0; w < W; ++w) {
                    const int t = S.wrun[w][k];
                    S.wrun[w][k] = run;
                    run += t;
                }
            }
            __syncthreads();
        } else {
            __syncthreads();
            for (int k = tid; k < nl; k += NT)
                S.wrun[0][k] = S.base[k];
            __syncthreads();
        }
        const int obits = (nl > 1) ? 32 - __clz(nl - 1) : 0;
        for (int c0 = r0; c0 < r1; c0 += 64) {
            const int i = c0 + lane;
            const bool valid = i < r1;
            const int own = valid ? (S.tb[i] >> 16) - 1 : -1;
            float t[8];
    #pragma unroll
            for (int q = 0; q < 8; ++q)
                t[q] = gnext[q];
            if (c0 + 64 + lane < r1)
                load_track(A, a + c0 + 64 + lane, gnext);
            // lanes with the same owner: one ballot per bit of the owner's
            // index, so the cost grows with log2 of the vertex count, not
            // with the number of owners present in the chunk
            unsigned long long mm = __ballot(own >= 0);
            for (int bit = 0; bit < obits; ++bit) {
                const bool set = (own >> bit) & 1;
                const unsigned long long bb = __ballot(set);
                mm &= set ? bb : ~bb;
            }
            int slot = -1;
            const unsigned long long below = mm & lanemask_lt(lane);
            if (own >= 0)
                slot = S.wrun[wave][own] + __popcll(below);
            __builtin_amdgcn_wave_barrier();
            if (own >= 0 && below == 0ull)
                S.wrun[wave][own] += __popcll(mm);
            __builtin_amdgcn_wave_barrier();
            if (valid) {
                const int g = a + i;
                if (slot >= 0) {
                    const float x = t[0], y = t[1], z = t[2], tx = t[3], ty = t[4];
                    const float vxx = t[5], vxtx = t[6], vtxtx = t[7];
                    // positions relative to the beamline point at the peak-bin centre
                    const int cq = S.live[own];
                    const float zr = bin_centre(S.cpk[cq], p);
                    const float dzr = zr - z;
                    S.u.f.X[slot] = fmaf(dzr, tx, x) - (p.bx + p.btx * zr);
                    S.u.f.Y[slot] = fmaf(dzr, ty, y) - (p.by + p.bty * zr);
                    S.u.f.TX[slot] = tx;
                    S.u.f.TY[slot] = ty;
                    // Eq. 2 at the seed: z_seed - z_trk = (z_i - z_trk) + delta dz
                    const float dzs = dzr + S.cd0[cq];
                    const float V = fmaf(dzs, fmaf(dzs, vtxtx, 2.0f * vxtx), vxx);
                    S.u.f.WT[slot] = (V > 0.0f && isfinite(V)) ? 1.0f / V : 0.0f;
                    S.u.f.IDX[slot] = (short)i;
                } else {
                    A.trk_vtx[g] = -1;
                    A.trk_w[g] = 0.0f;
                }
            }
        }
    } else {
        // Multi-vertex (Sec. 3.5, Sec. 5): every cluster is a candidate and
        // fits the tracks passing its pre-cut; one slot per (candidate, track)
        // pair, by candidate and, within one, by track index (each wavefront
        // takes its contiguous range of tracks, ranks within a chunk by
        // ballot), so the sums are reproducible.
        if (wave == 0) {
            for (int q = lane; q < S.n_cl; q += 64)
                S.live[q] = (short)q;
            if (lane == 0)
                S.n_live = S.n_cl;
        }
        for (int k = tid; k < W * Smem<W, CAP, BIG, MV>::V; k += NT)
            (&S.wrun[0][0])[k] = 0;
        __syncthreads();
        nl = S.n_live;
        stamp<DEBUG>(ts, 4);
        // With many candidates (high pile-up) each wavefront takes its tracks
        // in z order, 64 at a time, and skips the candidates whose seed lies
        // outside the union of the chunk's pre-cut ranges (mv_window): those
        // pairs fail the cut by a wide margin, so the lists are the same as
        // with every candidate tried.  The order comes from a stable counting
        // sort on 4 mm buckets of the central bin; sorted position j holds its
        // track index in the upper half of tb[j] (free in this variant).
        // Lists are then ordered by candidate and, within one, by that order.
        bool zsort = false;
        if (nl >= kMvSortMin) {
            // the candidates' seeds (C_zz's array is free until the counting
            // pass), in z order as the peak search emits them, so that a chunk
            // finds its candidates by two ballots; were they not in order, the
            // event would take the plain pre-cut
            if (wave == 0) {
                bool ordered = true;
                for (int k = lane; k < nl; k += 64) {
                    const float zk = bin_centre(S.cpk[k], p) + S.cd0[k];
                    S.czz[k] = zk;
                    if (k > 0)
                        ordered = ordered && (bin_centre(S.cpk[k - 1], p) + S.cd0[k - 1] <= zk);
                }
                const bool all = __ballot(!ordered) == 0ull;
                if (lane == 0)
                    S.zord = all ? 1 : 0;
            }
            __syncthreads();
            zsort = S.zord != 0;
        }
        if (zsort) {
            static_assert(sizeof(S.u) >= sizeof(int) * W * 256, "bucket counters must fit the track arrays");
            int *cw = reinterpret_cast<int *>(&S.u);   // [W][256] bucket counters; dead since the peak search
            auto key_of = [&](int i) __attribute__((always_inline)) {
                const int bin = (S.tb[i] & 0x1FFF) - 1;
                return bin < 0 ? 255 : min(bin >> 4, 254);
            };
            for (int k = tid; k < W * 256; k += NT)
                cw[k] = 0;
            __syncthreads();
            for (int i = r0 + lane; i < r1; i += 64)
                atomicAdd(&cw[wave * 256 + key_of(i)], 1);
            __syncthreads();
            if (wave == 0) {
                int run = 0;
                for (int b0 = 0; b0 < 256; b0 += 64) {
                    const int b = b0 + lane;
                    int c = 0;
                    for (int w = 0; w < W; ++w)
                        c += cw[w * 256 + b];
                    const int incl = wave_incl_scan(c, lane);
                    int r = run + incl - c;
                    for (int w = 0; w < W; ++w) {
                        const int cwb = cw[w * 256 + b];
                        cw[w * 256 + b] = r;
                        r += cwb;
                    }
                    run += __shfl(incl, 63);
                }
            }
            __syncthreads();
            for (int c0 = r0; c0 < r1; c0 += 64) {
                const int i = c0 + lane;
                const bool valid = i < r1;
                const int key = valid ? key_of(i) : 0;
                // lanes with the same key: one ballot per key bit
                unsigned long long mm = __ballot(valid);
                for (int bit = 0; bit < 8; ++bit) {
                    const bool set = (key >> bit) & 1;
                    const unsigned long long bb = __ballot(set);
                    mm &= set ? bb : ~bb;
                }
                const unsigned long long below = mm & lanemask_lt(lane);
                const int pos = valid ? cw[wave * 256 + key] + __popcll(below) : 0;
                __builtin_amdgcn_wave_barrier();
                if (valid && below == 0ull)
                    cw[wave * 256 + key] += __popcll(mm);
                __builtin_amdgcn_wave_barrier();
                if (valid)
                    atomicOr(&S.tb[pos], i << 16);
            }
            __syncthreads();
        }
        // the chunk of (sorted) positions c0 .. c0 + 63 of this wavefront: its
        // tracks, their indices and, sorted (ZS), the candidates [k_lo, k_hi)
        // whose seeds lie in the union of their pre-cut ranges.  The passes
        // below are compiled for both orders, so that without the z order
        // their loops stay those of the plain pre-cut.
        auto chunk_tracks = [&](auto zs, int c0, float t[8], int &i, bool &assoc, float &zlo, float &zhi, int &k_lo,
                                int &k_hi) __attribute__((always_inline)) {
            constexpr bool ZS = decltype(zs)::value;
            const int j = c0 + lane;
            k_lo = 0;
            k_hi = nl;
            if constexpr (!ZS) {
                i = (j < r1) ? j : -1;
                if (c0 == r0) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        t[q] = gnext[q];
                } else if (i >= 0) {
                    load_track(A, a + i, t);
                }
                assoc = i >= 0 && ((S.tb[i] >> 13) & kTrAssoc);
            } else {
                i = (j < r1) ? (S.tb[j] >> 16) : -1;
                if (i >= 0)
                    load_track(A, a + i, t);
                assoc = i >= 0 && ((S.tb[i] >> 13) & kTrAssoc);
                float lo = INFINITY, hi = -INFINITY;
                if (assoc)
                    mv_window(t, p, lo, hi);
                zlo = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_min_f(lo))));
                zhi = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_max_f(hi))));
                // seeds in order: the candidates below zlo, then those up to zhi
                int below = 0, upto = 0;
                for (int k0 = 0; k0 < nl; k0 += 64) {
                    const int k = k0 + lane;
                    const float zk = (k < nl) ? S.czz[k] : INFINITY;
                    below += __popcll(__ballot(zk < zlo));
                    upto += __popcll(__ballot(zk <= zhi));
                }
                k_lo = __builtin_amdgcn_readfirstlane(below);
                k_hi = __builtin_amdgcn_readfirstlane(upto);
            }
        };
        // pass 1: per wavefront and candidate, the tracks passing the pre-cut,
        // and per track the sum of its terms of Eq. 18 (kept in the per-track
        // key array, unused until the final pass)
        auto pass1 = [&](auto zs) __attribute__((always_inline)) {
            for (int c0 = r0; c0 < r1; c0 += 64) {
                float t[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                int i, k_lo, k_hi;
                bool assoc;
                float zlo = -INFINITY, zhi = INFINITY;
                chunk_tracks(zs, c0, t, i, assoc, zlo, zhi, k_lo, k_hi);
                float esum = 0.0f;
                for (int k = k_lo; k < k_hi; ++k) {
                    const MvPre m = mv_precut(t, bin_centre(S.cpk[k], p), S.cd0[k], p);
                    const bool pass = assoc && m.WT > 0.0f && m.chi2 < p.chi2_window_mv;
                    if (pass)
                        esum += __expf(-0.5f * m.chi2);
                    const unsigned long long mm = __ballot(pass);
                    if (lane == 0)
                        S.wrun[wave][k] += __popcll(mm);
                }
                if (i >= 0)
                    S.u.f.BEST[i] = __float_as_uint(esum);
            }
        };
        if (zsort)
            pass1(std::true_type{});
        else
            pass1(std::false_type{});
        __syncthreads();
        // list lengths, starts and each wavefront's first slot per candidate
        if (wave == 0) {
            int run = 0;
            for (int k0 = 0; k0 < nl; k0 += 64) {
                const int k = k0 + lane;
                int c = 0;
                if (k < nl)
                    for (int w = 0; w < W; ++w)
                        c += S.wrun[w][k];
                const int incl = wave_incl_scan(c, lane);
                if (k < nl) {
                    S.cnt[k] = c;
                    S.base[k] = run + incl - c;
                    int r = run + incl - c;
                    for (int w = 0; w < W; ++w) {
                        const int tw = S.wrun[w][k];
                        S.wrun[w][k] = r;
                        r += tw;
                    }
                }
                run += __shfl(incl, 63);
            }
            if (lane == 0) {
                S.n_slots = run;
                // the lists share the event's track capacity (else the event is
                // flagged), and must fit the team's slots (else deferred)
                if (run > p.max_tracks)
                    S.status |= PV_EV_TOO_MANY_TRACKS;
                else if (!BIG && run > CAP)
                    S.defer = 1;
            }
        }
        __syncthreads();
        if (!BIG && S.defer) {
            defer();
            return;
        }
        if (S.n_slots > p.max_tracks) {
            for (int i = tid; i < n; i += NT) {
                A.trk_vtx[a + i] = -1;
                A.trk_w[a + i] = 0.0f;
            }
            if (tid == 0) {
                A.nv_out[e] = 0;
                A.status_out[e] = S.status;
                if (DEBUG && A.dbg_ncl)
                    A.dbg_ncl[e] = S.n_cl;
            }
            if (DEBUG && A.dbg_cl && wave == 0)
                for (int q = lane; q < S.n_cl; q += 64) {
                    pv_cluster c;
                    c.lo = S.clo[q];
                    c.hi = S.chi[q];
                    c.peak = S.cpk[q];
                    c.z_seed = bin_centre(S.cpk[q], p) + S.cd0[q];
                    c.kept = 1;
                    c.n_assoc = S.cnt[q];
                    c.own_lo = c.own_hi = -1;
                    A.dbg_cl[(size_t)e * p.max_vertices + q] = c;
                }
            __syncthreads();
            return;
        }
        // pass 2: write the slots; the other candidates' terms of Eq. 18 are
        // the track's sum over its pre-cut passes minus this candidate's
        auto pass2 = [&](auto zs) __attribute__((always_inline)) {
            for (int c0 = r0; c0 < r1; c0 += 64) {
                float t[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                int i, k_lo, k_hi;
                bool assoc;
                float zlo = -INFINITY, zhi = INFINITY;
                chunk_tracks(zs, c0, t, i, assoc, zlo, zhi, k_lo, k_hi);
                float esum = 0.0f;
                if (i >= 0) {
                    esum = __uint_as_float(S.u.f.BEST[i]);
                    S.u.f.BEST[i] = 0u;
                }
                for (int k = k_lo; k < k_hi; ++k) {
                    const MvPre m = mv_precut(t, bin_centre(S.cpk[k], p), S.cd0[k], p);
                    const bool pass = assoc && m.WT > 0.0f && m.chi2 < p.chi2_window_mv;
                    const unsigned long long mm = __ballot(pass);
                    if (pass) {
                        const int slot = S.wrun[wave][k] + __popcll(mm & lanemask_lt(lane));
                        S.u.f.X[slot] = m.X;
                        S.u.f.Y[slot] = m.Y;
                        S.u.f.TX[slot] = t[3];
                        S.u.f.TY[slot] = t[4];
                        S.u.f.WT[slot] = m.WT;
                        S.u.f.OTH[slot] = fmaxf(esum - __expf(-0.5f * m.chi2), 0.0f);
                        S.u.f.IDX[slot] = (short)i;
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (lane == 0)
                        S.wrun[wave][k] += __popcll(mm);
                    __builtin_amdgcn_wave_barrier();
                }
            }
        };
        if (zsort)
            pass2(std::true_type{});
        else
            pass2(std::false_type{});
        if (DEBUG && A.dbg_cl && wave == 0)
            for (int q = lane; q < S.n_cl; q += 64) {
                pv_cluster c;
                c.lo = S.clo[q];
                c.hi = S.chi[q];
                c.peak = S.cpk[q];
                c.z_seed = bin_centre(S.cpk[q], p) + S.cd0[q];
                c.kept = 1;
                c.n_assoc = S.cnt[q];
                c.own_lo = c.own_hi = -1;
                A.dbg_cl[(size_t)e * p.max_vertices + q] = c;
            }
    }
    __syncthreads();
    stamp<DEBUG>(ts, 5);

    // fit (Sec. 3.5): L lanes per vertex, L the largest power of two with
    // L * vertices <= 64 for small teams with at most 8 vertices (one
    // wavefront fits them all and the others skip the fit: fewer instructions
    // per event than spreading the vertices over the team, whose narrower
    // groups need deeper sums, and the other teams on the CU use the freed
    // issue slots), <= the team's lanes otherwise (many vertices, or one
    // large-event team per CU, where latency decides)
    int lg = 6;
    {
        const int target = ((!BIG && nl <= 8) ? 64 : NT) / max(nl, 1);
        while (lg > 0 && (1 << lg) > target)
            --lg;
    }
    lg = __builtin_amdgcn_readfirstlane(lg);   // the same on every lane: keep it scalar
    const int L = 1 << lg;
    // Fits spread over the team (more than 8 vertices) give vertex k 2^lk
    // lanes, about in proportion to its tracks (a wavefront iterates until its
    // slowest vertex converges, so with equal groups the largest vertex would
    // set the pace): lk = floor(log2(c_k B / C)) for the team's B lanes and C
    // tracks in all (at least one; if those minimums overrun the budget, the
    // blocks that lose least are halved until they fit), then the vertex with
    // the most tracks per lane doubles its lanes while the budget allows.  The blocks are placed largest first, so
    // each is aligned to its size, as the group sums need.  Fewer vertices,
    // where the balancing costs more than it saves, and more than 64 keep L
    // lanes each.
    const bool prop = nl > 8 && nl <= 64;
    if (prop && wave == 0) {
        const int budget = NT;
        int lk = lg, off = lane << lg, used = 0;
        bool fits = false;
        {
            const int c = (lane < nl) ? S.cnt[lane] : 0;
            const int C = __shfl(wave_incl_scan(c, lane), 63);
            if (C > 0) {
                const int q = (lane < nl) ? max(1, (c * budget) / C) : 1;
                int lp = min(6, 31 - __clz(q));
                int tot = __shfl(wave_incl_scan((lane < nl) ? (1 << lp) : 0, lane), 63);
                // many small vertices beside a large one take more than the
                // budget at one lane each: halve the block that loses least
                // (fewest tracks per lane after halving) until they fit
                for (int it = 0; it < 64 && tot > budget; ++it) {
                    const int r = (lane < nl && lp > 0) ? ((c + (1 << (lp - 1)) - 1) >> (lp - 1)) : 0x7FFFFF;
                    const int key = wave_min((r << 8) | lane);
                    if ((key >> 8) == 0x7FFFFF)
                        break;
                    const int kb = key & 0xFF;
                    const int lb = __shfl(lp, kb);
                    if (lane == kb)
                        --lp;
                    tot -= 1 << (lb - 1);
                }
                if (tot <= budget) {
                    fits = true;
                    for (int it = 0; it < 64; ++it) {
                        // worst tracks per lane, lowest index on ties
                        const int r = (lane < nl) ? ((c + (1 << lp) - 1) >> lp) : 0;
                        const int key = -wave_min(-((r << 8) | (255 - lane)));
                        const int kb = 255 - (key & 0xFF);
                        const int lb = __shfl(lp, kb);
                        if ((key >> 8) <= 1 || lb >= 6 || tot + (1 << lb) > budget)
                            break;
                        if (lane == kb)
                            ++lp;
                        tot += 1 << lb;
                    }
                    lk = lp;
                    used = tot;
                    int run = 0;
                    for (int cl = 6; cl >= 0; --cl) {
                        const bool mine = lane < nl && lk == cl;
                        const unsigned long long mm = __ballot(mine);
                        if (mine)
                            off = run + (__popcll(mm & lanemask_lt(lane)) << cl);
                        run += __popcll(mm) << cl;
                    }
                }
            }
        }
        if (fits) {
            for (int t = used + lane; t < NT; t += 64)
                S.lmap[t] = -1;
            if (lane < nl)
                for (int u = 0; u < (1 << lk); ++u)
                    S.lmap[off + u] = (short)(lane | (lk << 8));
        } else {
            for (int t = lane; t < NT; t += 64) {
                const int kk = t >> lg;
                S.lmap[t] = (kk < nl) ? (short)(kk | (lg << 8)) : (short)-1;
            }
        }
    }
    if (prop)
        __syncthreads();
    fit_vertices<W, CAP, BIG, MV>(S, p, nl, lg, prop);
    __syncthreads();
    stamp<DEBUG>(ts, 6);

    if constexpr (!MV) {
        // final selection (Table 2, end of Sec. 3.5)
        if (wave == 0) {
            int kept = 0;
            for (int k0 = 0; k0 < nl; k0 += 64) {
                const int k = k0 + lane;
                bool keep = false;
                if (k < nl) {
                    const int cq = S.live[k];
                    const bool gas = S.cpk[cq] < p.gas_bin;
                    keep = !(S.vf.info[k] & kInfoFailed) && S.cnt[k] >= (gas ? p.pv_min_gas : p.pv_min_pp);
                    if (keep && !gas) {
                        const float zr = bin_centre(S.cpk[cq], p);
                        const float zv = zr + S.vf.dz[k];
                        const float xv = (p.bx + p.btx * zr) + S.vf.dx[k];
                        const float yv = (p.by + p.bty * zr) + S.vf.dy[k];
                        const float rx = xv - (p.bx + p.btx * zv);
                        const float ry = yv - (p.by + p.bty * zv);
                        keep = fmaf(rx, rx, ry * ry) <= p.max_rho2_pp;
                    }
                }
                const unsigned long long km = __ballot(keep);
                if (k < nl)
                    S.vout[k] = keep ? kept + __popcll(km & lanemask_lt(lane)) : -1;
                kept += __popcll(km);
            }
            if (lane == 0)
                S.n_keep = kept;
        }
    } else {
        // Multi-vertex: track counts (final weight >= w_count_mv) and C_zz of
        // every candidate, then duplicates and the selection of Table 2
        {
            const int G = NT >> lg;
            const int gid = tid >> lg, gl = tid & (L - 1);
            for (int k0 = 0; k0 < nl; k0 += G) {
                const int k = k0 + gid;
                const bool has = k < nl;
                const int beg = has ? S.base[k] : 0, ck = has ? S.cnt[k] : 0;
                const float dx = has ? S.vf.dx[k] : 0.0f, dy = has ? S.vf.dy[k] : 0.0f, dz = has ? S.vf.dz[k] : 0.0f;
                float c = 0.0f;
                for (int t = gl; t < ck; t += L) {
                    const int sl = beg + t;
                    const float rx = fmaf(dz, S.u.f.TX[sl], S.u.f.X[sl]) - dx;
                    const float ry = fmaf(dz, S.u.f.TY[sl], S.u.f.Y[sl]) - dy;
                    const float chi2 = S.u.f.WT[sl] * fmaf(rx, rx, ry * ry);
                    const float w = mv_weight(chi2, S.u.f.OTH[sl], p);
                    c += (w >= p.w_count_mv) ? 1.0f : 0.0f;
                    // the final pass reads the final weight and chi2 back
                    S.u.f.OTH[sl] = w;
                    S.u.f.X[sl] = chi2;
                }
                c = group_sum_rt(c, L);
                if (has && gl == 0) {
                    S.ntk[k] = (int)c;
                    float cf[6];
                    vertex_covariance(S.vf.a[k], S.vf.b[k], S.vf.c[k], S.vf.d[k], S.vf.tx[k], S.vf.ty[k],
                                      p.cond_fp64, cf);
                    S.czz[k] = cf[5];
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
            constexpr int KPL = (Smem<W, CAP, BIG, MV>::V + 63) / 64;   // candidates per lane
            bool ok[KPL], kept[KPL];
            int nk[KPL], rank[KPL];
            float zk[KPL], cz[KPL];
            // dm[u][w], in the lane of candidate c = lane + 64 u: bit j set when
            // c is a duplicate of candidate j + 64 w
            unsigned long long dm[KPL][KPL];
            int n_ok = 0;
#pragma unroll
            for (int u = 0; u < KPL; ++u) {
                const int k = lane + 64 * u;
                ok[u] = k < nl && !(S.vf.info[k] & kInfoFailed);
                zk[u] = ok[u] ? bin_centre(S.cpk[S.live[k]], p) + S.vf.dz[k] : 0.0f;
                cz[u] = ok[u] ? S.czz[k] : 0.0f;
                nk[u] = ok[u] ? S.ntk[k] : 0;
                rank[u] = 0;
#pragma unroll
                for (int w = 0; w < KPL; ++w)
                    dm[u][w] = 0ull;
                n_ok += __popcll(__ballot(ok[u]));
            }
            // One candidate q at a time, broadcast from its lane: the ranks
            // (more counted tracks first, then the lower index) and the row of
            // candidates q is a duplicate of, which q's lane keeps.
#pragma unroll
            for (int uq = 0; uq < KPL; ++uq) {
                const int lim = min(64, nl - 64 * uq);
                for (int lq = 0; lq < lim; ++lq) {
                    if (!__builtin_amdgcn_readlane((int)ok[uq], lq))
                        continue;
                    const int q = 64 * uq + lq;
                    const int nq = __builtin_amdgcn_readlane(nk[uq], lq);
                    const float zq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zk[uq]), lq));
                    const float cq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cz[uq]), lq));
#pragma unroll
                    for (int u = 0; u < KPL; ++u) {
                        const int k = lane + 64 * u;
                        const bool other = ok[u] && q != k;
                        rank[u] += (other && (nq > nk[u] || (nq == nk[u] && q < k))) ? 1 : 0;
                        const float d = zq - zk[u];
                        const unsigned long long row = __ballot(other && d * d < p.dup_ratio * (cq + cz[u]));
                        if (lane == lq)
                            dm[uq][u] = row;
                    }
                }
            }
            // by rank: kept unless a duplicate of one kept before it
            unsigned long long km[KPL];
#pragma unroll
            for (int w = 0; w < KPL; ++w)
                km[w] = 0ull;
            for (int r = 0; r < n_ok; ++r) {
                int src = 0, su = 0;
#pragma unroll
                for (int u = 0; u < KPL; ++u) {
                    const unsigned long long hm = __ballot(ok[u] && rank[u] == r);
                    if (hm) {
                        src = __ffsll((long long)hm) - 1;
                        su = u;
                    }
                }
                bool dup = false;
#pragma unroll
                for (int w = 0; w < KPL; ++w) {
                    unsigned long long row = 0ull;
#pragma unroll
                    for (int u = 0; u < KPL; ++u)
                        if (u == su)
                            row = readlane_u64(dm[u][w], src);
                    dup = dup || (row & km[w]) != 0ull;
                }
                if (!dup) {
#pragma unroll
                    for (int u = 0; u < KPL; ++u)
                        if (u == su)
                            km[u] |= 1ull << src;
                }
            }
#pragma unroll
            for (int u = 0; u < KPL; ++u)
                kept[u] = ((km[u] >> lane) & 1ull) != 0ull;
            int kept_n = 0;
#pragma unroll
            for (int u = 0; u < KPL; ++u) {
                const int k = lane + 64 * u;
                bool keep = false;
                if (kept[u]) {
                    const int cq = S.live[k];
                    const bool gas = S.cpk[cq] < p.gas_bin;
                    keep = S.ntk[k] >= (gas ? p.pv_min_gas : p.pv_min_pp);
                    if (keep && !gas) {
                        const float zr = bin_centre(S.cpk[cq], p);
                        const float zv = zr + S.vf.dz[k];
                        const float xv = (p.bx + p.btx * zr) + S.vf.dx[k];
                        const float yv = (p.by + p.bty * zr) + S.vf.dy[k];
                        const float rx = xv - (p.bx + p.btx * zv);
                        const float ry = yv - (p.by + p.bty * zv);
                        keep = fmaf(rx, rx, ry * ry) <= p.max_rho2_pp;
                    }
                }
                const unsigned long long km = __ballot(keep);
                if (k < nl)
                    S.vout[k] = keep ? kept_n + __popcll(km & lanemask_lt(lane)) : -1;
                kept_n += __popcll(km);
            }
            if (lane == 0)
                S.n_keep = kept_n;
        }
    }
    __syncthreads();
    stamp<DEBUG>(ts, 7);

    // final weights, vertex records
    final_pass<W, CAP, BIG, MV>(S, A, e, a, n, nl, L, lg);
    if (tid == 0) {
        A.nv_out[e] = S.n_keep;
        A.status_out[e] = S.status;
        if (DEBUG && A.dbg_ncl)
            A.dbg_ncl[e] = S.n_cl;
    }
    __syncthreads();
    stamp<DEBUG>(ts, 8);
    if (DEBUG && A.dbg_cycles && tid == 0)
        for (int k = 0; k < 8; ++k)
            A.dbg_cycles[(size_t)e * 8 + k] = (uint32_t)(ts.t[k + 1] - ts.t[k]);
}

// Large events: a persistent grid, one eight-wavefront team per CU, drains the
// list of events the small teams deferred.
template <bool MV, bool DEBUG>
__global__ __launch_bounds__(64 * kBigWaves) void pv_find_large(KArgs A)
{
    __shared__ Smem<kBigWaves, kBigCapacity, true, MV> S;
    const int tid = threadIdx.x;
    const int n_events = A.n_events_dev ? *A.n_events_dev : A.n_events;
    // Nothing deferred: the counters are all zero and stay so; leave without
    // touching them (n_big is not written while this grid runs, so every
    // workgroup sees the same value).
    if (__hip_atomic_load(&A.wq->n_big, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
        return;
    for (;;) {
        if (tid == 0) {
            int e = -1;
            const unsigned int k = atomicAdd(&A.wq->next_big, 1u);
            const unsigned int nbig = atomicAdd(&A.wq->n_big, 0u);
            if (k < nbig)
                e = A.wq->big[k];
            S.ev = e;
        }
        __syncthreads();
        const int e = S.ev;
        __syncthreads();
        if (e < 0)
            break;
        process_event<kBigWaves, kBigCapacity, true, MV, DEBUG>(S, A, e, n_events);
    }
    if (tid == 0) {
        __threadfence();
        const unsigned int prev = atomicAdd(&A.wq->done_big, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(&A.wq->next_big, 0u);
            atomicExch(&A.wq->n_big, 0u);
            atomicExch(&A.wq->done_big, 0u);
            __threadfence();
        }
    }
}

// One small team per event, hardware-scheduled (grid = events, or the batch
// capacity when the count is read from device memory).  Without a persistent
// loop no value has to live from one event to the next, which keeps the
// register footprint low.
// Wavefronts per SIMD that the teams fitting a CU by LDS give, at most 6: the
// register budget the compiler is held to (the second launch bound).
template <int W, int CAP, bool MV>
constexpr int small_waves_per_simd()
{
    constexpr int teams = (160 * 1024) / (int)sizeof(Smem<W, CAP, false, MV>);
    constexpr int waves = teams * W / 4;
    return waves < 1 ? 1 : (waves > 6 ? 6 : waves);
}

template <int W, int CAP, bool MV, bool DEBUG>
__global__ __launch_bounds__(64 * W, (small_waves_per_simd<W, CAP, MV>())) void pv_find_single(KArgs A)
{
    __shared__ Smem<W, CAP, false, MV> S;
    const int n_events = A.n_events_dev ? *A.n_events_dev : A.n_events;
    if ((int)blockIdx.x >= n_events)
        return;
    const int e = A.order ? A.order[blockIdx.x] : (int)blockIdx.x;
    process_event<W, CAP, false, MV, DEBUG>(S, A, e, n_events);
}

// ---------------------------------------------------------------------------
// Processing order of the sorted mode: events by decreasing track count
// (16-track buckets, the last open-ended), so that the largest events start
// first and the launch does not end on a long one.  The batch is cut into
// G = ceil(n / 1024) slices of near-equal length (the first n mod G of them
// one event longer); workgroup s counting-sorts slice s in LDS, one event per
// thread, and puts its event of rank r at position r G + s.  These positions
// are a permutation of [0, n): the r-th largest events of all slices sit side
// by side, so the order is largest first up to the spread between slices, and
// no workgroup depends on another.  The order within a bucket is unspecified,
// which the results do not depend on.  Events with invalid offsets go last.
// ---------------------------------------------------------------------------
constexpr int kOrderBuckets = 256;
constexpr int kOrderSlice = 1024;   // most events of one slice (one per thread)

__global__ __launch_bounds__(kOrderSlice) void order_events_kernel(const int32_t *offsets,
                                                                   const int32_t *n_events_dev,
                                                                   int32_t n_events_host, int32_t *order)
{
    __shared__ int cnt[kOrderBuckets];
    const int tid = threadIdx.x;
    const int n_events = n_events_dev ? *n_events_dev : n_events_host;
    const int G = (n_events + kOrderSlice - 1) / kOrderSlice;
    const int sl = blockIdx.x;
    if (sl >= G)   // graph replays launch the grid of the capacity
        return;
    const int L = n_events / G, rem = n_events % G;
    const int first = sl * L + min(sl, rem), len = L + (sl < rem ? 1 : 0);
    // the offset loads are issued before the counters are cleared
    const int total = offsets[n_events];
    int a = 0, b = 0;
    if (tid < len) {
        a = offsets[first + tid];
        b = offsets[first + tid + 1];
    }
    for (int k = tid; k < kOrderBuckets; k += blockDim.x)
        cnt[k] = 0;
    __syncthreads();
    const int bk = (tid >= len) ? -1 : ((a < 0 || b < a || b > total) ? 0 : min((b - a) >> 4, kOrderBuckets - 1));
    if (bk >= 0)
        atomicAdd(&cnt[bk], 1);
    __syncthreads();
    // exclusive prefix over the buckets, largest first: one wavefront
    if (tid < 64) {
        const int lane = tid;
        int run = 0;
        for (int k0 = kOrderBuckets - 64; k0 >= 0; k0 -= 64) {
            const int k = k0 + 63 - lane;   // lane 0 takes the largest bucket of the chunk
            const int c = cnt[k];
            const int incl = wave_incl_scan(c, lane);
            cnt[k] = run + incl - c;
            run += __shfl(incl, 63);
        }
    }
    __syncthreads();
    if (bk >= 0)
        order[atomicAdd(&cnt[bk], 1) * G + sl] = first + tid;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int device_cus()
{
    // per thread: the server's worker thread and callers may launch concurrently
    static thread_local int cached_dev = -1, cached_cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    if (dev != cached_dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached_dev = dev;
        cached_cus = cus;
    }
    return cached_cus;
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free entry point (pv_find_noalloc): one
// file-scope device array per device, holding the work-queue header, the
// deferred-event list and the event order for up to PV_NOALLOC_MAX_EVENTS
// events.  On the host the array's name is not a device address: host code
// uses only the address hipGetSymbolAddress returns for the current device,
// looked up once per device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = offsetof(WorkQueue, big) + 2 * sizeof(int32_t) * (size_t)PV_NOALLOC_MAX_EVENTS;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

int noalloc_workspace(WorkQueue **wq, int32_t **order)
{
    static std::mutex mu;
    static std::map<int, void *> addr;   // device -> address of its copy of `scratch`
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return (int)err;
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = addr.find(dev);
        if (it == addr.end()) {
            err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (err != hipSuccess)
                return (int)err;
            addr.emplace(dev, ptr);
        } else {
            ptr = it->second;
        }
    }
    *wq = static_cast<WorkQueue *>(ptr);
    *order = order_list(*wq, PV_NOALLOC_MAX_EVENTS);
    return (int)hipSuccess;
}

// the work-queue counters start every allocation-free call at zero (a kernel
// rather than a memset, so that the call may be captured in a graph)
__global__ void clear_queue_kernel(WorkQueue *wq)
{
    if (threadIdx.x < offsetof(WorkQueue, big) / sizeof(unsigned int))
        reinterpret_cast<unsigned int *>(wq)[threadIdx.x] = 0u;
}

int clear_queue(WorkQueue *wq, void *stream)
{
    hipLaunchKernelGGL(clear_queue_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), wq);
    return (int)hipGetLastError();
}

template <int W, int CAP, bool MV, bool DEBUG>
static hipError_t launch_small(const KArgs &A, hipStream_t st)
{
    if (A.n_events < 1)
        return hipSuccess;
    hipLaunchKernelGGL((pv_find_single<W, CAP, MV, DEBUG>), dim3(A.n_events), dim3(64 * W), 0, st, A);
    return hipGetLastError();
}

template <bool MV, bool DEBUG>
static hipError_t launch_large(const KArgs &A, hipStream_t st)
{
    auto *fn = pv_find_large<MV, DEBUG>;
    int occ = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * kBigWaves, 0);
    if (err != hipSuccess)
        return err;
    if (occ < 1)
        occ = 1;
    const int cus = device_cus();
    const int grid = occ * (cus > 0 ? cus : 256);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * kBigWaves), 0, st, A);
    return hipGetLastError();
}

static hipError_t record(void *ev, hipStream_t st)
{
    return ev ? hipEventRecord(reinterpret_cast<hipEvent_t>(ev), st) : hipSuccess;
}

template <int W, int CAP, bool MV, bool DEBUG>
static hipError_t launch_pair(const KArgs &args, hipStream_t st, LaunchEvents *ev)
{
    KArgs A = args;
    if (!A.n_events_dev && A.n_events < 2)
        A.order = nullptr;   // nothing to order
    hipError_t err = hipSuccess;
    if (A.order) {
        // one workgroup per slice of at most kOrderSlice events (of the
        // capacity when the batch size is read from device memory)
        const int slices = (A.n_events + kOrderSlice - 1) / kOrderSlice;
        hipLaunchKernelGGL(order_events_kernel, dim3(slices), dim3(kOrderSlice), 0, st, A.offsets, A.n_events_dev,
                           A.n_events, A.order);
        err = hipGetLastError();
    }
    // the main-kernel timing brackets the fused launch alone
    if (err == hipSuccess)
        err = record(ev ? ev->main_begin : nullptr, st);
    if (err == hipSuccess)
        err = launch_small<W, CAP, MV, DEBUG>(A, st);
    if (err == hipSuccess)
        err = record(ev ? ev->main_end : nullptr, st);
    if (err != hipSuccess)
        return err;
    // events with more tracks than CAP, more touched histogram words than the
    // pages, more clusters than the vertex slots or (multi-vertex) longer
    // candidate track lists than a small team holds were deferred to the
    // large-team launch (which returns at once if none was)
    if (ev)
        ev->large = true;
    err = record(ev ? ev->large_begin : nullptr, st);
    if (err == hipSuccess)
        err = launch_large<MV, DEBUG>(A, st);
    if (err == hipSuccess)
        err = record(ev ? ev->large_end : nullptr, st);
    return err;
}

template <bool MV, bool DEBUG>
static hipError_t launch_dispatch(const KArgs &A, const pv_schedule &s, hipStream_t st, LaunchEvents *ev)
{
    switch (s.waves_per_team * 10000 + s.track_capacity) {
    case 10256: return launch_pair<1, 256, MV, DEBUG>(A, st, ev);
    case 10512: return launch_pair<1, 512, MV, DEBUG>(A, st, ev);
    case 11024: return launch_pair<1, 1024, MV, DEBUG>(A, st, ev);
    case 11536: return launch_pair<1, 1536, MV, DEBUG>(A, st, ev);
    case 12048: return launch_pair<1, 2048, MV, DEBUG>(A, st, ev);
    case 20256: return launch_pair<2, 256, MV, DEBUG>(A, st, ev);
    case 20512: return launch_pair<2, 512, MV, DEBUG>(A, st, ev);
    case 21024: return launch_pair<2, 1024, MV, DEBUG>(A, st, ev);
    case 21536: return launch_pair<2, 1536, MV, DEBUG>(A, st, ev);
    case 22048: return launch_pair<2, 2048, MV, DEBUG>(A, st, ev);
    case 40256: return launch_pair<4, 256, MV, DEBUG>(A, st, ev);
    case 40512: return launch_pair<4, 512, MV, DEBUG>(A, st, ev);
    case 41024: return launch_pair<4, 1024, MV, DEBUG>(A, st, ev);
    case 41536: return launch_pair<4, 1536, MV, DEBUG>(A, st, ev);
    case 42048: return launch_pair<4, 2048, MV, DEBUG>(A, st, ev);
    case 81024: return launch_pair<8, 1024, MV, DEBUG>(A, st, ev);
    case 81536: return launch_pair<8, 1536, MV, DEBUG>(A, st, ev);
    case 82048: return launch_pair<8, 2048, MV, DEBUG>(A, st, ev);
    default: return hipErrorInvalidValue;
    }
}

int launch_batch(const KArgs &args, const pv_schedule &s, bool debug, void *stream, LaunchEvents *ev)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t err;
    if (args.p.mv)
        err = debug ? launch_dispatch<true, true>(args, s, st, ev) : launch_dispatch<true, false>(args, s, st, ev);
    else
        err = debug ? launch_dispatch<false, true>(args, s, st, ev) : launch_dispatch<false, false>(args, s, st, ev);
    return (int)err;
}

}  // namespace pvk
