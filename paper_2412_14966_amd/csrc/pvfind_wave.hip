// pvfind_wave.hip -- single-wavefront kernel of the primary-vertex path
// (arXiv:2412.14966, Sec. 3) for events of up to CAP tracks.
//
// One wavefront runs all five steps of one event, so every exchange between
// lanes is a wavefront-local LDS access or a cross-lane operation and no
// workgroup barrier is needed.  The event's LDS footprint is a few KiB, so
// many events are in flight per compute unit:
//   project   one pass over the tracks, Eq. 1 / Eq. 3 in binary32 exactly as
//             the multi-wavefront kernel computes them; each lane keeps z_poca,
//             1 / (u0 sigma) and the kernel window of its (up to CAP / 64)
//             tracks in registers, and the wavefront ORs the 64-bit mask of
//             touched 64-bin words
//   fill      only the touched words of the histogram exist: word w lives in
//             page popcount(mask below w).  Touched words that are neighbours
//             in z are neighbours in LDS, so every kernel window, every
//             proto-cluster run and every cluster maps to LDS by one offset
//   peaks     as in the multi-wavefront kernel, over the pages
//   associate partition points and iterative removal (Sec. 3.4)
//   gather    a stable list of track indices grouped by vertex (2 B per track,
//             in the space of the histogram pages, which are dead by then)
//   fit       L lanes per vertex read their tracks' inputs from global memory
//             (just read by the projection, so mostly cache hits) and keep
//             them in registers through the Newton iterations, the selection
//             and the final weights
// Events with more touched words than pages, more clusters than the vertex
// arrays hold or more tracks than CAP are handed to the large-team launch.
#include "pvfind_device.h"

namespace pvk {

constexpr int kPages = 16;          // 64-bin words of the histogram held per event
constexpr int kWaveRegTracks = 6;   // tracks per fit lane kept in registers
constexpr int kWaveVertices = 32;   // clusters per event

template <int CAP>
struct __align__(16) WaveSmem {
    union {
        int pg[kPages * 64];   // touched 64-bin words of the histogram, in z order
        short idx[CAP];        // track index within the event, grouped by vertex
    } u;
    int tb[CAP];               // (bin + 1) | flags << 13 | (owner + 1) << 16
    short clo[kWaveVertices], chi[kWaveVertices], cpk[kWaveVertices], live[kWaveVertices];
    float cd0[kWaveVertices];  // seed offset delta * dz from the centre of the peak bin (Eq. 4)
    int pb[kWaveVertices];     // last bin owned by live slot k
    int cnt[kWaveVertices];    // tracks owned by live slot k
    short kmap[kWaveVertices]; // live slot of cluster q (debug output)
    short ps[64], pe[64];      // pending proto-clusters
    int po[64];                // their LDS offsets
};

// LDS accesses of one wavefront execute in program order; this keeps the
// compiler from moving them across the exchange point.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long v)
{
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lo |= (unsigned)__shfl_xor((int)lo, off);
        hi |= (unsigned)__shfl_xor((int)hi, off);
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    return ((unsigned long long)hi << 32) | lo;
}

// LDS offset of the bins of touched word w: bin j of that word (and of the
// touched words that follow it without a gap) is pg[j + page_off(occ, w)]
__device__ __forceinline__ int page_off(unsigned long long occ, int w)
{
    return 64 * (__popcll(occ & ((1ull << w) - 1ull)) - w);
}

// bin j of the paged histogram, 0 in untouched words
__device__ __forceinline__ int page_bin(const int *pg, unsigned long long occ, int j)
{
    const int w = j >> 6;
    return ((occ >> w) & 1ull) ? pg[j + page_off(occ, w)] : 0;
}

__device__ __forceinline__ void wave_defer(const KArgs &A, int e)
{
    if (threadIdx.x == 0) {
        const unsigned int k = atomicAdd(&A.wq->n_big, 1u);
        A.wq->big[k] = e;
    }
}

// Fit frame quantities of track g (Eq. 2, Eq. 9): position at the frame's
// z relative to the beamline point there, slopes and 1 / V_x at the seed.
// Same operations as the multi-wavefront kernel's gather.
__device__ __forceinline__ void frame_track(const KArgs &A, unsigned g, float zr, float d0, float &X, float &Y,
                                            float &TX, float &TY, float &WT)
{
    const KParams &p = A.p;
    const float x = A.x[g], y = A.y[g], z = A.z[g], tx = A.tx[g], ty = A.ty[g];
    const float vxx = A.cxx[g], vxtx = A.cxtx[g], vtxtx = A.ctxtx[g];
    const float dzr = zr - z;
    X = fmaf(dzr, tx, x) - (p.bx + p.btx * zr);
    Y = fmaf(dzr, ty, y) - (p.by + p.bty * zr);
    TX = tx;
    TY = ty;
    const float dzs = dzr + d0;
    const float V = fmaf(dzs, fmaf(dzs, vtxtx, 2.0f * vxtx), vxx);
    WT = (V > 0.0f && isfinite(V)) ? 1.0f / V : 0.0f;
}

// Per-stage cycle counts of the debug variant, in the order of pv_debug_out.
struct WaveClock {
    unsigned long long last;
    unsigned int cyc[8];
};

template <bool DEBUG>
__device__ __forceinline__ void lap(WaveClock &c, int stage)
{
    if (DEBUG) {
        const unsigned long long t = clock64();
        c.cyc[stage] += (unsigned int)(t - c.last);
        c.last = t;
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.3: proto-clusters, dip search and seeds over the paged histogram.
// Returns the number of clusters found (possibly more than `cap`).
// ---------------------------------------------------------------------------
template <int CAP>
__device__ __forceinline__ int wave_peaks(WaveSmem<CAP> &S, const KParams &p, unsigned long long occ, int cap)
{
    const int lane = threadIdx.x;
    int n_found = 0, npend = 0, open_s = -1, open_off = 0, prev_w = -2, pgi = 0;
    unsigned long long rem = occ;
    auto push = [&](int s, int e, int off) __attribute__((always_inline)) {
        if (lane == 0) {
            S.ps[npend] = (short)s;
            S.pe[npend] = (short)e;
            S.po[npend] = off;
        }
        ++npend;
    };
    for (;;) {
        const bool last = (rem == 0ull);
        if (!last) {
            const int w = __ffsll((long long)rem) - 1;
            rem &= rem - 1ull;
            const int off = 64 * (pgi - w);
            if (open_s >= 0 && prev_w != w - 1) {
                push(open_s, 64 * prev_w + 63, open_off);
                open_s = -1;
            }
            const int j = 64 * w + lane;
            const int hv = (j < p.nb) ? S.u.pg[j + off] : 0;
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
        wave_sync();
        if (npend >= 32 || (last && npend > 0)) {
            const bool has = lane < npend;
            int s = 0, e = 0, off = 0;
            if (has) {
                s = S.ps[lane];
                e = S.pe[lane];
                off = S.po[lane];
            }
            const int tot = has ? sum_bins(S.u.pg, off, s, e) : 0;
            unsigned long long cw = 0ull;
            int ns = 0, fin = 0;
            const int c = has ? walk_proto(S.u.pg, off, S.clo, S.chi, cap, p, s, e, tot, false, 0, &cw, &ns, &fin) : 0;
            const int incl = wave_incl_scan(c, lane);
            const int first = n_found + incl - c;
            if (has && ns > 4) {
                walk_proto(S.u.pg, off, S.clo, S.chi, cap, p, s, e, tot, true, first);
            } else if (has) {
                int lo = s, q = first;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (k < ns) {
                        const int hi = (int)((cw >> (16 * k)) & 0xFFFFull);
                        if (q < cap) {
                            S.clo[q] = (short)lo;
                            S.chi[q] = (short)hi;
                        }
                        ++q;
                        lo = hi + 1;
                    }
                }
                if (fin && q < cap) {
                    S.clo[q] = (short)lo;
                    S.chi[q] = (short)e;
                }
            }
            n_found += __shfl(incl, 63);
            npend = 0;
            wave_sync();
        }
        if (last)
            break;
    }
    wave_sync();
    // seeds (Eq. 4-5): first highest bin, correction from the neighbours
    const int ncl = min(n_found, cap);
    for (int q = lane; q < ncl; q += 64) {
        const int lo = S.clo[q], hi = S.chi[q];
        const int off = page_off(occ, lo >> 6);
        const int im = argmax_bins(S.u.pg, off, lo, hi);
        const int Ni = S.u.pg[im + off];
        const int Nm = (im > 0) ? page_bin(S.u.pg, occ, im - 1) : 0;
        const int Np = (im + 1 < p.nb) ? page_bin(S.u.pg, occ, im + 1) : 0;
        const int den = 2 * Ni - Np - Nm;
        float delta = (den > 0) ? 0.5f * (float)(Np - Nm) / (float)den : 0.0f;
        delta = fminf(fmaxf(delta, -0.5f), 0.5f);
        S.cpk[q] = (short)im;
        S.cd0[q] = delta * p.dz;
    }
    wave_sync();
    return n_found;
}

// ---------------------------------------------------------------------------
// Sec. 3.5: fit, selection (Table 2, end of Sec. 3.5) and final weights of
// the nl live vertices, L lanes per vertex (L * nl <= 64).  Lane k of the
// wavefront holds base / count of live slot k in `base` / `count`.  L is
// wavefront-uniform.  Returns the number of kept vertices.
// ---------------------------------------------------------------------------
template <int CAP, bool DEBUG>
__device__ __forceinline__ int wave_fit(WaveSmem<CAP> &S, const KArgs &A, int e, int a, int nl, int L, int base,
                                        int count, WaveClock &clk)
{
    const KParams &p = A.p;
    const int lane = threadIdx.x;
    const int gid = lane / L, gl = lane & (L - 1);
    const bool has = gid < nl;
    const int beg = __shfl(base, gid);
    const int ck0 = __shfl(count, gid);
    const int ck = has ? ck0 : 0;
    const int cq = has ? S.live[gid] : 0;
    const float zr = bin_centre(S.cpk[cq], p);
    const float d0 = has ? S.cd0[cq] : 0.0f;

    float rX[kWaveRegTracks], rY[kWaveRegTracks], rTX[kWaveRegTracks], rTY[kWaveRegTracks], rW[kWaveRegTracks];
#pragma unroll
    for (int u = 0; u < kWaveRegTracks; ++u) {
        const int t = gl + u * L;
        if (t < ck)
            frame_track(A, a + S.u.idx[beg + t], zr, d0, rX[u], rY[u], rTX[u], rTY[u], rW[u]);
        else
            rX[u] = rY[u] = rTX[u] = rTY[u] = rW[u] = 0.0f;
    }

    // Newton iterations from the seed: on the beamline, delta dz above the bin centre
    float dx = p.btx * d0, dy = p.bty * d0, dz = d0, la = 0.0f, lb = 0.0f, lc = 0.0f, ld = 0.0f;
    int nit = 0;
    bool active = has, failed = false, conv = false;
    for (int it = 1; it <= p.max_iter; ++it) {
        if (!__any(active))
            break;
        FitSums s = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (active) {
#pragma unroll
            for (int u = 0; u < kWaveRegTracks; ++u)
                if (rW[u] > 0.0f)
                    accumulate(s, rX[u], rY[u], rTX[u], rTY[u], rW[u], dx, dy, dz, p);
            for (int t = gl + kWaveRegTracks * L; t < ck; t += L) {
                float X, Y, TX, TY, WT;
                frame_track(A, a + S.u.idx[beg + t], zr, d0, X, Y, TX, TY, WT);
                if (WT > 0.0f)
                    accumulate(s, X, Y, TX, TY, WT, dx, dy, dz, p);
            }
        }
        const float s0 = group_sum_rt(s.s0, L), sx = group_sum_rt(s.sx, L), sy = group_sum_rt(s.sy, L);
        const float szz = group_sum_rt(s.szz, L), gx = group_sum_rt(s.gx, L), gy = group_sum_rt(s.gy, L);
        const float gz = group_sum_rt(s.gz, L), sw = group_sum_rt(s.sw, L);
        if (active) {
            const float D = fmaf(s0, szz, -fmaf(sx, sx, sy * sy));
            if (!(sw > 0.0f) || !(s0 > 0.0f) || !(D > p.sing_ratio * (s0 * szz))) {
                failed = true;
                active = false;
            } else {
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
                if (fabsf(dchi2) < p.conv_dchi2 && fabsf(ddz) < p.conv_dz) {
                    conv = true;
                    active = false;
                }
            }
        }
    }
    lap<DEBUG>(clk, 5);

    // selection: every lane of a group holds its vertex's state
    bool keep = false;
    if (has) {
        const bool gas = S.cpk[cq] < p.gas_bin;
        keep = !failed && ck >= (gas ? p.pv_min_gas : p.pv_min_pp);
        if (keep && !gas) {
            const float zv = zr + dz;
            const float xv = (p.bx + p.btx * zr) + dx;
            const float yv = (p.by + p.bty * zr) + dy;
            const float rx = xv - (p.bx + p.btx * zv);
            const float ry = yv - (p.by + p.bty * zv);
            keep = fmaf(rx, rx, ry * ry) <= p.max_rho2_pp;
        }
    }
    const unsigned long long km = __ballot(keep && gl == 0);
    const int vo = keep ? __popcll(km & lanemask_lt(gid * L)) : -1;
    const int n_keep = __popcll(km);
    lap<DEBUG>(clk, 6);

    // final Tukey weights at the fitted position, chi2 and ndof (2 sum w - 3)
    float schi = 0.0f, swf = 0.0f;
    auto final_track = [&](int t, float X, float Y, float TX, float TY, float WT) __attribute__((always_inline)) {
        float w = 0.0f, chi2 = 0.0f;
        if (WT > 0.0f) {
            const float rx = fmaf(dz, TX, X) - dx;
            const float ry = fmaf(dz, TY, Y) - dy;
            chi2 = WT * fmaf(rx, rx, ry * ry);
            if (chi2 < p.chi2_max) {
                const float u = fmaf(-chi2, p.inv_chi2_max, 1.0f);
                w = u * u;
            }
        }
        schi = fmaf(w, chi2, schi);
        swf += w;
        const unsigned g = a + S.u.idx[beg + t];
        A.trk_vtx[g] = vo;
        A.trk_w[g] = (vo >= 0) ? w : 0.0f;
    };
#pragma unroll
    for (int u = 0; u < kWaveRegTracks; ++u) {
        const int t = gl + u * L;
        if (t < ck)
            final_track(t, rX[u], rY[u], rTX[u], rTY[u], rW[u]);
    }
    for (int t = gl + kWaveRegTracks * L; t < ck; t += L) {
        float X, Y, TX, TY, WT;
        frame_track(A, a + S.u.idx[beg + t], zr, d0, X, Y, TX, TY, WT);
        final_track(t, X, Y, TX, TY, WT);
    }
    schi = group_sum_rt(schi, L);
    swf = group_sum_rt(swf, L);
    if (has && gl == 0 && vo >= 0) {
        float cf[6];
        const float det = inverse_a<float>(la, lb, lc, ld, cf);
        const float na = fmaxf(fmaxf(la + fabsf(lb), la + fabsf(lc)), fabsf(lb) + fabsf(lc) + ld);
        const float ni = fmaxf(fmaxf(fabsf(cf[0]) + fabsf(cf[1]) + fabsf(cf[3]),
                                     fabsf(cf[1]) + fabsf(cf[2]) + fabsf(cf[4])),
                               fabsf(cf[3]) + fabsf(cf[4]) + fabsf(cf[5]));
        int flags = conv ? 0 : PV_VX_NOT_CONVERGED;
        if (!(det > 0.0f) || !(na * ni <= p.cond_fp64)) {
            double cd[6];
            inverse_a<double>((double)la, (double)lb, (double)lc, (double)ld, cd);
            for (int q = 0; q < 6; ++q)
                cf[q] = (float)cd[q];
            flags |= PV_VX_FP64_INVERSION;
        }
        pv_vertex v;
        v.x = (p.bx + p.btx * zr) + dx;
        v.y = (p.by + p.bty * zr) + dy;
        v.z = zr + dz;
        for (int q = 0; q < 6; ++q)
            v.cov[q] = cf[q];
        v.chi2 = schi;
        v.ndof = 2.0f * swf - 3.0f;
        v.z_seed = zr + S.cd0[cq];
        v.n_tracks = ck;
        v.bin_lo = S.clo[cq];
        v.bin_hi = S.chi[cq];
        v.peak_bin = S.cpk[cq];
        v.n_iter = (uint8_t)nit;
        v.flags = (uint8_t)flags;
        v.reserved = 0;
        A.vout[(size_t)e * p.max_vertices + vo] = v;
    }
    lap<DEBUG>(clk, 7);
    return n_keep;
}

// ---------------------------------------------------------------------------
// one event
// ---------------------------------------------------------------------------
template <int CAP, bool DEBUG>
__device__ __forceinline__ void wave_event(WaveSmem<CAP> &S, const KArgs &A, int e, int n_events)
{
    constexpr int CH = CAP / 64;
    const KParams &p = A.p;
    const int lane = threadIdx.x;
    wave_sync();   // the previous event's LDS accesses stay before this event's

    const int a = A.offsets[e], b = A.offsets[e + 1], total = A.offsets[n_events];
    const bool bad_offsets = (a < 0) || (b < a) || (b > total);
    const int n = bad_offsets ? 0 : b - a;
    if (bad_offsets || n > p.max_tracks) {
        if (!bad_offsets) {
            for (int i = lane; i < n; i += 64) {
                A.trk_vtx[(unsigned)(a + i)] = -1;
                A.trk_w[(unsigned)(a + i)] = 0.0f;
            }
        }
        if (DEBUG && A.dbg_hist)
            for (int j = lane; j < p.nb; j += 64)
                A.dbg_hist[(size_t)e * p.nb + j] = 0;
        if (lane == 0) {
            A.status_out[e] = bad_offsets ? PV_EV_OFFSETS_INVALID : PV_EV_TOO_MANY_TRACKS;
            A.nv_out[e] = 0;
            if (DEBUG && A.dbg_ncl)
                A.dbg_ncl[e] = 0;
        }
        return;
    }
    if (n > CAP) {
        wave_defer(A, e);
        return;
    }

    WaveClock clk;
    if (DEBUG) {
        clk.last = clock64();
        for (int k = 0; k < 8; ++k)
            clk.cyc[k] = 0;
    }

    // project: z_poca, 1 / (u0 sigma) and the window of each histogrammed track
    float zq[CH], rq[CH];
    int wq[CH];
    unsigned long long words = 0ull;
    bool nonfinite = false;
    {
        float cur[8], nxt[8];
        if (lane < n)
            load_track(A, a + lane, cur);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            zq[c] = 0.0f;
            rq[c] = 0.0f;
            wq[c] = 0;
            if (c * 64 < n) {
                const int i = c * 64 + lane;
                if (c + 1 < CH && i + 64 < n)
                    load_track(A, a + i + 64, nxt);
                if (i < n) {
                    const Proj r = project(cur[0], cur[1], cur[2], cur[3], cur[4], cur[5], cur[6], cur[7], p);
                    if (r.fl & kTrHist) {
                        const float sw = p.u0 * r.sg;
                        const Window w = track_window(r.zp, sw, p);
                        if (w.jh > w.jl) {
                            words |= window_words(w);
                            zq[c] = r.zp;
                            rq[c] = 1.0f / sw;
                            wq[c] = w.jl | (w.jh << 16);
                        }
                    }
                    nonfinite |= (r.fl & kTrNonfinite) != 0;
                    S.tb[i] = (r.bin + 1) | (r.fl << 13);
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
                if (c + 1 < CH) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        cur[q] = nxt[q];
                }
            }
        }
    }
    const unsigned long long occ = wave_or64(words);
    const int status = __ballot(nonfinite) ? PV_EV_NONFINITE_INPUT : 0;
    const int npg = __popcll(occ);
    if (npg > kPages) {
        wave_defer(A, e);
        return;
    }
    lap<DEBUG>(clk, 1);

    // clear the pages in use
    {
        int4 *h4 = reinterpret_cast<int4 *>(S.u.pg);
        for (int k = lane; k < npg * 16; k += 64)
            h4[k] = make_int4(0, 0, 0, 0);
    }
    wave_sync();
    lap<DEBUG>(clk, 0);

    // fill: windows of up to kShortWindow bins by their own lane, wider ones
    // by the whole wavefront one track at a time
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if (c * 64 < n) {
            bool wide = false;
            int off = 0;
            const Window w{wq[c] & 0xFFFF, wq[c] >> 16};
            if (rq[c] > 0.0f) {
                off = page_off(occ, w.jl >> 6);
                wide = (w.jh - w.jl) > kShortWindow;
                if (!wide)
                    fill_short(S.u.pg, off, w, zq[c], rq[c], p);
            }
            unsigned long long wm = __ballot(wide);
            while (wm) {
                const int src = __ffsll((long long)wm) - 1;
                wm &= wm - 1ull;
                const float zs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zq[c]), src));
                const float rs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rq[c]), src));
                const int jl = __builtin_amdgcn_readlane(w.jl, src);
                const int jh = __builtin_amdgcn_readlane(w.jh, src);
                const int os = __builtin_amdgcn_readlane(off, src);
                for (int j = jl + lane; j < jh; j += 64) {
                    const int d = code_at(j + 1, zs, rs, p) - code_at(j, zs, rs, p);
                    if (d != 0)
                        atomicAdd(&S.u.pg[j + os], d);
                }
            }
        }
    }
    wave_sync();
    if (DEBUG && A.dbg_hist)
        for (int j = lane; j < p.nb; j += 64)
            A.dbg_hist[(size_t)e * p.nb + j] = page_bin(S.u.pg, occ, j);
    lap<DEBUG>(clk, 1);

    // peaks and seeds
    const int cap = min(p.max_vertices, kWaveVertices);
    const int n_found = wave_peaks(S, p, occ, cap);
    if (n_found > kWaveVertices && p.max_vertices > kWaveVertices) {
        wave_defer(A, e);
        return;
    }
    const int ncl = min(n_found, cap);
    const int st_ev = status | ((n_found > p.max_vertices) ? PV_EV_VERTEX_OVERFLOW : 0);
    lap<DEBUG>(clk, 2);

    // association with iterative removal of the weakest cluster (Sec. 3.4)
    if (lane < ncl)
        S.live[lane] = (short)lane;
    int nl = ncl;
    wave_sync();
    for (;;) {
        if (lane < nl) {
            const int cq = S.live[lane];
            S.pb[lane] = (lane + 1 < nl) ? ((S.chi[cq] + S.clo[S.live[lane + 1]]) >> 1) : p.nb - 1;
            S.cnt[lane] = 0;
        }
        wave_sync();
        for (int i = lane; i < n; i += 64) {
            const int t = S.tb[i];
            int own = -1;
            if (((t >> 13) & kTrAssoc) && nl > 0) {
                own = lower_bound_bins(S.pb, nl, (t & 0x1FFF) - 1);
                atomicAdd(&S.cnt[own], 1);
            }
            S.tb[i] = (t & 0xFFFF) | ((own + 1) << 16);
        }
        wave_sync();
        int key = INT_MAX;
        if (lane < nl) {
            const int cq = S.live[lane];
            const int need = (S.cpk[cq] < p.gas_bin) ? p.part_min_gas : p.part_min_pp;
            const int c = S.cnt[lane];
            if (c < need)
                key = (c << 8) | lane;
        }
        key = wave_min(key);
        if (key == INT_MAX)
            break;
        const int kv = key & 0xFF;
        short v = 0;
        if (lane < nl - 1)
            v = S.live[lane + (lane >= kv ? 1 : 0)];
        wave_sync();
        if (lane < nl - 1)
            S.live[lane] = v;
        --nl;
        wave_sync();
    }
    const int count = (lane < nl) ? S.cnt[lane] : 0;
    lap<DEBUG>(clk, 3);

    if (DEBUG && A.dbg_cl) {
        if (lane < ncl)
            S.kmap[lane] = -1;
        wave_sync();
        if (lane < nl)
            S.kmap[S.live[lane]] = (short)lane;
        wave_sync();
        if (lane < ncl) {
            const int q = lane, k = S.kmap[q];
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

    // gather: stable list of track indices grouped by vertex; lane k keeps the
    // running slot of live slot k
    const int incl = wave_incl_scan(count, lane);
    const int base = incl - count;
    int run = base;
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int i = c0 + lane;
        const bool valid = i < n;
        const int own = valid ? (S.tb[i] >> 16) - 1 : -1;
        unsigned long long rem = __ballot(own >= 0);
        int slot = -1;
        while (rem) {
            const int leader = __ffsll((long long)rem) - 1;
            const int ol = __builtin_amdgcn_readlane(own, leader);
            const unsigned long long mm = __ballot(own == ol);
            const int r0 = __builtin_amdgcn_readlane(run, ol);
            if (own == ol)
                slot = r0 + __popcll(mm & lanemask_lt(lane));
            if (lane == ol)
                run += __popcll(mm);
            rem &= ~mm;
        }
        if (valid) {
            if (slot >= 0) {
                S.u.idx[slot] = (short)i;
            } else {
                A.trk_vtx[(unsigned)(a + i)] = -1;
                A.trk_w[(unsigned)(a + i)] = 0.0f;
            }
        }
    }
    wave_sync();
    lap<DEBUG>(clk, 4);

    // fit, selection and final weights, L the largest power of two with L * nl <= 64
    int n_keep = 0;
    if (nl > 0) {
        int L = 64;
        while (L > 1 && L * nl > 64)
            L >>= 1;
        n_keep = wave_fit<CAP, DEBUG>(S, A, e, a, nl, L, base, count, clk);
    }
    if (lane == 0) {
        A.nv_out[e] = n_keep;
        A.status_out[e] = st_ev;
        if (DEBUG && A.dbg_ncl)
            A.dbg_ncl[e] = ncl;
    }
    wave_sync();
    if (DEBUG && A.dbg_cycles && lane == 0)
        for (int k = 0; k < 8; ++k)
            A.dbg_cycles[(size_t)e * 8 + k] = clk.cyc[k];
}

// mode 0: one wavefront per event (grid = n_events); mode 1: persistent grid
// popping events from the device work queue.
template <int CAP, bool DEBUG>
__global__ __launch_bounds__(64) void pv_wave_kernel(KArgs A, int mode)
{
    __shared__ WaveSmem<CAP> S;
    const int n_events = A.n_events_dev ? *A.n_events_dev : A.n_events;
    if (mode == 1) {
        for (;;) {
            unsigned int k = 0u;
            if (threadIdx.x == 0)
                k = atomicAdd(&A.wq->next, 1u);
            k = (unsigned int)__builtin_amdgcn_readfirstlane((int)k);
            if (k >= (unsigned int)n_events)
                break;
            wave_event<CAP, DEBUG>(S, A, (int)k, n_events);
        }
        if (threadIdx.x == 0) {
            __threadfence();
            const unsigned int prev = atomicAdd(&A.wq->done, 1u);
            if (prev == gridDim.x - 1) {
                atomicExch(&A.wq->next, 0u);
                atomicExch(&A.wq->done, 0u);
                __threadfence();
            }
        }
    } else if ((int)blockIdx.x < n_events) {
        wave_event<CAP, DEBUG>(S, A, (int)blockIdx.x, n_events);
    }
}

template <int CAP, bool DEBUG>
static hipError_t launch_wave_cap(const KArgs &A, int mode, int teams_per_cu, int cus, hipStream_t st)
{
    auto *fn = pv_wave_kernel<CAP, DEBUG>;
    int grid = A.n_events;
    if (mode == 1) {
        int occ = 0;
        hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64, 0);
        if (err != hipSuccess)
            return err;
        if (occ < 1)
            occ = 1;
        if (teams_per_cu > 0 && teams_per_cu < occ)
            occ = teams_per_cu;
        grid = occ * (cus > 0 ? cus : 256);
        if (grid > A.n_events)
            grid = A.n_events;
        if (grid < 1)
            grid = 1;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64), 0, st, A, mode);
    return hipGetLastError();
}

int launch_wave(const KArgs &A, int capacity, int mode, int teams_per_cu, int cus, bool debug, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t err;
    if (capacity == 256)
        err = debug ? launch_wave_cap<256, true>(A, mode, teams_per_cu, cus, st)
                    : launch_wave_cap<256, false>(A, mode, teams_per_cu, cus, st);
    else if (capacity == 512)
        err = debug ? launch_wave_cap<512, true>(A, mode, teams_per_cu, cus, st)
                    : launch_wave_cap<512, false>(A, mode, teams_per_cu, cus, st);
    else
        err = hipErrorInvalidValue;
    return (int)err;
}

}  // namespace pvk
