// pvfind_device.h -- device helpers shared by the gfx950 kernels of the
// primary-vertex path (arXiv:2412.14966, Sec. 3): wavefront scans and group
// sums, the projection (Eq. 1, Eq. 3), the fixed-point kernel masses of the
// histogram (Sec. 3.2), the dip search (Sec. 3.3) and the fit's sums (Sec. 3.5).
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include "pvfind_internal.h"

namespace pvk {

constexpr int kInfoNotConv = 1 << 8;
constexpr int kInfoFailed = 1 << 9;

// the 64-bit value of lane `src` (wavefront-uniform)
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int src)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), src);
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane)
{
    return (1ull << lane) - 1ull;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off)
            v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = min(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ float wave_min_f(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fminf(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ float wave_max_f(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// Group sums below: every lane of a group gets the same bits (the pairs
// added are the same, addition is commutative).  Within a row of 16 lanes the
// partners come from DPP (quad permutes, half-row and row mirrors), across
// rows from a swizzle and a permute.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over aligned groups of L lanes, for a compile-time L.
template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    if (L >= 2)
        v += dpp_f<0xB1>(v);     // quad_perm [1,0,3,2]
    if (L >= 4)
        v += dpp_f<0x4E>(v);     // quad_perm [2,3,0,1]
    if (L >= 8)
        v += dpp_f<0x141>(v);    // row_half_mirror: lane i <-> 7 - i
    if (L >= 16)
        v += dpp_f<0x140>(v);    // row_mirror: lane i <-> 15 - i
    if (L >= 32)
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));   // xor 16
    if (L >= 64)
        v += __shfl_xor(v, 32);
    return v;
}

// Sum over aligned groups of L lanes, for a wavefront-uniform L (one copy of
// the caller's code serves every group size).  Every butterfly level runs and
// a select keeps the levels below L, so no branch depends on L.
__device__ __forceinline__ float group_sum_rt(float v, int L)
{
    float t = dpp_f<0xB1>(v);
    v = (L >= 2) ? v + t : v;
    t = dpp_f<0x4E>(v);
    v = (L >= 4) ? v + t : v;
    t = dpp_f<0x141>(v);
    v = (L >= 8) ? v + t : v;
    t = dpp_f<0x140>(v);
    v = (L >= 16) ? v + t : v;
    t = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    v = (L >= 32) ? v + t : v;
    t = __shfl_xor(v, 32);
    v = (L >= 64) ? v + t : v;
    return v;
}

// The N sums of one Newton step for groups whose size L = 2^lg varies from
// lane to lane: the groups are aligned blocks, so every butterfly partner of a
// lane lies in its own group.  The levels run up to lgmax, the wavefront's
// largest group (one scalar branch per level), each kept by a select where
// the lane's group is smaller.
template <int N>
__device__ __forceinline__ void group_sum_n_var_rt(float v[N], int L, int lgmax)
{
    if (lgmax >= 1)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const float t = dpp_f<0xB1>(v[q]);
            v[q] = (L >= 2) ? v[q] + t : v[q];
        }
    if (lgmax >= 2)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const float t = dpp_f<0x4E>(v[q]);
            v[q] = (L >= 4) ? v[q] + t : v[q];
        }
    if (lgmax >= 3)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const float t = dpp_f<0x141>(v[q]);
            v[q] = (L >= 8) ? v[q] + t : v[q];
        }
    if (lgmax >= 4)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const float t = dpp_f<0x140>(v[q]);
            v[q] = (L >= 16) ? v[q] + t : v[q];
        }
    if (lgmax >= 5)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const float t = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v[q]), 0x401F));
            v[q] = (L >= 32) ? v[q] + t : v[q];
        }
    if (lgmax >= 6)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const float t = __shfl_xor(v[q], 32);
            v[q] = (L >= 64) ? v[q] + t : v[q];
        }
}

// The N sums of one Newton step at once, for a wavefront-uniform group of
// L = 1 << lg lanes: one scalar branch picks the butterfly for that L.
template <int L, int N>
__device__ __forceinline__ void group_sum_n(float v[N])
{
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] = group_sum<L>(v[k]);
}

template <int N>
__device__ __forceinline__ void group_sum_n_rt(float v[N], int lg)
{
    switch (lg) {
    case 0: break;
    case 1: group_sum_n<2, N>(v); break;
    case 2: group_sum_n<4, N>(v); break;
    case 3: group_sum_n<8, N>(v); break;
    case 4: group_sum_n<16, N>(v); break;
    case 5: group_sum_n<32, N>(v); break;
    default: group_sum_n<64, N>(v); break;
    }
}

// Track indices are non-negative 32-bit values: unsigned indexing lets the
// loads use one 32-bit offset register against the arrays' scalar bases.
__device__ __forceinline__ void load_track(const KArgs &A, unsigned g, float t[8])
{
    t[0] = A.x[g];
    t[1] = A.y[g];
    t[2] = A.z[g];
    t[3] = A.tx[g];
    t[4] = A.ty[g];
    t[5] = A.cxx[g];
    t[6] = A.cxtx[g];
    t[7] = A.ctxtx[g];
}

// ---------------------------------------------------------------------------
// Sec. 3.1: projection to the point of closest approach (Eq. 1, Eq. 3)
// ---------------------------------------------------------------------------
struct Proj {
    float zp, sg;
    int bin, fl;
};

__device__ __forceinline__ Proj project(float x, float y, float z, float tx, float ty, float vxx,
                                        float vxtx, float vtxtx, const KParams &p)
{
    Proj r{0.0f, 0.0f, -1, 0};
    if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(tx) && isfinite(ty) && isfinite(vxx) &&
          isfinite(vxtx) && isfinite(vtxtx))) {
        r.fl = kTrNonfinite;
        return r;
    }
    const float dtx = tx - p.btx;
    const float dty = ty - p.bty;
    const float dx = p.bx - x;
    const float dy = p.by - y;
    const float num = dtx * dx + dty * dy;
    const float den = dtx * dtx + dty * dty;
    if (!(den > 0.0f) || !(vxx > 0.0f))
        return r;
    const float zp = z + num / den;
    const float s2 = vxx / den;
    const float sg = sqrtf(s2);
    r.zp = zp;
    r.sg = sg;
    if (!(zp >= p.z_min && zp < p.z_max))
        return r;
    // the bin is floor of a correctly rounded quotient; when dz is a power
    // of two the product with 1 / dz is that same quotient, exactly
    const float q = p.dz_pow2 ? (zp - p.z_min) * p.inv_dz : (zp - p.z_min) / p.dz;
    int b = (int)floorf(q);
    b = min(max(b, 0), p.nb - 1);
    r.bin = b;
    r.fl = kTrAssoc;
    const float smax = (b < p.gas_bin) ? p.sigma_max_gas : p.sigma_max_pp;
    const float sw = p.u0 * sg;
    if (s2 <= smax * smax && sw > 0.0f)
        r.fl |= kTrHist;
    return r;
}

// ---------------------------------------------------------------------------
// Sec. 3.2: kernel mass left of a bin edge, cubic cumulative, fixed point
// ---------------------------------------------------------------------------
// P * unit rounded to the nearest integer, ties to even: P * unit is exact
// (unit = 2^frac_bits, frac_bits <= 18, P in [0, 1]), so the fused
// multiply-add with 1.5 * 2^23 rounds the exact product once, to an integer
// held in the low mantissa bits
__device__ __forceinline__ int fixed_code(float P, float unit)
{
    return __float_as_int(__builtin_fmaf(P, unit, 12582912.0f)) - 0x4B400000;
}

// r = 1 / (u0 sigma), correctly rounded, once per track
__device__ __forceinline__ int edge_code(float e, float zp, float r, float unit)
{
    float s = (e - zp) * r;
    if (s < -1.0f)
        s = -1.0f;
    if (s > 1.0f)
        s = 1.0f;
    const float P = 0.5f + s * __builtin_fmaf(-0.25f, s * s, 0.75f);
    return fixed_code(P, unit);
}

// Window of edges [jl, jh] whose codes are computed for a track at zp with
// half-width sw: any superset of the kernel's support gives the same
// integers, so the bounds may be approximate; one extra edge on each side
// makes the end codes exactly 0 and 'full'.
struct Window {
    int jl, jh;   // bins jl .. jh-1 receive mass
};

__device__ __forceinline__ Window track_window(float zp, float sw, const KParams &p)
{
    const float fl = fmaxf(floorf((zp - sw - p.z_min) * p.inv_dz) - 1.0f, 0.0f);
    const float fh = fminf(ceilf((zp + sw - p.z_min) * p.inv_dz) + 1.0f, (float)p.nb);
    return Window{(int)fl, (int)fh};
}

__device__ __forceinline__ int code_at(int j, float zp, float r, const KParams &p)
{
    // first edge of the histogram: P = 0; last edge: P = 1
    if (j <= 0)
        return 0;
    if (j >= p.nb)
        return (int)p.unit;
    return edge_code(p.z_min + (float)j * p.dz, zp, r, p.unit);
}

constexpr int kShortWindow = 12;  // bins per lane in the per-lane pass

// per-lane pass: windows of at most kShortWindow bins, fixed trip count and
// no branch but the atomic's.  Edge jh (the window's last, jh <= nb) carries
// the full code and so does every edge after it (the window has one spare
// edge beyond the kernel's support, and the codes grow with the edge), so
// those edges are set to `unit` without evaluation and add nothing.
// hist[j + off] holds bin j.
// code of edge e (its z) for a track at zp with r = 1 / (u0 sigma).  The
// cubic's inner term 0.75 - 0.25 s^2 is one fused multiply-add: 0.25 s^2 is
// exact (a power-of-two scaling; below the normal range it is far under half
// an ulp of 0.75 either way), so the single rounding equals the two.
__device__ __forceinline__ int edge_code_z(float e, float zp, float r, const KParams &p)
{
    // clamp to [-1, 1]; s is finite here (zp and r are)
    const float s = __builtin_amdgcn_fmed3f((e - zp) * r, -1.0f, 1.0f);
    const float P = 0.5f + s * __builtin_fmaf(-0.25f, s * s, 0.75f);
    return fixed_code(P, p.unit);
}

__device__ __forceinline__ int edge_code_in(int j, float zp, float r, const KParams &p)
{
    return edge_code_z(p.z_min + (float)j * p.dz, zp, r, p);
}

template <int T = kShortWindow>
__device__ __forceinline__ void fill_short(int *hist, int off, Window w, float zp, float r, const KParams &p)
{
    const int full = (int)p.unit;
    if (p.edges_exact) {
        // every edge z_min + j dz is exact in binary32, so edge j + 1 is edge j
        // plus dz, exactly
        float e = p.z_min + (float)w.jl * p.dz;
        int prev = (w.jl <= 0) ? 0 : edge_code_z(e, zp, r, p);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const int j = w.jl + u;
            e += p.dz;
            const int c = edge_code_z(e, zp, r, p);
            const int next = (j + 1 >= w.jh) ? full : c;
            const int d = next - prev;
            if (d != 0)
                atomicAdd(&hist[j + off], d);
            prev = next;
        }
        return;
    }
    int prev = (w.jl <= 0) ? 0 : edge_code_in(w.jl, zp, r, p);
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int j = w.jl + u;
        const int c = edge_code_in(j + 1, zp, r, p);
        const int next = (j + 1 >= w.jh) ? full : c;
        const int d = next - prev;
        if (d != 0)
            atomicAdd(&hist[j + off], d);
        prev = next;
    }
}

__device__ __forceinline__ unsigned long long window_words(Window w)
{
    const int wl = w.jl >> 6, wh = (w.jh - 1) >> 6;
    return (2ull << wh) - (1ull << wl);
}

// ---------------------------------------------------------------------------
// Sec. 3.3: reads of the histogram by one lane
// ---------------------------------------------------------------------------
// Bins [s, e] are read 8 at a time with independent LDS loads so that one
// lane's serial walk pays the LDS latency once per 8 bins.  h[k + off] is
// bin k.
__device__ __forceinline__ int sum_bins(const int *h, int off, int s, int e)
{
    int tot = 0;
    for (int k0 = s; k0 <= e; k0 += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = (k0 + u <= e) ? h[k0 + u + off] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            tot += v[u];
    }
    return tot;
}

// first index of the highest bin in [s, e]
__device__ __forceinline__ int argmax_bins(const int *h, int off, int s, int e)
{
    int im = s, best = INT_MIN;
    for (int k0 = s; k0 <= e; k0 += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = (k0 + u <= e) ? h[k0 + u + off] : INT_MIN;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (v[u] > best) {
                best = v[u];
                im = k0 + u;
            }
    }
    return im;
}

// ---------------------------------------------------------------------------
// Sec. 3.3: dip search and z-ordered splitting of one proto-cluster [s, e]
// with bin total `tot`, and the seed bin of every cluster (Eq. 4: its first
// highest bin) tracked during the same walk.  h[k + off] is bin k.
// Returns the number of clusters.  With WRITE the clusters go to clo / chi /
// cpk from index `first` (below `cap`); otherwise the first four clusters
// closed by a split are packed into o.rec (end bin | seed bin << 16), their
// count into o.nsplit and the remainder's seed bin (-1: not a cluster) into
// o.fin_peak, so that the usual case needs no second walk.
// ---------------------------------------------------------------------------
struct WalkOut {
    unsigned rec[4];
    int nsplit;
    int fin_peak;
};

template <bool WRITE>
__device__ __forceinline__ int walk_proto(const int *h, int off, const KParams &p, int s, int e, int tot, WalkOut &o,
                                          short *clo, short *chi, short *cpk, int cap, int first)
{
    const bool strad = (s < p.gas_bin) && (e >= p.gas_bin);
    const int ifix = (s < p.gas_bin) ? p.min_int_gas : p.min_int_pp;
    // Table 2 threshold of a cluster whose seed bin is `peak`
    auto thr_at = [&](int peak) -> int { return (peak < p.gas_bin) ? p.min_int_gas : p.min_int_pp; };
    int count = 0;
    auto emit = [&](int lo, int hi, int pk) {
        if (WRITE) {
            const int q = first + count;
            if (q < cap) {
                clo[q] = (short)lo;
                chi[q] = (short)hi;
                cpk[q] = (short)pk;
            }
        } else {
            // registers, not an indexed array (which would live in scratch)
            const unsigned r = (unsigned)hi | ((unsigned)pk << 16);
            if (count == 0)
                o.rec[0] = r;
            else if (count == 1)
                o.rec[1] = r;
            else if (count == 2)
                o.rec[2] = r;
            else if (count == 3)
                o.rec[3] = r;
        }
        ++count;
    };
    int cs = s, pcs = 0;
    int up = 1, M = 0, m = 0, mj = s, pm = 0, pref = 0;
    // highest bin of [cs, k] (value, first index), of (mj, k], and of [cs, mj]
    int bM = INT_MIN, bI = s, aM = INT_MIN, aI = s, sI = s;
    for (int k0 = s; k0 <= e; k0 += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = (k0 + u <= e) ? h[k0 + u + off] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            if (k > e)
                break;
            const int hk = v[u];
            pref += hk;
            if (hk > bM) {
                bM = hk;
                bI = k;
            }
            if (hk > aM) {
                aM = hk;
                aI = k;
            }
            if (k == s) {
                M = hk;
            } else if (up) {
                if (hk > M) {
                    M = hk;
                } else if (hk <= M - p.dip_prom) {
                    up = 0;
                    m = hk;
                    mj = k;
                    pm = pref;
                    sI = bI;
                    aM = INT_MIN;
                }
            } else {
                if (hk < m) {
                    m = hk;
                    mj = k;
                    pm = pref;
                    sI = bI;
                    aM = INT_MIN;
                } else if (hk >= m + p.dip_prom) {
                    if (pm - pcs >= (strad ? thr_at(sI) : ifix) &&
                        tot - pm >= (strad ? thr_at(argmax_bins(h, off, mj + 1, e)) : ifix)) {
                        emit(cs, mj, sI);
                        cs = mj + 1;
                        pcs = pm;
                        bM = aM;
                        bI = aI;
                    }
                    up = 1;
                    M = hk;
                }
            }
        }
    }
    const bool last = tot - pcs >= (strad ? thr_at(bI) : ifix);
    if (last)
        emit(cs, e, bI);
    if (!WRITE) {
        o.nsplit = count - (last ? 1 : 0);
        o.fin_peak = last ? bI : -1;
    }
    return count;
}

// Write the clusters of one proto-cluster recorded by walk_proto<false>
// from index `first`; the caller re-walks with WRITE when o.nsplit > 4.
__device__ __forceinline__ void write_walk(const WalkOut &o, int s, int e, short *clo, short *chi, short *cpk, int cap,
                                           int first)
{
    int lo = s, q = first;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < o.nsplit) {
            const int hi = (int)(o.rec[k] & 0xFFFFu);
            if (q < cap) {
                clo[q] = (short)lo;
                chi[q] = (short)hi;
                cpk[q] = (short)(o.rec[k] >> 16);
            }
            ++q;
            lo = hi + 1;
        }
    }
    if (o.fin_peak >= 0 && q < cap) {
        clo[q] = (short)lo;
        chi[q] = (short)e;
        cpk[q] = (short)o.fin_peak;
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.3, x86 variant: a range is cut at the smallest significant minimum
// between its two largest maxima, and each part the same way, recursively
// (its extrema found anew within the part).  The maxima are the highest bins
// of the segments between consecutive significant minima; of equal maxima the
// lower z counts as larger, of equal minima the lower z is taken; the cut bin
// stays with the left part; a cut needs both parts to reach the integral
// threshold of their region.  h[k + off] is bin k.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int thr_of(int peak, const KParams &p)
{
    return (peak < p.gas_bin) ? p.min_int_gas : p.min_int_pp;
}

// cut bin of [lo, hi], or -1
__device__ __forceinline__ int recursive_cut(const int *h, int off, const KParams &p, int lo, int hi)
{
    // walk 1: the two largest segment maxima
    int up = 1, M = 0, m = 0, mj = lo;
    int segM = INT_MIN, segI = lo, aM = INT_MIN, aI = lo;
    int b1M = INT_MIN, b1I = -1, b2M = INT_MIN, b2I = -1, nseg = 0;
    for (int k = lo; k <= hi + 1; ++k) {
        if (k == hi + 1) {   // close the last segment
            ++nseg;
            const bool top = segM > b1M;
            const bool second = !top && segM > b2M;
            b2M = top ? b1M : (second ? segM : b2M);
            b2I = top ? b1I : (second ? segI : b2I);
            b1M = top ? segM : b1M;
            b1I = top ? segI : b1I;
            break;
        }
        const int hk = h[k + off];
        if (k == lo) {
            M = hk;
            segM = hk;
            segI = k;
        } else if (up) {
            if (hk > M)
                M = hk;
            if (hk > segM) {
                segM = hk;
                segI = k;
            }
            if (hk <= M - p.dip_prom) {
                up = 0;
                m = hk;
                mj = k;
                aM = INT_MIN;
            }
        } else if (hk < m) {
            m = hk;
            mj = k;
            aM = INT_MIN;
        } else if (hk >= m + p.dip_prom) {
            ++nseg;
            const bool top = segM > b1M;
            const bool second = !top && segM > b2M;
            b2M = top ? b1M : (second ? segM : b2M);
            b2I = top ? b1I : (second ? segI : b2I);
            b1M = top ? segM : b1M;
            b1I = top ? segI : b1I;
            // the new segment: bins (mj, k]
            segM = aM;
            segI = aI;
            if (hk > segM) {
                segM = hk;
                segI = k;
            }
            up = 1;
            M = hk;
        } else if (hk > aM) {
            aM = hk;
            aI = k;
        }
    }
    if (nseg < 2)
        return -1;
    const int p1 = min(b1I, b2I), p2 = max(b1I, b2I);
    // walk 2: the smallest significant minimum strictly between them
    int cut = -1, cutv = INT_MAX;
    up = 1;
    for (int k = lo; k <= p2; ++k) {
        const int hk = h[k + off];
        if (k == lo) {
            M = hk;
        } else if (up) {
            if (hk > M) {
                M = hk;
            } else if (hk <= M - p.dip_prom) {
                up = 0;
                m = hk;
                mj = k;
            }
        } else if (hk < m) {
            m = hk;
            mj = k;
        } else if (hk >= m + p.dip_prom) {
            if (mj > p1 && mj < p2 && m < cutv) {
                cut = mj;
                cutv = m;
            }
            up = 1;
            M = hk;
        }
    }
    if (cut < 0)
        return -1;
    if (sum_bins(h, off, lo, cut) < thr_of(argmax_bins(h, off, lo, cut), p) ||
        sum_bins(h, off, cut + 1, hi) < thr_of(argmax_bins(h, off, cut + 1, hi), p))
        return -1;
    return cut;
}

// Clusters of proto-cluster [s, e] in z order: each leaf is found by
// descending from the whole range towards the first bin not yet covered (no
// stack: the cuts are recomputed, each step shrinks the range, and each leaf
// advances the position).  With WRITE they go to clo / chi / cpk from index
// `first` (below `cap`).  Returns their number.
template <bool WRITE>
__device__ __forceinline__ int walk_recursive(const int *h, int off, const KParams &p, int s, int e, short *clo,
                                              short *chi, short *cpk, int cap, int first)
{
    int count = 0;
    for (int pos = s; pos <= e;) {
        int lo = s, hi = e;
        for (;;) {
            const int cut = recursive_cut(h, off, p, lo, hi);
            if (cut < 0)
                break;
            if (pos <= cut)
                hi = cut;
            else
                lo = cut + 1;
        }
        const int pk = argmax_bins(h, off, lo, hi);
        if (sum_bins(h, off, lo, hi) >= thr_of(pk, p)) {
            if (WRITE) {
                const int q = first + count;
                if (q < cap) {
                    clo[q] = (short)lo;
                    chi[q] = (short)hi;
                    cpk[q] = (short)pk;
                }
            }
            ++count;
        }
        pos = hi + 1;
    }
    return count;
}

// centre of bin i, z_i of Eq. 4; the fit's frame is anchored there because
// z_i is exact in binary32 for the usual ranges while z_seed is not
__device__ __forceinline__ float bin_centre(int i, const KParams &p)
{
    return p.z_min + ((float)i + 0.5f) * p.dz;
}

__device__ __forceinline__ int lower_bound_bins(const int *pb, int n, int bin)
{
    int lo = 0, hi = n - 1;   // pb[n-1] >= every bin
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pb[mid] >= bin)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// 3x3 covariance C = A^-1 for A = [[a, 0, -b], [0, a, -c], [-b, -c, d]] (Eq. 14).
template <typename T>
__device__ __forceinline__ T inverse_a(T a, T b, T c, T d, T out[6])
{
    const T D = a * d - b * b - c * c;
    const T det = a * D;
    const T r = T(1) / det;
    out[0] = (a * d - c * c) * r;   // xx
    out[1] = (b * c) * r;           // xy
    out[2] = (a * d - b * b) * r;   // yy
    out[3] = (a * b) * r;           // xz
    out[4] = (a * c) * r;           // yz
    out[5] = (a * a) * r;           // zz
    return det;
}

// C = J C' J^T for x = e_x + t_x z, y = e_y + t_y z: the covariance of
// (x, y, z) from that of (e_x, e_y, z) (packed xx, xy, yy, xz, yz, zz).
template <typename T>
__device__ __forceinline__ void map_covariance(const T cp[6], T tx, T ty, T c[6])
{
    c[5] = cp[5];
    c[3] = cp[3] + tx * cp[5];
    c[4] = cp[4] + ty * cp[5];
    c[0] = cp[0] + tx * (T(2) * cp[3] + tx * cp[5]);
    c[1] = cp[1] + tx * (cp[4] + ty * cp[5]) + ty * cp[3];
    c[2] = cp[2] + ty * (T(2) * cp[4] + ty * cp[5]);
}

// Covariance of a fitted vertex (Eq. 14).  The fit works with a reference
// slope t_ref (the mean of its tracks' slopes): unknowns e = (x, y) - z t_ref
// and slopes t - t_ref, whose normal matrix A' has a = s0, b = sx', c = sy',
// d = szz'.  C' = A'^-1 is mapped back to (x, y, z).  The 1-norm condition
// number is that of the normal matrix A of (x, y, z) (b = sx' + s0 t_x,
// c = sy' + s0 t_y, d = szz' + 2 t_ref . s' + s0 |t_ref|^2); above `cond`
// the inversion and the map are redone in binary64 (the return value).
__device__ __forceinline__ bool vertex_covariance(float la, float lb, float lc, float ld, float trx, float try_,
                                                  float cond, float cf[6])
{
    float cp[6];
    const float det = inverse_a<float>(la, lb, lc, ld, cp);
    map_covariance<float>(cp, trx, try_, cf);
    const float b = fmaf(la, trx, lb), c = fmaf(la, try_, lc);
    const float d = fmaf(la, fmaf(trx, trx, try_ * try_), fmaf(2.0f, fmaf(trx, lb, try_ * lc), ld));
    const float na = fmaxf(fmaxf(la + fabsf(b), la + fabsf(c)), fabsf(b) + fabsf(c) + d);
    const float ni = fmaxf(fmaxf(fabsf(cf[0]) + fabsf(cf[1]) + fabsf(cf[3]), fabsf(cf[1]) + fabsf(cf[2]) + fabsf(cf[4])),
                           fabsf(cf[3]) + fabsf(cf[4]) + fabsf(cf[5]));
    if (!(det > 0.0f) || !(na * ni <= cond)) {
        double cd[6], cm[6];
        inverse_a<double>((double)la, (double)lb, (double)lc, (double)ld, cd);
        map_covariance<double>(cd, (double)trx, (double)try_, cm);
        for (int q = 0; q < 6; ++q)
            cf[q] = (float)cm[q];
        return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Sec. 3.5: Newton-Raphson fit of every live vertex, L lanes per vertex.
// Each lane keeps up to kRegTracks of its vertex's tracks in registers for
// all iterations (the rest, if any, is re-read from LDS each iteration).
// ---------------------------------------------------------------------------
constexpr int kRegTracks = 5;

// The step needs no sum of the weights w alone: it is zero exactly when every
// w * (1 / V_x) is, i.e. when s0 is, and s0 <= 0 already fails the step.
struct FitSums {
    float s0, sx, sy, szz, gx, gy, gz;
};

__device__ __forceinline__ void accumulate(FitSums &a, float X, float Y, float tx, float ty, float wt, float dx,
                                           float dy, float dz, const KParams &p)
{
    // residual (Eq. 9) relative to the frame origin, chi2 (Eq. 7), Tukey weight
    // (Eq. 17; zero beyond chi2_max, where the terms below add exact zeros)
    const float rx = fmaf(dz, tx, X) - dx;
    const float ry = fmaf(dz, ty, Y) - dy;
    const float chi2 = wt * fmaf(rx, rx, ry * ry);
    const float u = (chi2 < p.chi2_max) ? fmaf(-chi2, p.inv_chi2_max, 1.0f) : 0.0f;
    const float w = u * u;
    const float ww = w * wt;
    a.s0 += ww;
    a.sx = fmaf(ww, tx, a.sx);
    a.sy = fmaf(ww, ty, a.sy);
    a.szz = fmaf(ww, fmaf(tx, tx, ty * ty), a.szz);
    const float px = ww * rx, py = ww * ry;
    a.gx += px;
    a.gy += py;
    a.gz = fmaf(px, tx, fmaf(py, ty, a.gz));
}

// Eq. 18 weight for a track of chi2 relative to this candidate, whose terms
// for the other candidates (at their seeds) sum to `oth`; e_max =
// exp(-chi2_max / 2).  No cut: far tracks fade out smoothly.
__device__ __forceinline__ float mv_weight(float chi2, float oth, const KParams &p)
{
    const float ex = __expf(-0.5f * chi2);
    return ex * __builtin_amdgcn_rcpf(p.e_max_mv + ex + oth);
}

__device__ __forceinline__ void accumulate_mv(FitSums &a, float X, float Y, float tx, float ty, float wt, float oth,
                                              float dx, float dy, float dz, const KParams &p)
{
    const float rx = fmaf(dz, tx, X) - dx;
    const float ry = fmaf(dz, ty, Y) - dy;
    const float chi2 = wt * fmaf(rx, rx, ry * ry);
    const float ww = mv_weight(chi2, oth, p) * wt;
    a.s0 += ww;
    a.sx = fmaf(ww, tx, a.sx);
    a.sy = fmaf(ww, ty, a.sy);
    a.szz = fmaf(ww, fmaf(tx, tx, ty * ty), a.szz);
    const float px = ww * rx, py = ww * ry;
    a.gx += px;
    a.gy += py;
    a.gz = fmaf(px, tx, fmaf(py, ty, a.gz));
}

// Multi-vertex pre-cut (Sec. 5) of a track for the candidate whose peak-bin
// centre is zr and seed offset d0: the track's fit frame values (position at
// zr relative to the beamline point there, 1 / V_x of Eq. 2 at the seed) and
// its chi2 at the seed (Eq. 7, Eq. 9).  Written out in binary32 with explicit
// fused multiply-adds: the pre-cut is an integer decision, the same for the
// same inputs on every run and schedule.
struct MvPre {
    float X, Y, WT, chi2;
};

__device__ __forceinline__ MvPre mv_precut(const float t[8], float zr, float d0, const KParams &p)
{
    const float x = t[0], y = t[1], z = t[2], tx = t[3], ty = t[4];
    const float dzr = zr - z;
    MvPre m;
    m.X = fmaf(dzr, tx, x) - (p.bx + p.btx * zr);
    m.Y = fmaf(dzr, ty, y) - (p.by + p.bty * zr);
    const float dzs = dzr + d0;
    const float V = fmaf(dzs, fmaf(dzs, t[7], 2.0f * t[6]), t[5]);
    // hardware reciprocal (within 1 ulp): this runs for every (track,
    // candidate) pair, twice, and a cut decision it could move lies far inside
    // the binary64 oracle's tie band
    m.WT = (V > 0.0f && isfinite(V)) ? __builtin_amdgcn_rcpf(V) : 0.0f;
    const float rx = fmaf(d0, tx, m.X) - p.btx * d0;
    const float ry = fmaf(d0, ty, m.Y) - p.bty * d0;
    m.chi2 = m.WT * fmaf(rx, rx, ry * ry);
    return m;
}

// The z range outside which a track cannot pass the pre-cut at any seed on
// the beamline.  The pre-cut's residual is affine in the seed's z, with the
// slope difference dt to the beamline, and its length is smallest at z_poca
// (Eq. 1), so |r(z_s)|^2 >= |dt|^2 (z_s - z_poca)^2; when the covariance is
// positive semi-definite, V_x(z_s) of Eq. 2 is at most
// (sigma_x + |z_s - z| sigma_tx)^2.  chi2 < cut then needs
// |z_s - z_poca| < s (sigma_x + |z_poca - z| sigma_tx) / (|dt| - s sigma_tx),
// s = sqrt(cut).  The bound is widened by 0.2 % and 1 micrometre, far above
// its binary32 rounding, so a seed outside the range fails the cut by a wide
// margin.  Tracks without a finite bound get the whole axis.
__device__ __forceinline__ void mv_window(const float t[8], const KParams &p, float &zlo, float &zhi)
{
    zlo = -INFINITY;
    zhi = INFINITY;
    const float dtx = t[3] - p.btx, dty = t[4] - p.bty;
    const float den = fmaf(dtx, dtx, dty * dty);
    const float vxx = t[5], vxtx = t[6], vtxtx = t[7];
    if (!(den > 0.0f) || !(vxx > 0.0f) || !(vtxtx >= 0.0f) || !(vxtx * vxtx <= vxx * vtxtx) || !isfinite(den) ||
        !isfinite(vxx) || !isfinite(vtxtx))
        return;
    // hardware square roots and reciprocals (1 ulp): the widening covers them
    const float zp = t[2] + fmaf(dtx, p.bx - t[0], dty * (p.by - t[1])) * __builtin_amdgcn_rcpf(den);
    const float s = 1.001f * __builtin_amdgcn_sqrtf(p.chi2_window_mv);
    const float stx = __builtin_amdgcn_sqrtf(vtxtx);
    const float g = __builtin_amdgcn_sqrtf(den) - s * stx;
    if (!(g > 0.0f) || !isfinite(zp))
        return;
    const float A =
        fmaf(1.001f * s, fmaf(fabsf(zp - t[2]), stx, __builtin_amdgcn_sqrtf(vxx)) * __builtin_amdgcn_rcpf(g), 1e-3f);
    if (!isfinite(A))
        return;
    zlo = zp - A;
    zhi = zp + A;
}

// Stage boundaries for the per-stage cycle counters of the debug variant.
struct Stamps {
    unsigned long long t[9];
};

template <bool DEBUG>
__device__ __forceinline__ void stamp(Stamps &st, int k)
{
    if (DEBUG)
        st.t[k] = clock64();
}

}  // namespace pvk
