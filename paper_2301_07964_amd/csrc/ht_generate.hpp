// ht_generate.hpp -- generate phase of blocked stage two (Section 3.2,
// "Generating the reflectors"; generate algorithm of the appendix).
//
// One workgroup (256 threads, 4 wavefronts) per sweep of the group
// j1..j2 (q <= r sweeps) and two helper workgroups per sweep (the far rows of
// H and of T); sweep w is workgroup 3w and its helpers 3w+1 (H) and 3w+2 (T),
// so every wait is on a workgroup with a lower index (forward progress needs
// no co-residency: workgroups are dispatched in index order).  Sweep j processes blocks k = 0..kext-1 in
// order; block (j,k) starts once sweep j-1 has finished block k+2 (progress
// flags in device memory, agent-scope release/acquire).  Steps that run
// concurrently touch disjoint columns of the scratch band, so no other
// synchronisation is needed.
//
// Every wait is bounded (GenArgs::wait_limit polls).  A wait that gives up
// sets the timeout bit in the device status word and publishes -1 in its own
// counter; a waiter that sees -1 gives up at once.  So every workgroup of the
// launch exits normally and the host learns of the failure from the status
// word (the output of that call is then invalid).
//
// Work of step (j,k), on the scratch band copy of H and T:
//   1. lazy left updates: the left reflectors of block k of the earlier sweeps
//      of the group are applied to the column of H that this step reduces
//      (jb) and to the column of T that enters its diagonal block (i1+r-1),
//      all at once in compact WY form, Q^H x = x - V T^H V^H x (each sweep
//      adds its column of T while its workgroup factors the T block);
//      blocks with fewer than two rows still perform these updates;
//   2. left reflector from H(i1:i2, jb) (xLARFG convention), applied to the
//      diagonal block T(i1:i2, i1:i2);
//   3. RQ factorisation of that block (Householder, last row first, with the
//      identity appended so that the first row of the orthogonal factor comes
//      out of the same rank-one updates), direction normalised to a real
//      positive first nonzero entry, then the opposite reflector by xLARFG;
//   4. eager right updates: H rows topH..i3 and T rows topT..i2 of columns
//      i1..i2, where topH = max(j1+1, j1+1+(k+1-d) r), topT = max(j1+1,
//      j1+1+(k-d) r), d = j2-j (T is skipped for the last sweep).
// Reflectors (v, tau) are stored, zero padded to r entries, for the delayed
// updates; tau = 0 marks a block that does not exist for that sweep.
//
// Latency is what matters here (the q workgroups form a pipeline whose pace
// is set by the slowest step), so the two long loops keep their rows in
// registers, with the block order RM >= r a compile-time constant: the RQ runs
// in one wavefront, lane l holding row l of the block and lane 32+l row l of
// the accumulated orthogonal factor, so that a step of the factorisation
// only broadcasts the pivot row; the eager right updates load a whole row
// segment before they write any of it back.  The kernel is also kept small:
// indices are 32-bit (band offsets stay below 2^31 for every n the library
// accepts: n * ldb elements), loops over steps are not unrolled, and each
// piece of work has one copy in the code, so that a workgroup's step loop
// stays within the instruction cache.
#pragma once
#include "ht_common.hpp"

namespace ht {

template <class S>
struct GenArgs {
    int64_t n, r, j1, j2, kext;
    Band band;
    S *SH, *ST;        // scratch band copies of H and T
    S *VL, *TL;        // left reflectors:  VL[((w*kext)+k)*r + i], TL[w*kext + k]
    S *VR, *TR;        // right reflectors
    S *TF;             // per (sweep w, block k): column w of the triangular factor of the compact WY
                       // form of the left reflectors of block k of sweeps j1..j1+w, TF[(w*kext+k)*kMaxR + i]
    int *progress;     // per sweep of the group: blocks whose step chain is finished (-1: gave up)
    int *hdone;        // per sweep: blocks whose far rows of H (hdone[w]) and of T (hdone[q+w]) are finished
    int *status;       // device status word: kStatus* bits, OR-ed in by a wait that gives up
    int64_t wait_limit;  // polls before a wait gives up (0: give up without polling)
    const int *flags;  // lookahead: per tile of 16 columns, raised by the previous group's left pass once the
                       // tile's scratch band is written; nullptr: the band is complete at launch
    int flag_need;     // value of a flag whose tile is ready
    int ntiles;        // number of tiles (ceil(n / 16))
};

// status bits of the device status word
constexpr int kStatusWaitTimeout = 1;
constexpr int kGaveUp = -1;           // counter value published by a workgroup that gave up
constexpr int kAllDone = 0x3fffffff;  // counter value after the last step

template <class S> __device__ inline S shfl_(S v, int src);
template <> __device__ inline double shfl_<double>(double v, int src) { return __shfl(v, src, 64); }
template <> __device__ inline zd shfl_<zd>(zd v, int src) { return mk<zd>(__shfl(v.re, src, 64), __shfl(v.im, src, 64)); }

__device__ inline void st_release(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int ld_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait of one thread until *c1 >= need1, *c2 >= need2 and
// *c3 >= need3 (c2, c3 may be null).  The counters are polled with relaxed
// loads (an acquiring load would invalidate the cache of the whole XCD at
// every poll); the caller issues one agent-scope acquire fence once the wait
// has succeeded, which orders its later loads after the releases it observed.
// Returns false when a counter holds kGaveUp (a predecessor gave up) or after
// `limit` polls (then the timeout bit is OR-ed into *status).  The poll count
// is tested before the counters are read, so limit 0 gives up without reading
// them.
__device__ inline bool bounded_wait(const int *c1, int need1, const int *c2, int need2, const int *c3, int need3,
                                    int64_t limit, int *status)
{
    for (int64_t polls = 0;; ++polls) {
        if (polls >= limit) {
            __hip_atomic_fetch_or(status, kStatusWaitTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        const int v1 = ld_relaxed(c1), v2 = c2 ? ld_relaxed(c2) : need2, v3 = c3 ? ld_relaxed(c3) : need3;
        if (v1 == kGaveUp || v2 == kGaveUp || v3 == kGaveUp) return false;
        if (v1 >= need1 && v2 >= need2 && v3 >= need3) return true;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Bounded wait of one wavefront (lane = lane index) until the tiles t0..tneed
// of the scratch band are ready (flags[t] >= need).  Lane l polls tile t0+l;
// every poll takes the whole run of ready tiles that starts at t0, so one
// wait usually covers many later steps.  Returns the first tile not known to
// be ready (> tneed), or -1 after `limit` polls (timeout bit OR-ed into
// *status).  Like bounded_wait, the caller issues the acquire fence.
__device__ inline int tiles_wait(const int *flags, int t0, int tneed, int ntiles, int need, int lane, int64_t limit,
                                 int *status)
{
    for (int64_t polls = 0;; ++polls) {
        if (polls >= limit) {
            if (lane == 0) __hip_atomic_fetch_or(status, kStatusWaitTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        const int t = t0 + lane;
        const bool ok = t >= ntiles || ld_relaxed(flags + t) >= need;
        const unsigned long long nr = ~__ballot(ok);
        t0 = min(ntiles, t0 + (nr ? __ffsll((long long)nr) - 1 : 64));
        if (t0 > tneed) return t0;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Householder generation in one wavefront.  Lane l holds x_l (l < m).
// Returns v_l (v_0 = 1), tau and beta in every lane.
template <class S>
__device__ inline void wave_larfg(S x, int lane, int m, S &v, S &tau, S &beta) {
    const S alpha = bcast(x, 0);
    double ss = wave_sum((lane >= 1 && lane < m) ? abs2(x) : 0.0);
    if (ss == 0.0 && im(alpha) == 0.0) {
        tau = zero<S>();
        beta = alpha;
        v = (lane == 0) ? one<S>() : x;
        return;
    }
    double b;
    S sc;
    larfg_core(alpha, ss, tau, b, sc);
    beta = mk<S>(b, 0.0);
    v = (lane == 0) ? one<S>() : mul(x, sc);
}

// Householder RQ of the m x m block held row-wise by one wavefront: lane l < m
// holds row l of the block in x[0..m-1], lane 32 + l row l of Y (on entry the
// identity).  Rows are processed from the last (step i annihilates entries
// 0..i-1 of row i with a reflector acting on columns 0..i, xLARFG convention),
// every reflector is applied to the block rows and to Y, so that on exit
// Y = Q^H and column 0 of Y (x[0] of lanes 32..32+m-1) is the first row of
// the orthogonal RQ factor, conjugated.  The pivot row is broadcast into
// scalar registers; each lane's product with it is formed while the norm,
// square root and divisions of the reflector are in flight.
template <class S, int RM>
__device__ inline void rq_rows(S (&x)[RM], int m)
{
#pragma unroll
    for (int i = RM - 1; i >= 1; --i) {
        if (i >= m) continue;
        S b[RM];
#pragma unroll
        for (int c = 0; c <= i; ++c) b[c] = conj_(bcast(x[c], i));
        // p = sum_{c<i} x_c b_c (per lane); in the pivot lane i, whose row b
        // is (conjugated), that sum is ||b_{0..i-1}||^2, real: the norm comes
        // from there instead of a second sum over the broadcast row
        // eight partial sums: the sum is on the critical path of the step
        S pa[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) pa[e] = zero<S>();
#pragma unroll
        for (int c = 0; c < i; ++c) pa[c & 7] = add(pa[c & 7], mul(x[c], b[c]));
        const S pp = add(add(add(pa[0], pa[1]), add(pa[2], pa[3])), add(add(pa[4], pa[5]), add(pa[6], pa[7])));
        const S alpha = b[i];
        const double ss = bcast(re(pp), i);
        if (ss == 0.0 && im(alpha) == 0.0) continue;              // tau = 0: identity
        S tau, sc;                                               // u_c = b_c sc (c < i), u_i = 1
        double bb;
        larfg_core(alpha, ss, tau, bb, sc);
        // s = (x_i + sum_{c<i} x_c u_c) tau;  x_c -= s conj(u_c) = (s conj(sc)) conj(b_c)
        const S sv = mul(add(x[i], mul(pp, sc)), tau);
        const S t = mul(sv, conj_(sc));
#pragma unroll
        for (int c = 0; c < i; ++c) x[c] = sub(x[c], mul(t, conj_(b[c])));
        x[i] = sub(x[i], sv);
    }
}

// 32-bit offsets into the band copy: element (i, c) (0-based) at
// (i - c + BU) + c * ldb.
struct Band32 {
    int BU, ldb;
    __device__ inline int idx(int i0, int c0) const { return (i0 - c0 + BU) + c0 * ldb; }
};

// The far rows of one step in one pass: rows [top, top+nrow) (1-based) of the
// band copy X in the block's columns i1 .. i1+m-1, X <- X (I - sig w w^H), the
// first column of the rows from zrow on written as exact zeros (T's column i1
// below the diagonal); each thread loads U row segments before it writes any,
// so U rounds of loads are in flight together.
template <class S, int RM, int U>
__device__ __forceinline__ void far_rows(S *X, const Band32 &B, int top, int nrow, int i1, int m, const S *sw,
                                         S sig, int tid, int zrow)
{
    const int cs = B.ldb - 1;                      // stride between the columns of one band row
    for (int e0 = tid; e0 < nrow; e0 += 256 * U) {
        S x[U][RM];
        int off[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + 256 * u;
            off[u] = e < nrow ? B.idx(top + e - 1, i1 - 1) : -1;
#pragma unroll
            for (int c = 0; c < RM; ++c) {
                x[u][c] = zero<S>();
                if (off[u] >= 0 && c < m) x[u][c] = X[off[u] + c * cs];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            S d0 = zero<S>(), d1 = zero<S>();
#pragma unroll
            for (int c = 0; c < RM; c += 2) {
                d0 = add(d0, mul(x[u][c], sw[c]));
                d1 = add(d1, mul(x[u][c + 1], sw[c + 1]));
            }
            const S sx = mul(add(d0, d1), sig);
            const bool zr = top + e0 + 256 * u >= zrow;
#pragma unroll
            for (int c = 0; c < RM; ++c)
                if (off[u] >= 0 && c < m) X[off[u] + c * cs] = (c == 0 && zr) ? zero<S>() : sub(x[u][c], mul(sx, conj_(sw[c])));
        }
    }
}

// Helper workgroups of sweep w: the "far" part of each step's eager right
// update, behind the sweep's own workgroup.  Step k's right reflector is
// applied by helper part 0 to rows topH .. j1+(k+1)r of H and by helper part 1
// (for all but the last sweep) to rows topT .. i2 of T in the block's columns,
// with the exact zeros of T's column i1 below the diagonal.  The two parts
// touch different matrices, about (q-1-w) r rows each.  The sweep's own
// workgroup has done the rows of H from j1+(k+1)r+1 on, the only ones its next
// steps read; the successor sweep waits for all three counters.
template <class S, int RM>
__device__ __forceinline__ void gen_far(const GenArgs<S> &a, int w, int part)
{
    const int tid = threadIdx.x;
    const int n = (int)a.n, r = (int)a.r, j1 = (int)a.j1, j2 = (int)a.j2, kext = (int)a.kext;
    const int j = j1 + w, d = j2 - j;
    const int nbj = (int)nblocks(n, r, j);
    const Band32 B{(int)a.band.BU, (int)a.band.ldb};
    const int q = j2 - j1 + 1;
    int *mine = a.hdone + part * q + w;
    S *X = part == 0 ? a.SH : a.ST;
    __shared__ int s_go;
    __shared__ S hsw[64];
    __shared__ S hsig;
    for (int k = 0; k < kext; ++k) {
        if (tid == 0) {
            s_go = bounded_wait(a.progress + w, k + 1, nullptr, 0, nullptr, 0, a.wait_limit, a.status) ? 1 : 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (!s_go) {                                // uniform: the sweep's workgroup gave up, or this wait did
            if (tid == 0) st_release(mine, kGaveUp);
            return;
        }
        if (k < nbj) {
            const int i1 = j + k * r + 1;
            const int i2 = min(j + (k + 1) * r, n);
            const int m = i2 - i1 + 1;
            if (tid < 64) hsw[tid] = tid < m ? a.VR[(w * kext + k) * r + tid] : zero<S>();
            if (tid == 0) hsig = a.TR[w * kext + k];
            __syncthreads();
            const S sig = hsig;
            const bool tdo = d >= 1 && !iszero(sig);
            int top = 0, nrow = 0;
            if (part == 0 && !iszero(sig)) {
                top = max(j1 + 1, j1 + 1 + (k + 1 - d) * r);
                nrow = max(top, j1 + (k + 1) * r + 1) - top;
            } else if (part == 1 && tdo) {
                top = max(j1 + 1, j1 + 1 + (k - d) * r);
                nrow = i2 - top + 1;
            }
            constexpr int U = sizeof(S) * RM <= 256 ? 2 : 1;     // two rows per thread while registers allow
            if (nrow > 0)
                far_rows<S, RM, U>(X, B, top, nrow, i1, m, hsw, sig, tid, part == 1 ? i1 + 1 : 0x7fffffff);
            if (part == 1 && !tdo)
                for (int e = tid; e < m - 1; e += 256) a.ST[B.idx(i1 + e, i1 - 1)] = zero<S>();
        }
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            st_release(mine, k + 1);
        }
    }
    __syncthreads();
    if (tid == 0) st_release(mine, kAllDone);
}

// Row stride of the staged reflectors and WY columns in LDS: a lane that
// walks its own row (lazy_wy, wy_column) would otherwise hit the same bank as
// every other lane (a stride of 32 doubles is 64 banks).
constexpr int kLS = kMaxR + 1;

// Stage the left reflectors V (v_s at lv[s*kLS ..]) and the columns of their
// WY factor T (column s at lT[s*kLS ..]) of block kk of the earlier sweeps
// s < nw into LDS, by NG groups of 32 threads (thread t: group t / 32, entry
// t % 32; r <= 32): all loads are issued before any is stored, so they are in
// flight together.
template <class S, int NG>
__device__ __forceinline__ void stage_lazy(const GenArgs<S> &a, int kk, int nw, S *lv, S *lT, int t)
{
    const int r = (int)a.r, kext = (int)a.kext;
    const int g = t >> 5, c = t & 31;
    constexpr int NS = kMaxR / NG;                 // sweeps per group
    S tv[NS], tt[NS];
#pragma unroll
    for (int it = 0; it < NS; ++it) {
        const int sw = g + NG * it;
        tv[it] = zero<S>();
        tt[it] = zero<S>();
        if (sw < nw) {
            if (c < r) tv[it] = a.VL[(sw * kext + kk) * r + c];
            tt[it] = a.TF[(sw * kext + kk) * kMaxR + c];
        }
    }
#pragma unroll
    for (int it = 0; it < NS; ++it) {
        const int sw = g + NG * it;
        if (sw < nw) {
            if (c < r) lv[sw * kLS + c] = tv[it];
            lT[sw * kLS + c] = tt[it];
        }
    }
}

// Q^H x for Q = G_0 ... G_{nw-1} = I - V T V^H, the compact WY form of the
// left reflectors of one block of the earlier sweeps (G_i = I - tau_i v_i
// v_i^H, v_i on rows base+i .. base+i+r-1): x <- x - V (T^H (V^H x)), equal
// to applying G_0^H, G_1^H, ... in turn.  Two wavefronts share one column
// (half = 0 holds x, lane l the entry of row base+l; half = 1 helps): each
// forms half of every sum of the three products (the terms t < (r+1)/2 or
// the rest of V^H x, the terms of one parity of T^H z and of V u), so the
// dependent chains are half as long.  Called by all four wavefronts of the
// workgroup (the H column on wavefronts 0 and 2, the T column on 1 and 3)
// with the workgroup's barriers between the products; act: this column
// takes part.  lv, lT as staged by stage_lazy; ws: this column's LDS scratch
// of 384 values.  Returns the result in the lanes of half 0.
template <class S>
__device__ __forceinline__ S lazy_wy(S x, int lane, int half, bool act, int nw, int r, const S *lv, const S *lT,
                                     S *ws)
{
    S *xs = ws, *zp = ws + 64, *up = ws + 128, *ap = ws + 192;   // zp, up: [2][32]; ap: [2][64]
    if (half == 0) xs[lane] = x;
    __syncthreads();
    S z0 = zero<S>(), z1 = zero<S>();              // z_i = v_i^H x   (lane i < nw), half of the terms
    if (act && lane < nw) {
        const int hr = (r + 1) >> 1, t0 = half ? hr : 0, t1 = half ? r : hr;
        for (int t = t0; t < t1; t += 2) {
            z0 = add(z0, cmul(lv[lane * kLS + t], xs[lane + t]));
            if (t + 1 < t1) z1 = add(z1, cmul(lv[lane * kLS + t + 1], xs[lane + t + 1]));
        }
    }
    if (lane < 32) zp[half * 32 + lane] = add(z0, z1);
    __syncthreads();
    S u0 = zero<S>();                              // u = T^H z, the terms jj of parity `half`
    if (act && lane < nw)
        for (int jj = half; jj <= lane; jj += 2) u0 = add(u0, cmul(lT[lane * kLS + jj], add(zp[jj], zp[32 + jj])));
    if (lane < 32) up[half * 32 + lane] = u0;
    __syncthreads();
    S a0 = zero<S>();                              // V u, the terms i of parity `half`
    if (act) {
        const int ilo = max(0, lane - r + 1), ihi = min(nw - 1, lane);
        for (int i = ilo + ((ilo ^ half) & 1); i <= ihi; i += 2)
            a0 = add(a0, mul(lv[i * kLS + (lane - i)], add(up[i], up[32 + i])));
    }
    ap[half * 64 + lane] = a0;
    __syncthreads();
    return sub(x, add(ap[lane], ap[64 + lane]));
}

// Column nw of the WY factor T for the reflectors of block k of sweeps
// 0..nw: T(0:nw-1, nw) = -tau T(0:nw-1, 0:nw-1) V^H v, T(nw, nw) = tau
// (v = sv, the new reflector, on rows base+nw ..; lv, lT as in lazy_wy).
// One wavefront; written to out[0..nw].
template <class S>
__device__ __forceinline__ void wy_column(int lane, int nw, int r, int m, const S *lv, const S *lT, const S *sv,
                                         S tau, S *ws, S *out)
{
    S *zs = ws;
    S z0 = zero<S>(), z1 = zero<S>();              // z_i = v_i^H v  (lane i < nw); row of v: e = i + t - nw
    if (lane < nw) {
        const int tlo = nw - lane, thi = min(r - 1, nw - lane + m - 1);
        for (int t = tlo; t <= thi; t += 2) {
            z0 = add(z0, cmul(lv[lane * kLS + t], sv[lane + t - nw]));
            if (t + 1 <= thi) z1 = add(z1, cmul(lv[lane * kLS + t + 1], sv[lane + t + 1 - nw]));
        }
    }
    if (lane < 32) zs[lane] = add(z0, z1);
    __builtin_amdgcn_wave_barrier();
    if (lane < nw) {
        S c0 = zero<S>(), c1 = zero<S>();
        for (int jj = lane; jj < nw; jj += 2) {
            c0 = add(c0, mul(lT[jj * kLS + lane], zs[jj]));
            if (jj + 1 < nw) c1 = add(c1, mul(lT[(jj + 1) * kLS + lane], zs[jj + 1]));
        }
        out[lane] = sub(zero<S>(), mul(tau, add(c0, c1)));
    }
    if (lane == nw) out[nw] = tau;
}

template <class S, int RM>
__global__ __launch_bounds__(256) void k_generate(GenArgs<S> a)
{
    const int role = (int)(blockIdx.x % 3);
    const int w = (int)(blockIdx.x / 3);
    if (role != 0) {                               // far-row helpers of sweep w: H (1), T (2)
        gen_far<S, RM>(a, w, role - 1);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = (int)a.n, r = (int)a.r, j1 = (int)a.j1, j2 = (int)a.j2, kext = (int)a.kext;
    const int j = j1 + w;
    const int nw = w;                              // earlier sweeps of the group
    const int nbj = (int)nblocks(n, r, j);
    const int d = j2 - j;
    const int q = j2 - j1 + 1;
    const Band32 B{(int)a.band.BU, (int)a.band.ldb};
    const int cs = B.ldb - 1;                      // stride between the columns of one band row
    S *SH = a.SH, *ST = a.ST;

    constexpr int LB = 33;                       // LDS leading dimension of 32x32 blocks
    constexpr int CP = RM / 4;                   // near rows: columns per lane (four lanes per row)
    __shared__ S sv[64], sw[64];
    __shared__ S blk[32 * LB];
    __shared__ S stau[4];
    __shared__ S lzv[2][kMaxR * kLS];            // staged lazy reflectors, by block parity
    __shared__ S lzT[2][kMaxR * kLS];            // their WY factor T
    __shared__ S lws[2][384];                    // per-column scratch of the WY products
    constexpr int NRS = RM + 1;                  // row stride of nrw (a multiple of 32 doubles would put
                                                 // every fourth lane on one bank)
    __shared__ S nrw[64 * NRS];                  // the near rows of the current step
    __shared__ int s_go;
    int tready = (j1 - 1) >> 4;                  // lookahead: tiles of the band below this one are ready

    for (int k = 0; k < kext; ++k) {
        if (w == 0 && a.flags) {
            // the first sweep reads columns j1 .. min(j1+(k+1)r, n) up to step k;
            // later sweeps read no column before this sweep has read it
            const int tneed = (min(j + (k + 1) * r, n) - 1) >> 4;
            if (tready <= tneed) {
                if (wid == 0) {
                    const int t = tiles_wait(a.flags, tready, tneed, a.ntiles, a.flag_need, lane, a.wait_limit,
                                             a.status);
                    if (lane == 0) {
                        s_go = t;
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                }
                __syncthreads();
                tready = s_go;
                if (tready < 0) {
                    if (tid == 0) st_release(a.progress + w, kGaveUp);
                    return;
                }
            }
        }
        if (w > 0) {
            // step k of this sweep follows steps 0..k+2 of the previous sweep
            // (the last of them writes the column this step's near rows
            // update) and that sweep's far rows of H and T of steps 0..k+1
            // (step k+1's reach this step's T block, its lazy T column and its
            // near rows; step k+2's lie right of every column this step
            // touches).  The wait is bounded (see the protocol at the top of
            // the file).
            if (tid == 0) {
                s_go = bounded_wait(a.progress + w - 1, k + 3, a.hdone + w - 1, k + 2, a.hdone + q + w - 1, k + 2,
                                    a.wait_limit, a.status) ? 1 : 0;
                // one acquire per workgroup: it invalidates the caches the
                // workgroup's waves read through, and the barrier orders their
                // loads after it
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            if (!s_go) {
                if (tid == 0) st_release(a.progress + w, kGaveUp);
                return;
            }
        }
        const int buf = k & 1;
        // the lazy reflectors of block 0 are staged here; those of block k+1
        // are staged during step k (every earlier sweep has finished its step
        // k+1 by the time this step's wait returns)
        if (k == 0 && nw > 0) stage_lazy<S, 8>(a, 0, nw, lzv[0], lzT[0], tid);

        const int jb = j + max(0, (k - 1) * r + 1);
        const int i1 = j + k * r + 1;
        const int i2 = min(j + (k + 1) * r, n);
        const int i3 = min(j + (k + 2) * r, n);
        const bool full = k < nbj;
        const int m = full ? i2 - i1 + 1 : 0;            // 2..r
        // lazy range: rows base..rowmax of the columns jb (H) and i1+r-1 (T)
        const int base = j1 + k * r + 1;
        const int rowmax = min(j - 1 + (k + 1) * r, n);
        const int colT = i1 + r - 1;
        const bool lazyH = nw > 0 && jb <= n;
        const bool lazyT = nw > 0 && colT <= n;          // then, for a full block, colT == i2
        const int cend = full ? i2 : rowmax;             // last row of the two columns this step reads
        // near rows of the eager right update (this workgroup's part): H rows nr0..i3, columns i1..i2
        const int topH = max(j1 + 1, j1 + 1 + (k + 1 - d) * r);
        const int nr0 = max(topH, j1 + (k + 1) * r + 1);

        // ---- A. every load of the step, issued together
        const int row = base + lane;                     // row of this lane in the two columns
        S xh = zero<S>(), xt = zero<S>();
        if (wid == 0 && (lazyH || full) && row <= cend) xh = SH[B.idx(row - 1, jb - 1)];
        if (wid == 1 && lazyT && row <= cend) xt = ST[B.idx(row - 1, colT - 1)];
        constexpr int NB = (32 * 32 + 255) / 256;
        const int mcols = (full && lazyT) ? m - 1 : m;   // the last column comes from wave 1
        const int boff = B.idx(i1 - 1, i1 - 1);          // T block entry (0, 0); (ii, cc) at boff + ii + cc*cs
        S tb[NB];
        int tbi[NB], tbc[NB];
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            const int e = tid + 256 * it;
            tbc[it] = full ? e / m : 0;                  // block column
            tbi[it] = e - tbc[it] * m;                   // block row
            tb[it] = zero<S>();
            if (full && e < m * mcols) tb[it] = ST[boff + tbi[it] + tbc[it] * cs];
        }
        S xn[CP];
        const int nrow = nr0 + (tid >> 2);
        const int part = tid & 3;
        const bool non = full && nrow <= i3;
        const int noff = B.idx(nrow - 1, i1 - 1);
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            const int cc = part * CP + c;
            xn[c] = zero<S>();
            if (non && cc < m) xn[c] = SH[noff + cc * cs];
        }
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            const int e = tid + 256 * it;
            if (full && e < m * mcols) blk[tbc[it] * LB + tbi[it]] = tb[it];
        }
#pragma unroll
        for (int c = 0; c < CP; ++c) nrw[(tid >> 2) * NRS + part * CP + c] = xn[c];
        __syncthreads();

        // ---- B. lazy left updates (H column jb on waves 0 and 2, T column
        // i1+r-1 on waves 1 and 3) with the left reflectors of block k of the
        // earlier sweeps; then the left reflector from H(i1:i2, jb) (wave 0)
        S x = wid == 0 ? xh : xt;
        if (nw > 0) {
            // rows past the last lazy row (rowmax) take no part: the
            // reflectors are zero there
            const S y = lazy_wy<S>(x, lane, wid >> 1, (wid & 1) ? lazyT : lazyH, nw, r, lzv[buf], lzT[buf],
                                   lws[wid & 1]);
            if (wid < 2 && ((wid & 1) ? lazyT : lazyH)) x = y;
        }
        if (wid < 2) {
            const bool isH = (wid == 0);
            if (isH ? lazyH : lazyT) {
                // rows above the block go back now; the block's rows are
                // reduced (H) or take part in the T block (T)
                const int wlast = full ? i1 - 1 : rowmax;
                if (row <= wlast) (isH ? SH[B.idx(row - 1, jb - 1)] : ST[B.idx(row - 1, colT - 1)]) = x;
            }
            if (!isH && full && lazyT && row >= i1 && row <= i2) blk[(m - 1) * LB + (row - i1)] = x;
            if (isH && full) {
                // rows i1..i2 of column jb to lanes 0..m-1
                S y = shfl_(x, (lane + i1 - base) & 63);
                if (lane >= m) y = zero<S>();
                S v, tau, beta;
                wave_larfg(y, lane, m, v, tau, beta);
                if (lane < r) {
                    S vs = lane < m ? v : zero<S>();
                    a.VL[(w * kext + k) * r + lane] = vs;
                    sv[lane] = vs;
                }
                if (lane == 0) {
                    a.TL[w * kext + k] = tau;
                    stau[0] = tau;
                    SH[B.idx(i1 - 1, jb - 1)] = beta;
                } else if (lane < m) {
                    SH[B.idx(i1 - 1 + lane, jb - 1)] = zero<S>();
                }
            }
        }
        __syncthreads();

        if (full) {
            {   // ---- C. apply G^H to the T block: 8 lanes per column
                const S tau = stau[0];
                const int cc = tid >> 3, sub8 = tid & 7;
                S prt = zero<S>();
                if (cc < m)
                    for (int ii = sub8; ii < m; ii += 8) prt = add(prt, cmul(sv[ii], blk[cc * LB + ii]));
                S s = group_sum<8>(prt);
                s = mul(conj_(tau), s);
                if (cc < m && !iszero(tau))
                    for (int ii = sub8; ii < m; ii += 8) blk[cc * LB + ii] = sub(blk[cc * LB + ii], mul(s, sv[ii]));
            }
            __syncthreads();
            // ---- D. the block goes back to the band (all threads); its RQ
            // (last row first) on [blk; I] in the registers of wave 0, while
            // wave 1 forms this sweep's column of the WY factor and waves 2-3
            // stage the lazy reflectors of the next block
#pragma unroll
            for (int it = 0; it < NB; ++it) {
                const int e = tid + 256 * it;
                if (e < m * m) ST[boff + tbi[it] + tbc[it] * cs] = blk[tbc[it] * LB + tbi[it]];
            }
            if (wid == 0) {
                S x[RM];
#pragma unroll
                for (int c = 0; c < RM; ++c) {
                    S v = zero<S>();
                    if (lane < m && c < m) v = blk[c * LB + lane];
                    if (lane == 32 + c && c < m) v = one<S>();
                    x[c] = v;
                }
                rq_rows<S, RM>(x, m);
                // ---- normalise y = Y(:,0) and generate the opposite reflector
                S y = shfl_(x[0], 32 + (lane & 31));
                if (lane >= m) y = zero<S>();
                unsigned long long mask = __ballot(lane < m && !iszero(y));
                const int pv = mask ? (__ffsll((long long)mask) - 1) : 0;
                const S yp = bcast(y, pv);
                if (!iszero(yp)) {
                    const double ra = 1.0 / sqrt(abs2(yp));
                    if (im(yp) == 0.0) {
                        if (re(yp) < 0.0) y = mk<S>(-re(y), -im(y));
                    } else {
                        S ph = mk<S>(re(yp) * ra, -im(yp) * ra);
                        y = mul(y, ph);
                        if (lane == pv) y = mk<S>(re(y), 0.0);
                    }
                }
                S v, tau, beta;
                wave_larfg(y, lane, m, v, tau, beta);
                if (lane < r) a.VR[(w * kext + k) * r + lane] = lane < m ? v : zero<S>();
                if (lane < RM) sw[lane] = lane < m ? v : zero<S>();
                if (lane == 0) { a.TR[w * kext + k] = tau; stau[2] = tau; }
            } else if (wid == 1) {
                // this sweep's column of the WY factor of block k, for the later sweeps' lazy updates
                wy_column<S>(lane, nw, r, m, lzv[buf], lzT[buf], sv, stau[0], lws[1], a.TF + (w * kext + k) * kMaxR);
            } else if (nw > 0 && k + 1 < kext) {
                stage_lazy<S, 4>(a, k + 1, nw, lzv[buf ^ 1], lzT[buf ^ 1], tid - 128);
            }
            __syncthreads();

            // ---- E. eager right update of the near rows (from LDS): X <- X (I - sig w w^H),
            // four lanes per row, each with CP of the row's columns
            const S sig = stau[2];
            if (!iszero(sig)) {
                S ds = zero<S>();
#pragma unroll
                for (int c = 0; c < CP; ++c) {
                    const int cc = part * CP + c;
                    xn[c] = nrw[(tid >> 2) * NRS + cc];
                    ds = add(ds, mul(xn[c], sw[cc]));
                }
                ds = add(ds, shfl_(ds, lane ^ 1));         // every lane takes part in the exchange
                ds = add(ds, shfl_(ds, lane ^ 2));
                const S sx = mul(ds, sig);
                if (non) {
#pragma unroll
                    for (int c = 0; c < CP; ++c) {
                        const int cc = part * CP + c;
                        if (cc < m) SH[noff + cc * cs] = sub(xn[c], mul(sx, conj_(sw[cc])));
                    }
                }
            }
        } else {
            // absent block: mark both reflectors as identities
            if (tid < r) {
                a.VL[(w * kext + k) * r + tid] = zero<S>();
                a.VR[(w * kext + k) * r + tid] = zero<S>();
            }
            if (tid == 0) { a.TL[w * kext + k] = zero<S>(); a.TR[w * kext + k] = zero<S>(); }
            if (tid <= nw) a.TF[(w * kext + k) * kMaxR + tid] = zero<S>();
            if (nw > 0 && k + 1 < kext) stage_lazy<S, 8>(a, k + 1, nw, lzv[buf ^ 1], lzT[buf ^ 1], tid);
        }
        // the barrier completes every wave's stores; one agent-scope release
        // (a write-back of the shared cache) then publishes them with the flag
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            st_release(a.progress + w, k + 1);
        }
    }
    __syncthreads();
    if (tid == 0) st_release(a.progress + w, kAllDone);
}

}  // namespace ht
