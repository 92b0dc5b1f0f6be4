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
//      (jb) and to the column of T that enters its diagonal block (i1+r-1);
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
// segment before they write any of it back.
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
    int *progress;     // per sweep of the group: blocks whose step chain is finished (-1: gave up)
    int *hdone;        // per sweep: blocks whose far rows of H (hdone[w]) and of T (hdone[q+w]) are finished
    int *status;       // device status word: kStatus* bits, OR-ed in by a wait that gives up
    int64_t wait_limit;  // polls before a wait gives up (0: give up without polling)
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
        // p = sum_{c<i} x_c b_c (per lane) and ||b_{0..i-1}||^2 (uniform)
        S p0 = zero<S>(), p1 = zero<S>();
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int c = 0; c < i; ++c) {
            if (c & 1) p1 = add(p1, mul(x[c], b[c])); else p0 = add(p0, mul(x[c], b[c]));
            switch (c & 3) {
                case 0: s0 += abs2(b[c]); break;
                case 1: s1 += abs2(b[c]); break;
                case 2: s2 += abs2(b[c]); break;
                default: s3 += abs2(b[c]); break;
            }
        }
        const S alpha = b[i];
        const double ss = (s0 + s1) + (s2 + s3);
        if (ss == 0.0 && im(alpha) == 0.0) continue;              // tau = 0: identity
        S tau, sc;                                               // u_c = b_c sc (c < i), u_i = 1
        double bb;
        larfg_core(alpha, ss, tau, bb, sc);
        // s = (x_i + sum_{c<i} x_c u_c) tau;  x_c -= s conj(u_c) = (s conj(sc)) conj(b_c)
        const S sv = mul(add(x[i], mul(add(p0, p1), sc)), tau);
        const S t = mul(sv, conj_(sc));
#pragma unroll
        for (int c = 0; c < i; ++c) x[c] = sub(x[c], mul(t, conj_(b[c])));
        x[i] = sub(x[i], sv);
    }
}

// rows [top, bot] (1-based) of the band copy X, columns i1 .. i1+m-1:
// X <- X (I - sig w w^H), four lanes per row (each with RM/4 columns of it, the
// dot product summed over the four), 64 rows per pass of the workgroup; a
// row's entries are all loaded before any of them is written back.
template <class S, int RM>
__device__ inline void near_rows(S *X, const Band &B, int64_t top, int64_t bot, int64_t i1, int m,
                                 const S *sw, S sig, int tid)
{
    constexpr int CP = RM / 4;                     // columns per lane
    const int64_t cs = B.ldb - 1;                  // stride between columns of one band row
    const int part = tid & 3, lane = tid & 63;
    for (int64_t r0 = top; r0 <= bot; r0 += 64) {
        const int64_t row = r0 + (tid >> 2);
        const bool on = row <= bot;
        S *p = X + B.idx(row - 1, i1 - 1);
        S x[CP];
        S ds = zero<S>();
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            const int cc = part * CP + c;
            x[c] = zero<S>();
            if (on && cc < m) x[c] = p[cc * cs];
            ds = add(ds, mul(x[c], sw[cc]));
        }
        ds = add(ds, shfl_(ds, lane ^ 1));         // every lane takes part in the exchange
        ds = add(ds, shfl_(ds, lane ^ 2));
        const S sx = mul(ds, sig);
#pragma unroll
        for (int c = 0; c < CP; ++c) {
            const int cc = part * CP + c;
            if (on && cc < m) p[cc * cs] = sub(x[c], mul(sx, conj_(sw[cc])));
        }
    }
}

// The far rows of one step in one pass: rows [topH, topH+nH) of H, then rows
// [topT, topT+nT) of T (the first column zeroed from row zrowT on), as one
// index space over the workgroup; each thread loads U row segments before it
// writes any, so U rounds of loads are in flight together.
template <class S, int RM, int U>
__device__ __forceinline__ void far_rows(S *XH, S *XT, const Band &B, int64_t topH, int64_t nH, int64_t topT,
                                         int64_t nT, int64_t i1, int m, const S *sw, S sig, int tid, int64_t zrowT)
{
    const int64_t cs = B.ldb - 1;
    const int64_t tot = nH + nT;
    for (int64_t e0 = tid; e0 < tot; e0 += 256 * U) {
        S x[U][RM];
        S *p[U];
        bool zr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + 256 * u;
            const bool isH = e < nH;
            const int64_t row = isH ? topH + e : topT + (e - nH);
            p[u] = e < tot ? (isH ? XH : XT) + B.idx(row - 1, i1 - 1) : nullptr;
            zr[u] = !isH && row >= zrowT;
#pragma unroll
            for (int c = 0; c < RM; ++c) {
                x[u][c] = zero<S>();
                if (p[u] != nullptr && c < m) x[u][c] = p[u][c * cs];
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
#pragma unroll
            for (int c = 0; c < RM; ++c)
                if (p[u] != nullptr && c < m) p[u][c * cs] = (c == 0 && zr[u]) ? zero<S>() : sub(x[u][c], mul(sx, conj_(sw[c])));
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
__device__ __forceinline__ void gen_far(GenArgs<S> a, int w, int part)
{
    const int tid = threadIdx.x;
    const int64_t n = a.n, r = a.r, j1 = a.j1, j2 = a.j2, kext = a.kext;
    const int64_t j = j1 + w, d = j2 - j;
    const int64_t nbj = nblocks(n, r, j);
    const Band B = a.band;
    const int64_t q = j2 - j1 + 1;
    int *mine = a.hdone + part * q + w;
    __shared__ int s_go;
    __shared__ S hsw[64];
    __shared__ S hsig;
    for (int64_t k = 0; k < kext; ++k) {
        if (tid == 0) {
            s_go = bounded_wait(a.progress + w, (int)(k + 1), nullptr, 0, nullptr, 0, a.wait_limit, a.status) ? 1 : 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (!s_go) {                                // uniform: the sweep's workgroup gave up, or this wait did
            if (tid == 0) st_release(mine, kGaveUp);
            return;
        }
        if (k < nbj) {
            const int64_t i1 = j + k * r + 1;
            const int64_t i2 = i64min(j + (k + 1) * r, n);
            const int m = (int)(i2 - i1 + 1);
            if (tid < 64) hsw[tid] = tid < m ? a.VR[(w * kext + k) * r + tid] : zero<S>();
            if (tid == 0) hsig = a.TR[w * kext + k];
            __syncthreads();
            const S sig = hsig;
            const bool tdo = d >= 1 && !iszero(sig);
            if (!iszero(sig)) {
                const int64_t topH = i64max(j1 + 1, j1 + 1 + (k + 1 - d) * r);
                const int64_t nlo = i64max(topH, j1 + (k + 1) * r + 1);
                const int64_t topT = i64max(j1 + 1, j1 + 1 + (k - d) * r);
                constexpr int U = sizeof(S) * RM <= 256 ? 2 : 1;     // two rows per thread while registers allow
                if (part == 0)
                    far_rows<S, RM, U>(a.SH, a.ST, B, topH, nlo - topH, topT, 0, i1, m, hsw, sig, tid, i1 + 1);
                else if (tdo)
                    far_rows<S, RM, U>(a.SH, a.ST, B, topH, 0, topT, i2 - topT + 1, i1, m, hsw, sig, tid, i1 + 1);
            }
            if (part == 1 && !tdo)
                for (int e = tid; e < m - 1; e += 256) a.ST[B.idx(i1 + e, i1 - 1)] = zero<S>();
        }
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            st_release(mine, (int)(k + 1));
        }
    }
    __syncthreads();
    if (tid == 0) st_release(mine, kAllDone);
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
    const int64_t n = a.n, r = a.r, j1 = a.j1, j2 = a.j2, kext = a.kext;
    const int64_t j = j1 + w;
    const int64_t nbj = nblocks(n, r, j);
    const Band B = a.band;
    S *SH = a.SH, *ST = a.ST;

    constexpr int LB = 33;                       // LDS leading dimension of 32x32 blocks
    __shared__ S sv[64], sw[64], su[64];
    __shared__ S blk[32 * LB];
    __shared__ S stau[4];
    __shared__ S lzv[kMaxR * kMaxR];            // staged lazy reflectors (sweeps j1..j-1, block k)
    __shared__ S lzt[kMaxR];

    for (int64_t k = 0; k < kext; ++k) {
        if (w > 0) {
            // step k of this sweep follows steps 0..k+2 of the previous sweep
            // (the last of them writes the column this step's near rows
            // update) and that sweep's far rows of H and T of steps 0..k+1
            // (step k+1's reach this step's T block, its lazy T column and its
            // near rows; step k+2's lie right of every column this step
            // touches).  The wait is bounded (see the protocol at the top of
            // the file).
            __shared__ int s_go;
            if (tid == 0) {
                const int64_t q = j2 - j1 + 1;
                s_go = bounded_wait(a.progress + w - 1, (int)(k + 3), a.hdone + w - 1, (int)(k + 2),
                                    a.hdone + q + w - 1, (int)(k + 2), a.wait_limit, a.status) ? 1 : 0;
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
        const int64_t jb = j + i64max(0, (k - 1) * r + 1);
        const int64_t i1 = j + k * r + 1;
        const int64_t i2 = i64min(j + (k + 1) * r, n);
        const int64_t i3 = i64min(j + (k + 2) * r, n);
        const bool full = k < nbj;

        // ---- 1. lazy left updates (wave 0: H column jb, wave 1: T column i1+r-1);
        // the reflectors of block k of the earlier sweeps are first staged in
        // LDS with one parallel round trip
        if (j > j1) {
            const int nw = (int)(j - j1);
            constexpr int NV = (kMaxR * kMaxR + 255) / 256;      // fixed trip count: loads in flight together
            S tv[NV];
#pragma unroll
            for (int it = 0; it < NV; ++it) {
                const int e = tid + 256 * it;
                tv[it] = zero<S>();
                if (e < nw * r) tv[it] = a.VL[((e / (int)r) * kext + k) * r + e % (int)r];
            }
            if (tid < nw) lzt[tid] = a.TL[tid * kext + k];
#pragma unroll
            for (int it = 0; it < NV; ++it) {
                const int e = tid + 256 * it;
                if (e < nw * r) lzv[e] = tv[it];
            }
            __syncthreads();
        }
        if (wid < 2 && j > j1) {
            const bool isH = (wid == 0);
            const int64_t col = isH ? jb : i1 + r - 1;          // 1-based
            if (col <= n) {
                S *X = isH ? SH : ST;
                const int64_t base = j1 + k * r + 1;             // top row of the lazy range
                const int64_t rowmax = i64min(j - 1 + (k + 1) * r, n);
                const int64_t row = base + lane;
                const bool inr = row <= rowmax;
                S x = inr ? X[B.idx(row - 1, col - 1)] : zero<S>();
                for (int64_t jh = j1; jh < j; ++jh) {
                    const int64_t wh = jh - j1;
                    const S tau = lzt[wh];
                    if (iszero(tau)) continue;                  // block (jh,k) absent or trivial
                    const int64_t aa = jh + k * r + 1;
                    const int64_t bb = i64min(jh + (k + 1) * r, n);
                    const bool inb = row >= aa && row <= bb;
                    const S vi = inb ? lzv[wh * r + (row - aa)] : zero<S>();
                    S s = wave_sum(cmul(vi, x));
                    s = mul(conj_(tau), s);
                    if (inb) x = sub(x, mul(s, vi));
                }
                if (inr) X[B.idx(row - 1, col - 1)] = x;
            }
        }
        __syncthreads();

        if (full) {
            const int m = (int)(i2 - i1 + 1);               // 2..r
            // ---- 2. left reflector from H(i1:i2, jb)
            if (wid == 0) {
                S x = lane < m ? SH[B.idx(i1 - 1 + lane, jb - 1)] : zero<S>();
                S v, tau, beta;
                wave_larfg(x, lane, m, v, tau, beta);
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
            // T block -> LDS
            {
                constexpr int NB = (32 * 32 + 255) / 256;
                S tb[NB];
#pragma unroll
                for (int it = 0; it < NB; ++it) {
                    const int e = tid + 256 * it, ii = e % m, cc = e / m;
                    tb[it] = zero<S>();
                    if (e < m * m) tb[it] = ST[B.idx(i1 - 1 + ii, i1 - 1 + cc)];
                }
#pragma unroll
                for (int it = 0; it < NB; ++it) {
                    const int e = tid + 256 * it, ii = e % m, cc = e / m;
                    if (e < m * m) blk[cc * LB + ii] = tb[it];
                }
            }
            __syncthreads();
            {   // apply G^H to the block: 8 lanes per column
                const S tau = stau[0];
                const int cc = tid >> 3, sub8 = tid & 7;
                S part = zero<S>();
                if (cc < m)
                    for (int ii = sub8; ii < m; ii += 8) part = add(part, cmul(sv[ii], blk[cc * LB + ii]));
                S s = group_sum<8>(part);
                s = mul(conj_(tau), s);
                if (cc < m && !iszero(tau))
                    for (int ii = sub8; ii < m; ii += 8) blk[cc * LB + ii] = sub(blk[cc * LB + ii], mul(s, sv[ii]));
            }
            __syncthreads();
            for (int e = tid; e < m * m; e += 256) {
                const int ii = e % m, cc = e / m;
                ST[B.idx(i1 - 1 + ii, i1 - 1 + cc)] = blk[cc * LB + ii];
            }
            __syncthreads();

            // ---- 3. RQ of the block (last row first) on [blk; I], in registers
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
                const int p = mask ? (__ffsll((long long)mask) - 1) : 0;
                const S yp = bcast(y, p);
                if (!iszero(yp)) {
                    const double ra = 1.0 / sqrt(abs2(yp));
                    if (im(yp) == 0.0) {
                        if (re(yp) < 0.0) y = mk<S>(-re(y), -im(y));
                    } else {
                        S ph = mk<S>(re(yp) * ra, -im(yp) * ra);
                        y = mul(y, ph);
                        if (lane == p) y = mk<S>(re(y), 0.0);
                    }
                }
                S v, tau, beta;
                wave_larfg(y, lane, m, v, tau, beta);
                if (lane < r) a.VR[(w * kext + k) * r + lane] = lane < m ? v : zero<S>();
                if (lane < RM) sw[lane] = lane < m ? v : zero<S>();
                if (lane == 0) { a.TR[w * kext + k] = tau; stau[2] = tau; }
            }
            __syncthreads();

            // ---- 4. eager right updates: the rows of H this sweep's next steps
            // read (from j1+(k+1)r+1 on); the helper workgroup does the rest
            const S sig = stau[2];
            if (!iszero(sig)) {
                const int64_t d = j2 - j;
                const int64_t topH = i64max(j1 + 1, j1 + 1 + (k + 1 - d) * r);
                near_rows<S, RM>(SH, B, i64max(topH, j1 + (k + 1) * r + 1), i3, i1, m, sw, sig, tid);
            }
        } else {
            // absent block: mark both reflectors as identities
            if (tid < r) {
                a.VL[(w * kext + k) * r + tid] = zero<S>();
                a.VR[(w * kext + k) * r + tid] = zero<S>();
            }
            if (tid == 0) { a.TL[w * kext + k] = zero<S>(); a.TR[w * kext + k] = zero<S>(); }
        }
        // the barrier completes every wave's stores; one agent-scope release
        // (a write-back of the shared cache) then publishes them with the flag
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            st_release(a.progress + w, (int)(k + 1));
        }
    }
    __syncthreads();
    if (tid == 0) st_release(a.progress + w, kAllDone);
}

}  // namespace ht
