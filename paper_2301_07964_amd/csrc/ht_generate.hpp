// ht_generate.hpp -- generate phase of blocked stage two (Section 3.2,
// "Generating the reflectors"; generate algorithm of the appendix).
//
// One workgroup (256 threads, 4 wavefronts) per sweep of the group
// j1..j2 (q <= r sweeps).  Sweep j processes blocks k = 0..kext-1 in order;
// block (j,k) starts once sweep j-1 has finished block k+2 (progress flags in
// device memory, agent-scope release/acquire).  Steps that run concurrently
// touch disjoint columns of the scratch band, so no other synchronisation is
// needed.
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
    int *progress;     // per sweep of the group: number of finished blocks
};

template <class S> __device__ inline S shfl_(S v, int src);
template <> __device__ inline double shfl_<double>(double v, int src) { return __shfl(v, src, 64); }
template <> __device__ inline zd shfl_<zd>(zd v, int src) { return mk<zd>(__shfl(v.re, src, 64), __shfl(v.im, src, 64)); }

__device__ inline int ld_acquire(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Householder generation in one wavefront.  Lane l holds x_l (l < m).
// Returns v_l (v_0 = 1), tau and beta in every lane.
template <class S>
__device__ inline void wave_larfg(S x, int lane, int m, S &v, S &tau, S &beta) {
    S alpha = shfl_(x, 0);
    double ss = wave_sum((lane >= 1 && lane < m) ? abs2(x) : 0.0);
    if (ss == 0.0 && im(alpha) == 0.0) {
        tau = zero<S>();
        beta = alpha;
        v = (lane == 0) ? one<S>() : x;
        return;
    }
    double b = -(re(alpha) >= 0.0 ? 1.0 : -1.0) * sqrt(abs2(alpha) + ss);
    tau = mk<S>((b - re(alpha)) / b, -im(alpha) / b);
    beta = mk<S>(b, 0.0);
    S sc = recip(sub(alpha, beta));
    v = (lane == 0) ? one<S>() : mul(x, sc);
}

template <class S>
__global__ __launch_bounds__(256) void k_generate(GenArgs<S> a)
{
    const int w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t n = a.n, r = a.r, j1 = a.j1, j2 = a.j2, kext = a.kext;
    const int64_t j = j1 + w;
    const int64_t nbj = nblocks(n, r, j);
    const Band B = a.band;
    S *SH = a.SH, *ST = a.ST;

    constexpr int LB = 33;                       // LDS leading dimension of 32x32 blocks
    __shared__ S sv[64], sw[64], su[64];
    __shared__ S blk[32 * LB];
    __shared__ S yb[32 * LB];
    __shared__ S stau[4];
    __shared__ S lzv[kMaxR * kMaxR];            // staged lazy reflectors (sweeps j1..j-1, block k)
    __shared__ S lzt[kMaxR];

    for (int64_t k = 0; k < kext; ++k) {
        if (w > 0) {
            // bounded wait: a predecessor step takes microseconds; after ~2^22
            // polls the workgroup gives up (the output is then invalid) so that
            // no wave can spin forever
            __shared__ int s_abort;
            if (tid == 0) {
                int polls = 0;
                s_abort = 0;
                while (ld_acquire(a.progress + w - 1) < (int)(k + 3)) {
                    if (++polls > (1 << 22)) { s_abort = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if (s_abort) {
                if (tid == 0) st_release(a.progress + w, 0x3fffffff);
                return;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
            for (int e = tid; e < nw * r; e += 256) {
                const int wh = e / (int)r, ii = e % (int)r;
                lzv[e] = a.VL[(wh * kext + k) * r + ii];
            }
            for (int e = tid; e < nw; e += 256) lzt[e] = a.TL[e * kext + k];
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
            for (int e = tid; e < m * m; e += 256) {
                const int ii = e % m, cc = e / m;
                blk[cc * LB + ii] = ST[B.idx(i1 - 1 + ii, i1 - 1 + cc)];
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
                yb[cc * LB + ii] = (ii == cc) ? one<S>() : zero<S>();
            }
            __syncthreads();

            // ---- 3. RQ of the block (last row first) on [blk; I]
            for (int i = m - 1; i >= 1; --i) {
                if (wid == 0) {
                    S b = lane <= i ? conj_(blk[lane * LB + i]) : zero<S>();
                    // xLARFG with alpha = b_i, x = b_0..b_{i-1}
                    S alpha = shfl_(b, i);
                    double ss = wave_sum(lane < i ? abs2(b) : 0.0);
                    S tau, u;
                    if (ss == 0.0 && im(alpha) == 0.0) {
                        tau = zero<S>();
                        u = zero<S>();
                    } else {
                        double bb = -(re(alpha) >= 0.0 ? 1.0 : -1.0) * sqrt(abs2(alpha) + ss);
                        tau = mk<S>((bb - re(alpha)) / bb, -im(alpha) / bb);
                        S sc = recip(sub(alpha, mk<S>(bb, 0.0)));
                        u = lane < i ? mul(b, sc) : (lane == i ? one<S>() : zero<S>());
                    }
                    if (lane <= i) su[lane] = u;
                    if (lane == 0) stau[1] = tau;
                }
                __syncthreads();
                const S tau = stau[1];
                if (!iszero(tau)) {
                    // rows 0..i-1 of blk and rows 0..m-1 of yb: X(row, 0:i) <- X (I - tau u u^H)
                    const int rr = tid >> 2, sub4 = tid & 3;
                    S *X = nullptr;
                    int row = 0;
                    if (rr < i) { X = blk; row = rr; }
                    else if (rr < i + m) { X = yb; row = rr - i; }
                    S part = zero<S>();
                    if (X)
                        for (int c = sub4; c <= i; c += 4) part = add(part, mul(X[c * LB + row], su[c]));
                    S s = group_sum<4>(part);
                    s = mul(s, tau);
                    if (X)
                        for (int c = sub4; c <= i; c += 4) X[c * LB + row] = sub(X[c * LB + row], mul(s, conj_(su[c])));
                }
                __syncthreads();
            }
            // ---- normalise y = Y(:,0) and generate the opposite reflector
            if (wid == 0) {
                S y = lane < m ? yb[lane] : zero<S>();
                unsigned long long mask = __ballot(lane < m && !iszero(y));
                const int p = mask ? (__ffsll((long long)mask) - 1) : 0;
                S yp = shfl_(y, p);
                if (!iszero(yp)) {
                    const double aa = sqrt(abs2(yp));
                    if (im(yp) == 0.0) {
                        if (re(yp) < 0.0) y = mk<S>(-re(y), -im(y));
                    } else {
                        S ph = mk<S>(re(yp) / aa, -im(yp) / aa);
                        y = mul(y, ph);
                        if (lane == p) y = mk<S>(re(y), 0.0);
                    }
                }
                S v, tau, beta;
                wave_larfg(y, lane, m, v, tau, beta);
                if (lane < r) {
                    S vs = lane < m ? v : zero<S>();
                    a.VR[(w * kext + k) * r + lane] = vs;
                    sw[lane] = vs;
                }
                if (lane == 0) { a.TR[w * kext + k] = tau; stau[2] = tau; }
            }
            __syncthreads();

            // ---- 4. eager right updates on the band
            const S sig = stau[2];
            if (!iszero(sig)) {
                const int64_t d = j2 - j;
                const int64_t topH = i64max(j1 + 1, j1 + 1 + (k + 1 - d) * r);
                for (int64_t row = topH + tid; row <= i3; row += 256) {
                    S s = zero<S>();
                    for (int c = 0; c < m; ++c) s = add(s, mul(SH[B.idx(row - 1, i1 - 1 + c)], sw[c]));
                    s = mul(s, sig);
                    for (int c = 0; c < m; ++c) {
                        S *p = SH + B.idx(row - 1, i1 - 1 + c);
                        *p = sub(*p, mul(s, conj_(sw[c])));
                    }
                }
                if (d >= 1) {
                    const int64_t topT = i64max(j1 + 1, j1 + 1 + (k - d) * r);
                    for (int64_t row = topT + tid; row <= i2; row += 256) {
                        S s = zero<S>();
                        for (int c = 0; c < m; ++c) s = add(s, mul(ST[B.idx(row - 1, i1 - 1 + c)], sw[c]));
                        s = mul(s, sig);
                        for (int c = 0; c < m; ++c) {
                            S *p = ST + B.idx(row - 1, i1 - 1 + c);
                            *p = sub(*p, mul(s, conj_(sw[c])));
                        }
                    }
                }
            }
            __syncthreads();
            for (int e = tid; e < m - 1; e += 256) ST[B.idx(i1 + e, i1 - 1)] = zero<S>();
        } else {
            // absent block: mark both reflectors as identities
            if (tid < r) {
                a.VL[(w * kext + k) * r + tid] = zero<S>();
                a.VR[(w * kext + k) * r + tid] = zero<S>();
            }
            if (tid == 0) { a.TL[w * kext + k] = zero<S>(); a.TR[w * kext + k] = zero<S>(); }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) st_release(a.progress + w, (int)(k + 1));
    }
    __syncthreads();
    if (tid == 0) st_release(a.progress + w, 0x3fffffff);
}

}  // namespace ht
