// ht_update.hpp -- application phase of blocked stage two (Section 3.2,
// "Applying the reflectors"; application algorithm of the appendix).
//
// After the generate phase of a group of q sweeps, the reflectors are applied
// to the full matrices in the grouped order the paper derives: every window k
// (the q reflectors of block k, acting on indices lo_k .. lo_k+q+r-2 with
// lo_k = j1 + k r, 0-based) is applied as a unit, windows from the bottom
// (k = kmax-1) to the top (k = 0).  Within a window the reflectors are applied
// in sweep order.  Right updates (columns of H, T, Z with the right reflectors,
// columns of Q with the left ones) run first over all rows; then left updates
// (rows of H and T with G^H).  Because every reflector is applied in full, the
// result equals the unblocked algorithm up to rounding; the right pass creates
// a transient fill up to about q*r below the band that the left pass removes,
// hence the row/column limits (LIM) below.
//
// Kernel shape: one wavefront per panel of 64 rows (right mode, lane = row)
// or 64 columns (left mode, lane = column).  The panel streams through the
// windows keeping the current window in an LDS ring of 2r slots: every window
// loads r new vectors from HBM and retires r finished ones, so each entry is
// read and written once per group.
#pragma once
#include "ht_common.hpp"

namespace ht {

template <class S>
struct UpdJob {
    S *X;
    int64_t ld;
    int64_t lim;       // < 0: every window; else window k active iff p0 < hi_k+1+lim (right) / c0+64 > lo_k-lim (left)
    int64_t npanels;
    int side;          // 0: left reflectors (VL/TL), 1: right reflectors (VR/TR)
};

template <class S>
struct UpdArgs {
    int64_t n, r, q, j1, kmax, kext;
    const S *VL, *TL, *VR, *TR;
    UpdJob<S> job[4];
    int njobs;
};

// ring slot of local index c (< 2r) of window k (streaming from k = kmax-1
// downwards): windows advance by r and the ring has 2r slots, so only the
// parity of the window count matters
__device__ inline int ring_slot(int64_t k, int64_t kmax, int64_t r, int c, int rs) {
    const int s = c - (int)(((kmax - 1 - k) & 1) * r);
    return s < 0 ? s + rs : s;
}

// Right mode: X(rows, window) <- X(rows, window) * G_{j1} ... G_{j2}
template <class S>
__global__ __launch_bounds__(64) void k_update_right(UpdArgs<S> a)
{
    int64_t b = blockIdx.x;
    int jid = 0;
    while (jid < a.njobs - 1 && b >= a.job[jid].npanels) { b -= a.job[jid].npanels; ++jid; }
    const UpdJob<S> J = a.job[jid];
    const int lane = threadIdx.x;
    const int64_t n = a.n, r = a.r, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    const int64_t W = q + r - 1;               // window width
    const int rs = (int)(2 * r);               // ring slots (>= W since q <= r)
    const int64_t p0 = b * 64, row = p0 + lane;
    const bool rowok = row < n;
    const S *V = J.side ? a.VR : a.VL;
    const S *Tv = J.side ? a.TR : a.TL;

    int64_t kend = 0;
    if (J.lim >= 0) {
        // smallest k with p0 < hi_k + 1 + lim, hi_k = min(lo_k + W - 1, n - 1)
        while (kend < kmax && !(p0 < i64min(j1 + kend * r + W - 1, n - 1) + 1 + J.lim)) ++kend;
        if (kend >= kmax) return;
    }
    extern __shared__ unsigned char smem_raw[];
    S *ring = reinterpret_cast<S *>(smem_raw);          // [rs][64]

    for (int64_t k = kmax - 1; k >= kend; --k) {
        const int64_t lo = j1 + k * r;                 // 0-based first column of window k
        const bool first = (k == kmax - 1), last = (k == kend);
        const int64_t nload = first ? W : r;
        for (int c = 0; c < nload; ++c) {
            const int64_t col = lo + c;
            S x = (rowok && col < n) ? J.X[row + col * J.ld] : zero<S>();
            ring[ring_slot(k, kmax, r, c, rs) * 64 + lane] = x;
        }
        for (int w = 0; w < q; ++w) {
            const S tau = Tv[w * kext + k];
            if (iszero(tau)) continue;
            const S *v = V + (w * kext + k) * r;
            S dot = zero<S>();
            for (int i = 0; i < r; ++i)
                dot = add(dot, mul(ring[ring_slot(k, kmax, r, w + i, rs) * 64 + lane], v[i]));
            const S s = mul(dot, tau);
            for (int i = 0; i < r; ++i) {
                S *p = ring + ring_slot(k, kmax, r, w + i, rs) * 64 + lane;
                *p = sub(*p, mul(s, conj_(v[i])));
            }
        }
        const int64_t c0 = last ? 0 : q - 1;
        for (int64_t c = c0; c < W; ++c) {
            const int64_t col = lo + c;
            if (rowok && col < n) J.X[row + col * J.ld] = ring[ring_slot(k, kmax, r, (int)c, rs) * 64 + lane];
        }
    }
}

// Left mode: X(window, cols) <- G_{j2}^H ... G_{j1}^H X(window, cols)
template <class S>
__global__ __launch_bounds__(64) void k_update_left(UpdArgs<S> a)
{
    int64_t b = blockIdx.x;
    int jid = 0;
    while (jid < a.njobs - 1 && b >= a.job[jid].npanels) { b -= a.job[jid].npanels; ++jid; }
    const UpdJob<S> J = a.job[jid];
    const int lane = threadIdx.x;
    const int64_t n = a.n, r = a.r, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    const int64_t W = q + r - 1;
    const int rs = (int)(2 * r);
    const int64_t c0 = b * 64;
    const S *V = a.VL;
    const S *Tv = a.TL;

    int64_t kstart = kmax - 1;
    if (J.lim >= 0) {
        // largest k with c0 + 64 > lo_k - lim
        while (kstart >= 0 && !(c0 + 64 > j1 + kstart * r - J.lim)) --kstart;
        if (kstart < 0) return;
    }
    extern __shared__ unsigned char smem_raw[];
    S *ring = reinterpret_cast<S *>(smem_raw);          // [rs][64]: ring[slot*64 + column]
    S *stage = ring + rs * 64;                          // [64 cols][65] transpose staging

    for (int64_t k = kstart; k >= 0; --k) {
        const int64_t lo = j1 + k * r;
        const bool first = (k == kstart), last = (k == 0);
        const int64_t nload = first ? W : r;
        // coalesced load of rows lo .. lo+nload-1 of the 64 columns, via staging
        for (int64_t e = lane; e < nload * 64; e += 64) {
            const int64_t rr = e % nload, cc = e / nload;
            const int64_t row = lo + rr, col = c0 + cc;
            stage[cc * 65 + rr] = (row < n && col < n) ? J.X[row + col * J.ld] : zero<S>();
        }
        __syncthreads();
        for (int c = 0; c < nload; ++c) ring[ring_slot(k, kmax, r, c, rs) * 64 + lane] = stage[lane * 65 + c];
        __syncthreads();
        for (int w = 0; w < q; ++w) {
            const S tau = Tv[w * kext + k];
            if (iszero(tau)) continue;
            const S *v = V + (w * kext + k) * r;
            S dot = zero<S>();
            for (int i = 0; i < r; ++i)
                dot = add(dot, cmul(v[i], ring[ring_slot(k, kmax, r, w + i, rs) * 64 + lane]));
            const S s = mul(conj_(tau), dot);
            for (int i = 0; i < r; ++i) {
                S *p = ring + ring_slot(k, kmax, r, w + i, rs) * 64 + lane;
                *p = sub(*p, mul(s, v[i]));
            }
        }
        const int64_t f0 = last ? 0 : q - 1;
        const int64_t nst = W - f0;
        for (int64_t c = 0; c < nst; ++c) stage[lane * 65 + c] = ring[ring_slot(k, kmax, r, (int)(f0 + c), rs) * 64 + lane];
        __syncthreads();
        for (int64_t e = lane; e < nst * 64; e += 64) {
            const int64_t rr = e % nst, cc = e / nst;
            const int64_t row = lo + f0 + rr, col = c0 + cc;
            if (row < n && col < n) J.X[row + col * J.ld] = stage[cc * 65 + rr];
        }
        __syncthreads();
    }
}

}  // namespace ht
