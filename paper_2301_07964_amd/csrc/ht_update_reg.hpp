// ht_update_reg.hpp -- register-ring variants of the application-phase
// kernels for r in {4, 8, 16, 32} (see ht_update.hpp for the method).
//
// One wavefront per panel of 64 rows (right mode) or 64 columns (left mode);
// lane l owns one row (or column) of the panel and keeps the current window in
// a ring of 2r registers.  Windows advance by r, so the ring slot of local
// index c in the t-th window of the panel is (c - (t mod 2) r) mod 2r: the
// window loop is unrolled by two and every register index is a compile-time
// constant.  The reflector vectors and scalars are wave-uniform (scalar
// loads).  Each window loads r new vectors, applies its q reflectors with the
// algorithmic flop count (no dense window factor) and stores r finished ones.
#pragma once
#include "ht_common.hpp"
#include "ht_update.hpp"

namespace ht {

template <int R, int P>
__device__ constexpr int rslot(int c) { return ((c - P * R) % (2 * R) + 2 * R) % (2 * R); }

// ------------------------------------------------------------- right mode
template <class S, int R, int P>
__device__ __forceinline__ void right_window(S (&x)[2 * R], const UpdJob<S> &J, const S *V, const S *Tv,
                                             int64_t n, int64_t q, int64_t kext, int64_t k, int64_t lo,
                                             bool first, bool last, int64_t row, bool rowok)
{
    const int64_t W = q + R - 1;
    S *X = J.X;
    const int64_t ld = J.ld;
    // new columns 0 .. r-1 always; the carried columns r .. W-1 only in the
    // first window (straight-line selects keep every ring index constant)
#pragma unroll
    for (int c = 0; c < 2 * R - 1; ++c) {
        const int64_t col = lo + c;
        const bool fresh = c < R || first;
        S v = zero<S>();
        if (fresh && c < W && rowok && col < n) v = X[row + col * ld];
        x[rslot<R, P>(c)] = sel(fresh, v, x[rslot<R, P>(c)]);
    }
#pragma unroll
    for (int w = 0; w < R; ++w) {
        if (w < q) {
            const S tau = Tv[w * kext + k];
            if (!iszero(tau)) {
                const S *v = V + (w * kext + k) * R;
                S d0 = zero<S>(), d1 = zero<S>();
#pragma unroll
                for (int i = 0; i < R; i += 2) {
                    d0 = add(d0, mul(x[rslot<R, P>(w + i)], v[i]));
                    d1 = add(d1, mul(x[rslot<R, P>(w + i + 1)], v[i + 1]));
                }
                const S s = mul(add(d0, d1), tau);
#pragma unroll
                for (int i = 0; i < R; ++i) x[rslot<R, P>(w + i)] = sub(x[rslot<R, P>(w + i)], mul(s, conj_(v[i])));
            }
        }
    }
    const int64_t f0 = last ? 0 : q - 1;
#pragma unroll
    for (int c = 0; c < 2 * R - 1; ++c) {
        const int64_t col = lo + c;
        if (c >= f0 && c < W && rowok && col < n) X[row + col * ld] = x[rslot<R, P>(c)];
    }
}

template <class S, int R>
__global__ __launch_bounds__(64) void k_update_right_reg(UpdArgs<S> a)
{
    int64_t b = blockIdx.x;
    int jid = 0;
    while (jid < a.njobs - 1 && b >= a.job[jid].npanels) { b -= a.job[jid].npanels; ++jid; }
    const UpdJob<S> J = a.job[jid];
    const int64_t n = a.n, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    const int64_t W = q + R - 1;
    const int64_t p0 = b * 64, row = p0 + threadIdx.x;
    const bool rowok = row < n;
    const S *V = J.side ? a.VR : a.VL;
    const S *Tv = J.side ? a.TR : a.TL;
    int64_t kend = 0;
    if (J.lim >= 0) {
        while (kend < kmax && !(p0 < i64min(j1 + kend * R + W - 1, n - 1) + 1 + J.lim)) ++kend;
        if (kend >= kmax) return;
    }
    S x[2 * R];
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) x[i] = zero<S>();
    for (int64_t k = kmax - 1; k >= kend; k -= 2) {
        right_window<S, R, 0>(x, J, V, Tv, n, q, kext, k, j1 + k * R, k == kmax - 1, k == kend, row, rowok);
        if (k - 1 < kend) break;
        right_window<S, R, 1>(x, J, V, Tv, n, q, kext, k - 1, j1 + (k - 1) * R, false, k - 1 == kend, row, rowok);
    }
}

// -------------------------------------------------------------- left mode
template <class S, int R, int P>
__device__ __forceinline__ void left_window(S (&x)[2 * R], S *stage, const UpdJob<S> &J, const S *V, const S *Tv,
                                            int64_t n, int64_t q, int64_t kext, int64_t k, int64_t lo,
                                            bool first, bool last, int64_t c0, int lane)
{
    constexpr int SP = 2 * R + 1;                 // staging leading dimension (rows)
    const int64_t W = q + R - 1;
    S *X = J.X;
    const int64_t ld = J.ld;
    const int64_t nload = first ? W : R;
    for (int64_t e = lane; e < nload * 64; e += 64) {
        const int64_t rr = e % nload, cc = e / nload;
        const int64_t row = lo + rr, col = c0 + cc;
        stage[cc * SP + rr] = (row < n && col < n) ? X[row + col * ld] : zero<S>();
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2 * R - 1; ++c) {
        const bool fresh = c < R || first;
        S v = zero<S>();
        if (fresh && c < W) v = stage[lane * SP + c];
        x[rslot<R, P>(c)] = sel(fresh, v, x[rslot<R, P>(c)]);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < R; ++w) {
        if (w < q) {
            const S tau = Tv[w * kext + k];
            if (!iszero(tau)) {
                const S *v = V + (w * kext + k) * R;
                S d0 = zero<S>(), d1 = zero<S>();
#pragma unroll
                for (int i = 0; i < R; i += 2) {
                    d0 = add(d0, cmul(v[i], x[rslot<R, P>(w + i)]));
                    d1 = add(d1, cmul(v[i + 1], x[rslot<R, P>(w + i + 1)]));
                }
                const S s = mul(conj_(tau), add(d0, d1));
#pragma unroll
                for (int i = 0; i < R; ++i) x[rslot<R, P>(w + i)] = sub(x[rslot<R, P>(w + i)], mul(s, v[i]));
            }
        }
    }
    const int64_t f0 = last ? 0 : q - 1;
    const int64_t nst = W - f0;
#pragma unroll
    for (int c = 0; c < 2 * R - 1; ++c)
        if (c >= f0 && c < W) stage[lane * SP + (c - f0)] = x[rslot<R, P>(c)];
    __syncthreads();
    for (int64_t e = lane; e < nst * 64; e += 64) {
        const int64_t rr = e % nst, cc = e / nst;
        const int64_t row = lo + f0 + rr, col = c0 + cc;
        if (row < n && col < n) X[row + col * ld] = stage[cc * SP + rr];
    }
    __syncthreads();
}

template <class S, int R>
__global__ __launch_bounds__(64) void k_update_left_reg(UpdArgs<S> a)
{
    int64_t b = blockIdx.x;
    int jid = 0;
    while (jid < a.njobs - 1 && b >= a.job[jid].npanels) { b -= a.job[jid].npanels; ++jid; }
    const UpdJob<S> J = a.job[jid];
    const int lane = threadIdx.x;
    const int64_t n = a.n, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    const int64_t c0 = b * 64;
    int64_t kstart = kmax - 1;
    if (J.lim >= 0) {
        while (kstart >= 0 && !(c0 + 64 > j1 + kstart * R - J.lim)) --kstart;
        if (kstart < 0) return;
    }
    __shared__ S stage[64 * (2 * R + 1)];
    S x[2 * R];
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) x[i] = zero<S>();
    for (int64_t k = kstart; k >= 0; k -= 2) {
        left_window<S, R, 0>(x, stage, J, a.VL, a.TL, n, q, kext, k, j1 + k * R, k == kstart, k == 0, c0, lane);
        if (k - 1 < 0) break;
        left_window<S, R, 1>(x, stage, J, a.VL, a.TL, n, q, kext, k - 1, j1 + (k - 1) * R, false, k - 1 == 0, c0, lane);
    }
}

}  // namespace ht
