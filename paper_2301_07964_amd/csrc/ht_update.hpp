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
    int mat;           // 0: H, 1: T, 2: Q or Z (selects the rule of the exact zeros and the scratch band)
};

// Exact zeros of the structure after the last sweep j2 of a group, for one
// column (0-based c).  In exact arithmetic the delayed updates leave zeros
// there; in floating point they leave rounding residue that the unblocked
// algorithm never has (it writes the annihilated entries as zeros and never
// touches the others).  If the residue stayed, the next group's scratch copy
// would inherit it and the generate phase's restricted update ranges would
// treat it inconsistently, and the mismatch feeds back from group to group.
// Below the diagonal, T keeps only the blocks I(j2,k) x I(j2,k) without their
// first column; H keeps the first subdiagonal for columns <= j2, and for later
// columns the r-band plus the fill blocks I(j2,k+1) x (I(j2,k) minus its first
// column).  Rows are 1-based in keepH / keepT.
struct CleanCol {
    int64_t c1, r, n, j2, a, b;
    bool inblk;        // c1 lies in a block of sweep j2 and is not its first column
    __host__ __device__ CleanCol(int64_t c, int64_t r_, int64_t n_, int64_t j2_) : c1(c + 1), r(r_), n(n_), j2(j2_)
    {
        a = 0; b = 0; inblk = false;
        if (c1 >= j2 + 1) {
            const int64_t kb = (c1 - j2 - 1) / r;
            if (kb < nblocks(n, r, j2)) {
                a = j2 + kb * r + 1;
                b = i64min(a + r - 1, n);
                inblk = c1 > a;
            }
        }
    }
    __host__ __device__ bool keepT(int64_t i1b) const { return inblk && i1b <= b; }
    __host__ __device__ bool keepH(int64_t i1b) const
    {
        if (c1 <= j2) return i1b <= c1 + 1;
        if (i1b <= c1 + r) return true;
        const int64_t a2 = a + r, b2 = i64min(a2 + r - 1, n);
        return inblk && a2 <= n && i1b >= a2 && i1b <= b2;
    }
};

// Epilogue of the left pass for lookahead (the next group's generation runs
// while this pass is still going): once a tile of columns has taken its last
// window, it writes the group's exact zeros in those columns, copies their
// band into the next group's scratch band and adds one to the tile's flag
// (agent-scope release), so that after group g every flag reads 2 (g + 1):
// one for the H tile, one for the T tile.
template <class S>
struct LeftEpi {
    S *SH, *ST;            // scratch band of the next group
    Band band;
    int64_t c0;            // first column (0-based) of the next group's band; >= n: nothing to copy
    int64_t j2;            // last sweep of this group (1-based)
    int64_t cc0, depth;    // exact zeros in columns >= cc0, rows c+1 .. c+depth (0-based)
    int *flags;            // per tile of 16 columns; nullptr: no epilogue
};

template <class S>
struct UpdArgs {
    int64_t n, r, q, j1, kmax, kext;
    const S *VL, *TL, *VR, *TR;
    UpdJob<S> job[4];
    int njobs;
    LeftEpi<S> epi;
};

// The epilogue for columns p0 .. p0+ncol-1 of job J, by nthr threads (thread
// t); the caller has made the tile's updates of X visible to every thread.
template <class S>
__device__ inline void left_epilogue(const UpdArgs<S> &a, const UpdJob<S> &J, int64_t p0, int ncol, int t, int nthr)
{
    const LeftEpi<S> &e = a.epi;
    const int64_t n = a.n;
    S *X = J.X;
    S *SB = J.mat == 1 ? e.ST : e.SH;
    const Band B = e.band;
    for (int cl = 0; cl < ncol; ++cl) {
        const int64_t c = p0 + cl;
        if (c >= n) break;
        const CleanCol cc(c, a.r, n, e.j2);
        const bool cln = c >= e.cc0;
        const int64_t zlast = cln ? i64min(n - 1, c + e.depth) : c;    // last row of the exact zeros
        const bool cpy = c >= e.c0;
        const int64_t blo = i64max(0, c - B.BU), bhi = i64min(n - 1, c + B.BL);
        const int64_t rlo = cpy ? blo : c + 1, rhi = cpy ? i64max(bhi, zlast) : zlast;
        for (int64_t i = rlo + t; i <= rhi; i += nthr) {
            const bool z = i > c && i <= zlast && !(J.mat == 1 ? cc.keepT(i + 1) : cc.keepH(i + 1));
            S v = zero<S>();
            if (z) X[i + c * J.ld] = v;
            else if (cpy && i <= bhi) v = X[i + c * J.ld];
            if (cpy && i <= bhi) SB[B.idx(i, c)] = v;
        }
    }
}

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
