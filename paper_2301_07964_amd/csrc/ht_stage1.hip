// ht_stage1.hip -- stage one: dense pencil (A, B) -> r-Hessenberg-triangular
// form (Section 2.2 and the blocked stage-one algorithm of the appendix),
// preceded by the QR factorisation of B.  C ABI: ht_rhess, ht_rhess_z,
// ht_rhess_p, ht_rhess_z_p, ht_rhess_default_p.
//
// Panels of nb = r columns.  For panel j the rows j+nb..n are covered by
// blocks of bm = p*nb rows that overlap by nb rows (block k starts at row
// j+nb+k(p-1)nb), processed from the bottom:
//   left phase:  QR of A(block k, panel) (Householder, one workgroup for the
//                whole chain of blocks, the block in LDS); then every block's
//                reflectors are applied, bottom-up, to the columns of A right
//                of the panel and to B (chain kernels, 64 columns per
//                workgroup), and Q <- Q Q_k (64 rows per workgroup);
//   right phase: per block from the bottom, RQ of the filled B block in LDS,
//                the first nb rows of its orthogonal factor from the stored
//                reflectors, their LQ factorisation by reflectors P_t applied
//                from the right; a wide kernel applies P_0..P_{nb-1} to the
//                rows 1..i2 of B (the next block's RQ reads them) and writes
//                the exact zeros of the block's first nb columns; after the
//                last block, A and Z receive all blocks' P_t (chain kernels).
// The QR of B uses the same block-QR and chain kernels (blocks start at the
// panel's first row).  All arithmetic is FP64 / complex128.  With the
// overlapped schedule (below) the Q and Z passes and the far rows of each
// block's pass over B run on two more streams beside the caller's.
#include "ht_common.hpp"
#include "ht_workspace.hpp"
#include "ht.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <utility>

namespace ht {

extern thread_local char g_errmsg[256];
int launch_check(const char *what);

constexpr int kS1MaxBM = 64;      // largest block order p*nb (LDS budget of the RQ)
constexpr int kS1MaxNB = 32;

// block sum over 256 threads (result in every thread); red: >= 4 doubles of LDS
__device__ inline double block_sum256(double v, double *red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// xLARFG on (alpha, ||x||^2): tau, beta and the scale 1/(alpha - beta) of x
template <class S>
__device__ inline void larfg_scalars(S alpha, double ss, S &tau, S &beta, S &scal, bool &trivial)
{
    trivial = (ss == 0.0 && im(alpha) == 0.0);
    if (trivial) { tau = zero<S>(); beta = alpha; scal = one<S>(); return; }
    double b;
    larfg_core(alpha, ss, tau, b, scal);
    beta = mk<S>(b, 0.0);
}

// Geometry of the chain of blocks of one panel (0-based rows).
struct Blocks {
    int64_t row0, step, bm, nblk, n;
    __device__ __host__ int64_t r0(int64_t k) const { return row0 + k * step; }
    __device__ __host__ int64_t r1(int64_t k) const { return i64min(n, row0 + k * step + bm) - 1; }
};

// ---------------------------------------------------------------- left QR
// QR of X(block k rows, cols c0..c0+nc-1) for k = nblk-1 .. 0 (one
// workgroup).  The R factor and exact zeros go back to X; the reflectors to
// V[k*bm*nc + s*bm + i] (unit lower trapezoidal, zeros above) and tau[k*nc+s].
// Column s of the block is held in registers by the 8 threads 8s..8s+7
// (rows 8u + (tid & 7)); one barrier per reflector.
template <class S>
__global__ __launch_bounds__(256) void k_s1_block_qr(S *X, int64_t ld, Blocks bl, int64_t c0, int nc, S *V, S *tau)
{
    __shared__ S vb[2][kS1MaxBM];
    __shared__ S tb[2];
    const int tid = threadIdx.x, s = tid >> 3, part = tid & 7;
    const int bm = (int)bl.bm;
    const bool col = s < nc;
    for (int64_t k = bl.nblk - 1; k >= 0; --k) {
        const int64_t r0 = bl.r0(k);
        const int m = (int)(bl.r1(k) - r0 + 1);
        S x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = 8 * u + part;
            x[u] = (col && i < m) ? X[r0 + i + (c0 + s) * ld] : zero<S>();
        }
        const int ns = m < nc ? m : nc;
        for (int st = 0; st < ns; ++st) {
            const int b = st & 1;
            if (s == st) {                                   // the pivot column's 8 threads
                S al = zero<S>();
                double ssp = 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = 8 * u + part;
                    al = sel(i == st, x[u], al);
                    ssp += (i > st) ? abs2(x[u]) : 0.0;     // rows >= m hold zeros
                }
                al = group_sum<8>(al);
                const double ss = group_sum<8>(ssp);
                S t, be, f;
                bool triv;
                larfg_scalars(al, ss, t, be, f, triv);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = 8 * u + part;
                    S v = zero<S>();
                    if (i == st) v = one<S>();
                    else if (i > st && i < m) v = iszero(t) ? x[u] : mul(x[u], f);
                    if (i < bm) V[(k * bm) * nc + st * bm + i] = v;
                    vb[b][i] = v;
                    x[u] = (i == st) ? be : ((i > st) ? zero<S>() : x[u]);
                }
                if (part == 0) { tau[k * nc + st] = t; tb[b] = t; }
            }
            __syncthreads();
            const S tt = tb[b];
            if (s > st && col && !iszero(tt)) {              // G^H on the later columns
                S p = zero<S>();
#pragma unroll
                for (int u = 0; u < 8; ++u) p = add(p, cmul(vb[b][8 * u + part], x[u]));
                const S d = mul(conj_(tt), group_sum<8>(p));
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = sub(x[u], mul(d, vb[b][8 * u + part]));
            }
        }
        // R and exact zeros back to X (the next block reads the overlap rows)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = 8 * u + part;
            if (col && i < m) X[r0 + i + (c0 + s) * ld] = x[u];
        }
        __syncthreads();
    }
}

// Stage block k's reflectors (m x nc, column s at s*bm) and taus into LDS;
// NT threads, fixed trip counts so that the loads are in flight together.
template <int NT, class S>
__device__ inline void stage_refl(S *vs, S *ts, const S *V, const S *tau, int64_t k, int bm, int nc, int t)
{
    const S *Vk = V + k * bm * nc;
    constexpr int CH = 8;
    const int tot = bm * nc;
    for (int e0 = 0; e0 < tot; e0 += NT * CH) {
        S buf[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + u * NT + t;
            buf[u] = e < tot ? Vk[e] : zero<S>();
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + u * NT + t;
            if (e < tot) vs[e] = buf[u];
        }
    }
    if (t < nc) ts[t] = tau[k * nc + t];
}

constexpr int kS1Cols = 16;      // columns (left chain) or rows (right chain) per workgroup
constexpr int kS1ChainThreads = 256;

// ------------------------------------------------------ left chain (columns)
// For k = nblk-1 .. 0: X(block k rows, c) <- Q_k^H X(block k rows, c) for the
// columns c in [cfirst, clast] with c >= (cfrom_block ? r0(k) : cfirst).
// 16 columns per workgroup of 256 threads: the block's rows are staged through
// LDS with coalesced loads (lane = row), then column cc is held in registers
// by the 16 threads 16cc..16cc+15 (rows 16u + (t & 15)).
template <class S>
__global__ __launch_bounds__(kS1ChainThreads) void k_s1_left_chain(S *X, int64_t ld, Blocks bl, int nc, const S *V,
                                                                   const S *tau, int64_t cfirst, int64_t clast,
                                                                   int cfrom_block)
{
    constexpr int NT = kS1ChainThreads, CW = kS1Cols, LT = CW + 1, RPT = kS1MaxBM / 16;
    __shared__ S xs[kS1MaxBM * LT];                 // row i, column cc at xs[i*LT + cc]
    __shared__ S vs[kS1MaxBM * kS1MaxNB];
    __shared__ S ts[kS1MaxNB];
    const int t = threadIdx.x, cc = t >> 4, part = t & 15;
    const int lr = t & 63, lc = t >> 6;             // staging: row lr, columns lc + 4u
    const int64_t cb = cfirst + (int64_t)blockIdx.x * CW;
    const int bm = (int)bl.bm;
    for (int64_t k = bl.nblk - 1; k >= 0; --k) {
        const int64_t r0 = bl.r0(k);
        const int m = (int)(bl.r1(k) - r0 + 1);
        const int64_t clo = cfrom_block ? i64max(cfirst, r0) : cfirst;
        if (cb + CW - 1 < clo) continue;                // uniform: the workgroup has no column here
        stage_refl<NT>(vs, ts, V, tau, k, bm, nc, t);
        {
            S buf[CW / 4];
#pragma unroll
            for (int u = 0; u < CW / 4; ++u) {
                const int64_t col = cb + lc + 4 * u;
                buf[u] = (lr < m && col <= clast) ? X[r0 + lr + col * ld] : zero<S>();
            }
#pragma unroll
            for (int u = 0; u < CW / 4; ++u) xs[lr * LT + lc + 4 * u] = buf[u];
        }
        __syncthreads();
        S x[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u) x[u] = xs[(16 * u + part) * LT + cc];
        const int ns = m < nc ? m : nc;
        for (int s = 0; s < ns; ++s) {
            const S tsv = ts[s];
            if (iszero(tsv)) continue;                  // uniform
            const S *v = vs + s * bm;
            S vi[RPT];
#pragma unroll
            for (int u = 0; u < RPT; ++u) vi[u] = (16 * u + part < bm) ? v[16 * u + part] : zero<S>();
            S p = zero<S>();
#pragma unroll
            for (int u = 0; u < RPT; ++u) p = add(p, cmul(vi[u], x[u]));
            const S d = mul(conj_(tsv), group_sum<16>(p));
#pragma unroll
            for (int u = 0; u < RPT; ++u) x[u] = sub(x[u], mul(d, vi[u]));
        }
#pragma unroll
        for (int u = 0; u < RPT; ++u) xs[(16 * u + part) * LT + cc] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CW / 4; ++u) {
            const int64_t col = cb + lc + 4 * u;
            if (lr < m && col <= clast && col >= clo) X[r0 + lr + col * ld] = xs[lr * LT + lc + 4 * u];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ right chain (rows)
// For k = nblk-1 .. 0: X(rho, block k columns) <- X(rho, block k columns) G_0
// ... G_{nc-1} for rows rho in [0, rlast]; the block's columns are the block's
// rows (r0(k) .. r1(k)).  16 rows per workgroup of 256 threads, staged through
// LDS; row rr is held in registers by the threads 16rr..16rr+15 (columns
// 16u + (t & 15)).
template <class S>
__global__ __launch_bounds__(kS1ChainThreads) void k_s1_right_chain(S *X, int64_t ld, Blocks bl, int nc, const S *V,
                                                                    const S *tau, int64_t rlast)
{
    constexpr int NT = kS1ChainThreads, RW = kS1Cols, LT = kS1MaxBM + 1, CPT = kS1MaxBM / 16;
    __shared__ S xs[RW * LT];                       // row rr, column c at xs[rr*LT + c]
    __shared__ S vs[kS1MaxBM * kS1MaxNB];
    __shared__ S ts[kS1MaxNB];
    const int t = threadIdx.x, rr = t >> 4, part = t & 15;
    const int lr = t & (RW - 1), lc = t >> 4;       // staging: row lr, columns lc + 16u
    const int64_t rb = (int64_t)blockIdx.x * RW;
    const bool okst = rb + lr <= rlast;
    const int bm = (int)bl.bm;
    for (int64_t k = bl.nblk - 1; k >= 0; --k) {
        const int64_t c0 = bl.r0(k);
        const int m = (int)(bl.r1(k) - c0 + 1);
        stage_refl<NT>(vs, ts, V, tau, k, bm, nc, t);
        {
            S buf[CPT];
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = lc + 16 * u;
                buf[u] = (okst && c < m) ? X[rb + lr + (c0 + c) * ld] : zero<S>();
            }
#pragma unroll
            for (int u = 0; u < CPT; ++u) xs[lr * LT + lc + 16 * u] = buf[u];
        }
        __syncthreads();
        S x[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) x[u] = xs[rr * LT + 16 * u + part];
        const int ns = m < nc ? m : nc;
        for (int s = 0; s < ns; ++s) {
            const S tsv = ts[s];
            if (iszero(tsv)) continue;                  // uniform
            const S *v = vs + s * bm;
            S vc[CPT];
#pragma unroll
            for (int u = 0; u < CPT; ++u) vc[u] = (16 * u + part < bm) ? v[16 * u + part] : zero<S>();
            S p = zero<S>();
#pragma unroll
            for (int u = 0; u < CPT; ++u) p = add(p, mul(x[u], vc[u]));
            const S d = mul(group_sum<16>(p), tsv);
#pragma unroll
            for (int u = 0; u < CPT; ++u) x[u] = sub(x[u], mul(d, conj_(vc[u])));
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) xs[rr * LT + 16 * u + part] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = lc + 16 * u;
            if (okst && c < m) X[rb + lr + (c0 + c) * ld] = xs[lr * LT + c];
        }
        __syncthreads();
    }
}

// ------------------------------------------------ right factor (one block)
// RQ of B(block k, block k) = Rt Qt (Householder, last row first), the first
// nr rows of Qt, and their LQ factorisation: reflectors P_t (acting on local
// columns t..m-1, zeros above) into VR[k*bm*nc + t*bm + i], tau into
// tauR[k*nc + t].
//   RQ:  row i of the block is held in registers by threads 4i..4i+3
//        (columns 4u + (tid & 3)); step i's reflector u_i goes to LDS (kept
//        for the next phase), one barrier per step;
//   Yc = U_{m-1} ... U_1 [e_0 .. e_{nr-1}]: column c by threads 8c..8c+7
//        (rows 8v + (tid & 7)), no barriers;
//   LQ of M = Yc^H: row t of M is column t of Yc, in the same registers; one
//        barrier per reflector.
template <class S>
__global__ __launch_bounds__(256) void k_s1_right_factor(const S *B, int64_t ld, Blocks bl, int64_t k, int nb,
                                                         S *VR, S *tauR)
{
    __shared__ S U[kS1MaxBM * kS1MaxBM];             // U[i*64 + c], c < i: RQ reflector of row i
    __shared__ S ut[kS1MaxBM];
    __shared__ S vbuf[2][kS1MaxBM];
    __shared__ S tbuf[2];
    const int tid = threadIdx.x;
    const int bm = (int)bl.bm;
    const int64_t r0 = bl.r0(k);
    const int m = (int)(bl.r1(k) - r0 + 1);
    const int nr = m < nb ? m : nb;
    // ---- RQ, rows m-1 .. 1
    {
        const int row = tid >> 2, part = tid & 3;
        S w[kS1MaxBM / 4];
#pragma unroll
        for (int u = 0; u < kS1MaxBM / 4; ++u) {
            const int c = 4 * u + part;
            w[u] = (row < m && c < m) ? B[r0 + row + (r0 + c) * ld] : zero<S>();
        }
        for (int i = m - 1; i >= 1; --i) {
            if (row == i) {
                S al = zero<S>();
                double ssp = 0.0;
#pragma unroll
                for (int u = 0; u < kS1MaxBM / 4; ++u) {
                    const int c = 4 * u + part;
                    al = sel(c == i, w[u], al);
                    ssp += (c < i) ? abs2(w[u]) : 0.0;
                }
                al = group_sum<4>(al);
                const double ss = group_sum<4>(ssp);
                S t, be, f;
                bool triv;
                larfg_scalars(conj_(al), ss, t, be, f, triv);
#pragma unroll
                for (int u = 0; u < kS1MaxBM / 4; ++u) {     // the whole row: u_c (c < i), 1, zeros
                    const int c = 4 * u + part;
                    S uc = zero<S>();
                    if (c < i) uc = iszero(t) ? zero<S>() : mul(conj_(w[u]), f);
                    else if (c == i) uc = one<S>();
                    U[i * kS1MaxBM + c] = uc;
                }
                if (part == 0) ut[i] = t;
            }
            __syncthreads();
            const S t = ut[i];
            if (row < i && !iszero(t)) {                 // rows 0..i-1: W <- W (I - t u u^H)
                S uc[kS1MaxBM / 4];
#pragma unroll
                for (int u = 0; u < kS1MaxBM / 4; ++u) uc[u] = U[i * kS1MaxBM + 4 * u + part];
                S p = zero<S>();
#pragma unroll
                for (int u = 0; u < kS1MaxBM / 4; ++u) p = add(p, mul(w[u], uc[u]));
                const S d = mul(group_sum<4>(p), t);
#pragma unroll
                for (int u = 0; u < kS1MaxBM / 4; ++u) w[u] = sub(w[u], mul(d, conj_(uc[u])));
            }
        }
    }
    __syncthreads();
    // ---- Yc = U_{m-1} ... U_1 [e_0 .. e_{nr-1}]; column yc by 8 threads
    const int yc = tid >> 3, yp = tid & 7;
    S y[kS1MaxBM / 8];
#pragma unroll
    for (int v = 0; v < kS1MaxBM / 8; ++v) y[v] = (8 * v + yp == yc) ? one<S>() : zero<S>();
    for (int i = 1; i < m; ++i) {
        const S t = ut[i];
        if (iszero(t)) continue;                          // uniform
        S uc[kS1MaxBM / 8];
#pragma unroll
        for (int v = 0; v < kS1MaxBM / 8; ++v) uc[v] = U[i * kS1MaxBM + 8 * v + yp];
        S p = zero<S>();
#pragma unroll
        for (int v = 0; v < kS1MaxBM / 8; ++v) p = add(p, cmul(uc[v], y[v]));
        const S d = mul(group_sum<8>(p), t);
#pragma unroll
        for (int v = 0; v < kS1MaxBM / 8; ++v) y[v] = sub(y[v], mul(d, uc[v]));
    }
    // ---- LQ of M = Qt(0:nr, :) = Yc^H: row yc of M, entries 8v + yp
#pragma unroll
    for (int v = 0; v < kS1MaxBM / 8; ++v) y[v] = conj_(y[v]);
    for (int t = 0; t < nr; ++t) {
        const int b = t & 1;
        if (yc == t) {
            S al = zero<S>();
            double ssp = 0.0;
#pragma unroll
            for (int v = 0; v < kS1MaxBM / 8; ++v) {
                const int c = 8 * v + yp;
                al = sel(c == t, y[v], al);
                ssp += (c > t && c < m) ? abs2(y[v]) : 0.0;
            }
            al = group_sum<8>(al);
            const double ss = group_sum<8>(ssp);
            S ta, be, f;
            bool triv;
            larfg_scalars(conj_(al), ss, ta, be, f, triv);
#pragma unroll
            for (int v = 0; v < kS1MaxBM / 8; ++v) {
                const int c = 8 * v + yp;
                S vv = zero<S>();
                if (c == t) vv = one<S>();
                else if (c > t && c < m) vv = iszero(ta) ? zero<S>() : mul(conj_(y[v]), f);
                if (c < bm) VR[(k * bm) * nb + t * bm + c] = vv;
                vbuf[b][c] = vv;
            }
            if (yp == 0) { tauR[k * nb + t] = ta; tbuf[b] = ta; }
        }
        __syncthreads();
        const S ta = tbuf[b];
        if (yc > t && yc < nr && !iszero(ta)) {           // rows t+1..nr-1: M <- M P_t
            S p = zero<S>();
#pragma unroll
            for (int v = 0; v < kS1MaxBM / 8; ++v) p = add(p, mul(y[v], vbuf[b][8 * v + yp]));
            const S d = mul(group_sum<8>(p), ta);
#pragma unroll
            for (int v = 0; v < kS1MaxBM / 8; ++v) y[v] = sub(y[v], mul(d, conj_(vbuf[b][8 * v + yp])));
        }
    }
}

// exact zeros below the diagonal of the first nr columns of block k of B
template <class S>
__global__ __launch_bounds__(256) void k_s1_zero_block(S *B, int64_t ld, Blocks bl, int64_t k, int nb)
{
    const int64_t c0 = bl.r0(k), r1 = bl.r1(k);
    const int m = (int)(r1 - c0 + 1), nr = m < nb ? m : nb;
    for (int e = threadIdx.x; e < nr * m; e += 256) {
        const int i = e % m, cc = e / m;
        if (i > cc) B[c0 + i + (c0 + cc) * ld] = zero<S>();
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_s1_zero_pattern(S *A, S *B, int64_t ld, int64_t n, int64_t r)
{
    const int64_t c = blockIdx.x;
    for (int64_t i = c + r + 1 + threadIdx.x; i < n; i += 256) A[i + c * ld] = zero<S>();
    for (int64_t i = c + 1 + threadIdx.x; i < n; i += 256) B[i + c * ld] = zero<S>();
}

// ------------------------------------------------------------------ host
static int64_t s1_default_p(int64_t nb) { return i64max(2, i64min(8, kS1MaxBM / nb)); }

// workspace of one call: left and right reflectors and taus of every block of a panel
static size_t s1_workspace_bytes(int64_t n, int64_t nb, int64_t p, size_t elem)
{
    const int64_t maxblk = n / ((p - 1) * nb) + 2;
    return 2 * ((size_t)maxblk * p * nb * nb * elem + (size_t)maxblk * nb * elem) + 1024;
}

// ------------------------------------------------------------ overlap
// The tasks of parallel stage one (Section 2.3): generating a panel's left
// reflectors (block QRs) and right reflectors (the per-block factors with
// their pass over B) stay on the caller's stream.  Applying them to Q (left)
// and Z (right) depends on nothing else, and the left pass over A only has to
// precede the right pass over A and the next block QR, so those three passes
// run on a second stream `qz` beside the rest.  In each block's pass over B
// only the rows that the next factors read (from a lower bound L down the
// chain) stay on the caller's stream; the rows above L go to a third stream
// `far`, which during the QR of B (no factors yet) takes the passes over A
// instead.  L is moved down once every kS1Chunk blocks, and only then does
// the caller's stream wait for the far rows already queued: adjacent blocks
// share columns, so rows handed to `far` for block k+1 must be finished before
// the caller's stream updates them for block k.  Every entry receives the same
// operations in the same order as in the one-stream schedule, so the results
// are bitwise equal.
constexpr int64_t kS1Chunk = 8;        // blocks per position of the bound L
constexpr int64_t kS1OverlapMinN = 1024;

struct S1Ctx {
    hipStream_t far = nullptr, qz = nullptr;
    hipEvent_t fac = nullptr, far_done = nullptr, gl = nullptr, lq = nullptr, gr = nullptr, rz = nullptr, fa = nullptr;
    bool ok = false;
};
static std::mutex g_s1_mu;
static std::map<std::pair<int, hipStream_t>, S1Ctx> g_s1;

static S1Ctx *s1_ctx(hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_s1_mu);
    S1Ctx &c = g_s1[{dev, st}];
    if (c.ok) return &c;
    if (!c.far && hipStreamCreateWithFlags(&c.far, hipStreamNonBlocking) != hipSuccess) { c.far = nullptr; return nullptr; }
    if (!c.qz && hipStreamCreateWithFlags(&c.qz, hipStreamNonBlocking) != hipSuccess) { c.qz = nullptr; return nullptr; }
    hipEvent_t *ev[] = {&c.fac, &c.far_done, &c.gl, &c.lq, &c.gr, &c.rz, &c.fa};
    for (hipEvent_t *e : ev)
        if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) { *e = nullptr; return nullptr; }
    c.ok = true;
    return &c;
}

// Which events of the context this call has recorded (a stream waits only for
// an event recorded earlier in the same call).
struct S1Sched {
    S1Ctx *c = nullptr;                // null: everything on the caller's stream
    hipStream_t st = nullptr;
    bool far_rec = false, lq_rec = false, rz_rec = false, fa_rec = false;
    hipStream_t qz_stream() const { return c ? c->qz : st; }
    int record(hipEvent_t e, hipStream_t s) { return hipEventRecord(e, s) == hipSuccess ? 0 : 1; }
    int wait(hipStream_t s, hipEvent_t e) { return hipStreamWaitEvent(s, e, 0) == hipSuccess ? 0 : 1; }
    // the caller's stream waits for everything queued on the other two
    int join()
    {
        if (!c) return 0;
        int rc = 0;
        if (hipEventRecord(c->far_done, c->far) != hipSuccess || hipStreamWaitEvent(st, c->far_done, 0) != hipSuccess) rc = 1;
        if (hipEventRecord(c->rz, c->qz) != hipSuccess || hipStreamWaitEvent(st, c->rz, 0) != hipSuccess) rc = 1;
        return rc;
    }
};

template <class S>
static int right_chain(S *X, int64_t ld, const Blocks &bl, int nb, const S *V, const S *tau, int64_t rfirst,
                       int64_t rlast, hipStream_t s)
{
    if (rlast < rfirst) return 0;
    // rows rfirst..rlast: the kernel's rows are relative to X, its columns absolute
    const int64_t rows = rlast - rfirst + 1;
    hipLaunchKernelGGL(k_s1_right_chain<S>, dim3((unsigned)((rows + kS1Cols - 1) / kS1Cols)), dim3(kS1ChainThreads), 0, s,
                       X + rfirst, ld, bl, nb, V, tau, rows - 1);
    return launch_check("k_s1_right_chain");
}

template <class S>
static int left_phase(S *X, S *A2, S *B2, S *Q, int64_t ld, int64_t n, const Blocks &bl, int64_t c0, int nc,
                      S *V, S *tau, int64_t a2first, int64_t b2first, int b2from_block, bool qr_of_b, S1Sched &sc)
{
    int rc;
    const hipStream_t st = sc.st;
    // the previous panel's passes over Q and A read V and tau
    if (sc.lq_rec && (rc = sc.wait(st, sc.c->lq))) return rc;
    if (sc.fa_rec) {
        if ((rc = sc.wait(st, sc.c->fa))) return rc;
        sc.fa_rec = false;
    }
    hipLaunchKernelGGL(k_s1_block_qr<S>, dim3(1), dim3(256), 0, st, X, ld, bl, c0, nc, V, tau);
    if ((rc = launch_check("k_s1_block_qr"))) return rc;
    // Q and the columns of A right of the panel (or all of A for the QR of B):
    // only the right pass over A and the next block QR wait for them.  The
    // pass over A runs on `qz` after Q's, except in the QR of B, where `far`
    // is idle and takes it (no factor chain to hide the two passes behind)
    const bool has_a = A2 && a2first <= n - 1;
    const hipStream_t qs = sc.qz_stream();
    const hipStream_t as = sc.c ? (qr_of_b ? sc.c->far : sc.c->qz) : st;
    if (sc.c && (Q || has_a) && (rc = sc.record(sc.c->gl, st))) return rc;
    if (Q) {
        if (sc.c && (rc = sc.wait(qs, sc.c->gl))) return rc;
        if ((rc = right_chain<S>(Q, ld, bl, nc, V, tau, 0, n - 1, qs))) return rc;
    }
    if (has_a) {
        if (sc.c && (rc = sc.wait(as, sc.c->gl))) return rc;
        const int64_t ncols = n - a2first;
        hipLaunchKernelGGL(k_s1_left_chain<S>, dim3((unsigned)((ncols + kS1Cols - 1) / kS1Cols)), dim3(kS1ChainThreads), 0, as, A2, ld, bl, nc,
                           (const S *)V, (const S *)tau, a2first, n - 1, 0);
        if ((rc = launch_check("k_s1_left_chain"))) return rc;
    }
    if (sc.c && (Q || (has_a && as == sc.c->qz))) {
        if ((rc = sc.record(sc.c->lq, qs))) return rc;
        sc.lq_rec = true;
    }
    if (sc.c && has_a && as == sc.c->far) {
        if ((rc = sc.record(sc.c->fa, as))) return rc;
        sc.fa_rec = true;
    }
    if (B2 && b2first <= n - 1) {
        // the previous panel's far rows of B
        if (sc.far_rec && (rc = sc.wait(st, sc.c->far_done))) return rc;
        const int64_t ncols = n - b2first;
        hipLaunchKernelGGL(k_s1_left_chain<S>, dim3((unsigned)((ncols + kS1Cols - 1) / kS1Cols)), dim3(kS1ChainThreads), 0, st, B2, ld, bl, nc,
                           (const S *)V, (const S *)tau, b2first, n - 1, b2from_block);
        if ((rc = launch_check("k_s1_left_chain"))) return rc;
    }
    return 0;
}

// Right phase of one panel: per block from the bottom, the factor, its pass
// over rows 0..r1(k) of B (rows from L(k) on the caller's stream, the rest on
// `far`), the exact zeros; then Z on `qz` and A on the caller's stream (after
// the panel's left pass over A).
template <class S>
static int right_phase(S *A, S *B, S *Z, int64_t ld, int64_t n, const Blocks &bl, int nb, S *VR, S *TR, S1Sched &sc)
{
    int rc;
    const hipStream_t st = sc.st;
    const int64_t bm = bl.bm, nblk = bl.nblk;
    // the previous panel's Z pass reads VR and TR
    if (sc.rz_rec && (rc = sc.wait(st, sc.c->rz))) return rc;
    int64_t Lprev = -1;
    for (int64_t k = nblk - 1; k >= 0; --k) {
        hipLaunchKernelGGL(k_s1_right_factor<S>, dim3(1), dim3(256), 0, st, (const S *)B, ld, bl, k, nb, VR, TR);
        if ((rc = launch_check("k_s1_right_factor"))) return rc;
        const S *Vk = VR + k * bm * nb, *Tk = TR + k * nb;
        const Blocks one_blk{bl.r0(k), bl.step, bm, 1, n};
        // L(k) <= r0(k-1): the factor of block k-1 reads rows r0(k-1)..r1(k-1)
        const int64_t kc = (k / kS1Chunk) * kS1Chunk;
        const int64_t L = sc.c ? bl.r0(kc > 0 ? kc - 1 : 0) : 0;
        if (sc.c) {
            if ((rc = sc.record(sc.c->fac, st))) return rc;
            // rows L..L(k+1)-1 were handed to `far` for block k+1
            if (Lprev >= 0 && L < Lprev && (rc = sc.wait(st, sc.c->far_done))) return rc;
        }
        if ((rc = right_chain<S>(B, ld, one_blk, nb, Vk, Tk, L, bl.r1(k), st))) return rc;
        hipLaunchKernelGGL(k_s1_zero_block<S>, dim3(1), dim3(256), 0, st, B, ld, bl, k, nb);
        if ((rc = launch_check("k_s1_zero_block"))) return rc;
        if (sc.c && L > 0) {
            if ((rc = sc.wait(sc.c->far, sc.c->fac))) return rc;
            if ((rc = right_chain<S>(B, ld, one_blk, nb, Vk, Tk, 0, L - 1, sc.c->far))) return rc;
            if ((rc = sc.record(sc.c->far_done, sc.c->far))) return rc;
            sc.far_rec = true;
        }
        Lprev = L;
    }
    if (Z) {
        if (sc.c) {
            if ((rc = sc.record(sc.c->gr, st)) || (rc = sc.wait(sc.c->qz, sc.c->gr))) return rc;
        }
        if ((rc = right_chain<S>(Z, ld, bl, nb, VR, TR, 0, n - 1, sc.qz_stream()))) return rc;
        if (sc.c) {
            if ((rc = sc.record(sc.c->rz, sc.c->qz))) return rc;
            sc.rz_rec = true;
        }
    }
    // the left pass over A of this panel
    if (sc.lq_rec && (rc = sc.wait(st, sc.c->lq))) return rc;
    return right_chain<S>(A, ld, bl, nb, VR, TR, 0, n - 1, st);
}

template <class S>
static int rhess_body(S *A, S *B, S *Q, S *Z, int64_t n, int64_t nb, int64_t p, int64_t ld, S *VL, S *TL, S *VR,
                      S *TR, S1Sched &sc)
{
    int rc = 0;
    const int64_t bm = p * nb;
    // 1. QR of B (panels of nb columns, blocks from the panel's first row)
    for (int64_t c0 = 0; c0 + 1 < n; c0 += nb) {
        const int nc = (int)i64min(nb, n - c0);
        const int64_t rows = n - c0;
        const int64_t nblk = rows <= bm ? 1 : 1 + (rows - bm + (p - 1) * nb - 1) / ((p - 1) * nb);
        const Blocks bl{c0, (p - 1) * nb, bm, nblk, n};
        // B is dense here: every block's reflectors reach all trailing columns
        if ((rc = left_phase<S>(B, A, B, Q, ld, n, bl, c0, nc, VL, TL, 0, c0 + nc, 0, true, sc))) return rc;
    }
    // 2. panels of stage one (1-based j = 1, 1+nb, ...; 0-based first column j-1)
    for (int64_t j = 1; j <= n - 2; j += nb) {
        const int64_t j2 = i64min(n, j + nb - 1);
        const int64_t num = n - nb - j + 1;
        if (num <= 0) break;
        const int64_t nblk = (num + (p - 1) * nb - 1) / ((p - 1) * nb);
        const Blocks bl{j + nb - 1, (p - 1) * nb, bm, nblk, n};
        const int nc = (int)(j2 - j + 1);
        // left: QR of the panel blocks; A right of the panel, B from each block's first column, Q
        if ((rc = left_phase<S>(A, A, B, Q, ld, n, bl, j - 1, nc, VL, TL, j2, bl.r0(0), 1, false, sc))) return rc;
        // right: per block from the bottom; then A and Z
        if ((rc = right_phase<S>(A, B, Z, ld, n, bl, (int)nb, VR, TR, sc))) return rc;
    }
    return 0;
}

template <class S>
static int rhess_impl(S *A, S *B, S *Q, S *Z, int64_t n, int64_t r, int64_t ld, int64_t p, void *stream)
{
    if (n < 0) return -5;
    if (r < 1) return -6;
    if (ld < (n > 1 ? n : 1)) return -7;
    if (n > 0 && !A) return -1;
    if (n > 0 && !B) return -2;
    if (n == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    g_errmsg[0] = 0;
    const int64_t nb = i64min(r, i64max(n - 1, 1));
    if (nb > kS1MaxNB) return HT_ERR_NOTSUP;
    if (p == 0) p = s1_default_p(nb);
    if (p < 2 || p * nb > kS1MaxBM) return -8;
    const int64_t bm = p * nb;
    const int64_t maxblk = n / ((p - 1) * nb) + 2;
    const size_t vb = (size_t)maxblk * bm * nb * sizeof(S), tb = (size_t)maxblk * nb * sizeof(S);
    int rc = 0;
    unsigned char *ws = (unsigned char *)workspace_get(s1_workspace_bytes(n, nb, p, sizeof(S)), st, &rc);
    if (!ws) return rc;
    S *VL = (S *)ws, *TL = (S *)(ws + vb), *VR = (S *)(ws + vb + tb), *TR = (S *)(ws + 2 * vb + tb);
    S1Sched sc;
    sc.st = st;
    const int64_t knob_la = knob(HT_KNOB_LOOKAHEAD);
    if (knob_la == 2 || (knob_la == 1 && n >= kS1OverlapMinN)) {
        sc.c = s1_ctx(st);
        // (every launch on the other streams waits for an event recorded on
        // the caller's stream after the work queued there before this call)
        if (!sc.c) { (void)hipGetLastError(); return 1; }
    }
    rc = rhess_body<S>(A, B, Q, Z, n, nb, p, ld, VL, TL, VR, TR, sc);
    // on every path, the caller's stream covers the work queued on the others
    const int jrc = sc.join();
    if (rc) return rc;
    if (jrc) return jrc;
    hipLaunchKernelGGL(k_s1_zero_pattern<S>, dim3((unsigned)n), dim3(256), 0, st, A, B, ld, n, nb);
    return launch_check("k_s1_zero_pattern");
}

}  // namespace ht

extern "C" {
int64_t ht_rhess_default_p(int64_t n, int64_t r)
{
    if (n < 0 || r < 1) return -1;
    return ht::s1_default_p(ht::i64min(r, ht::i64max(n - 1, 1)));
}
int64_t ht_rhess_workspace_bytes(int64_t n, int64_t r, int64_t p, int is_complex)
{
    if (n < 0 || r < 1 || p < 0) return -1;
    if (n == 0) return 0;
    const int64_t nb = ht::i64min(r, ht::i64max(n - 1, 1));
    if (nb > ht::kS1MaxNB) return -1;
    if (p == 0) p = ht::s1_default_p(nb);
    if (p < 2 || p * nb > ht::kS1MaxBM) return -1;
    return (int64_t)ht::s1_workspace_bytes(n, nb, p, is_complex ? 16 : 8);
}
int ht_rhess(double *A, double *B, double *Q, double *Z, int64_t n, int64_t r, int64_t ld, void *stream)
{
    return ht::rhess_impl<double>(A, B, Q, Z, n, r, ld, 0, stream);
}
int ht_rhess_z(void *A, void *B, void *Q, void *Z, int64_t n, int64_t r, int64_t ld, void *stream)
{
    return ht::rhess_impl<ht::zd>((ht::zd *)A, (ht::zd *)B, (ht::zd *)Q, (ht::zd *)Z, n, r, ld, 0, stream);
}
int ht_rhess_p(double *A, double *B, double *Q, double *Z, int64_t n, int64_t r, int64_t ld, int64_t p, void *stream)
{
    return ht::rhess_impl<double>(A, B, Q, Z, n, r, ld, p, stream);
}
int ht_rhess_z_p(void *A, void *B, void *Q, void *Z, int64_t n, int64_t r, int64_t ld, int64_t p, void *stream)
{
    return ht::rhess_impl<ht::zd>((ht::zd *)A, (ht::zd *)B, (ht::zd *)Q, (ht::zd *)Z, n, r, ld, p, stream);
}
}
