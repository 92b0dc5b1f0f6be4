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
// panel's first row).  All arithmetic is FP64 / complex128.
#include "ht_common.hpp"
#include "ht_workspace.hpp"
#include "ht.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

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
    const double b = -(re(alpha) >= 0.0 ? 1.0 : -1.0) * sqrt(abs2(alpha) + ss);
    tau = mk<S>((b - re(alpha)) / b, -im(alpha) / b);
    beta = mk<S>(b, 0.0);
    scal = recip(sub(alpha, beta));
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
template <class S>
__global__ __launch_bounds__(256) void k_s1_block_qr(S *X, int64_t ld, Blocks bl, int64_t c0, int nc, S *V, S *tau)
{
    __shared__ S P[kS1MaxBM * kS1MaxNB];
    __shared__ double red[4];
    __shared__ S sc[3];
    const int tid = threadIdx.x;
    const int bm = (int)bl.bm;
    for (int64_t k = bl.nblk - 1; k >= 0; --k) {
        const int64_t r0 = bl.r0(k);
        const int m = (int)(bl.r1(k) - r0 + 1);
        {
            constexpr int NT = kS1MaxBM * kS1MaxNB / 256;      // fixed trip count: loads in flight together
            S buf[NT];
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int e = tid + 256 * u, i = e % m, s = e / m;
                buf[u] = e < m * nc ? X[r0 + i + (c0 + s) * ld] : zero<S>();
            }
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int e = tid + 256 * u, i = e % m, s = e / m;
                if (e < m * nc) P[s * bm + i] = buf[u];
            }
        }
        __syncthreads();
        const int ns = m < nc ? m : nc;
        for (int s = 0; s < ns; ++s) {
            double part = 0.0;
            for (int i = s + 1 + tid; i < m; i += 256) part += abs2(P[s * bm + i]);
            const double ss = block_sum256(part, red);
            if (tid == 0) {
                S t, b, f;
                bool triv;
                larfg_scalars(P[s * bm + s], ss, t, b, f, triv);
                sc[0] = t; sc[1] = b; sc[2] = f;
            }
            __syncthreads();
            const S t = sc[0], f = sc[2];
            for (int i = s + 1 + tid; i < m; i += 256) P[s * bm + i] = iszero(t) ? P[s * bm + i] : mul(P[s * bm + i], f);
            if (tid == 0) P[s * bm + s] = sc[1];
            for (int i = tid; i < bm; i += 256) {
                S v = zero<S>();
                if (i == s) v = one<S>();
                else if (i > s && i < m) v = P[s * bm + i];
                V[(k * bm + 0) * nc + s * bm + i] = v;
            }
            if (tid == 0) tau[k * nc + s] = t;
            __syncthreads();
            // apply G^H to the remaining columns of the block: 8 threads per column
            if (!iszero(t)) {
                const int c = s + 1 + (tid >> 3), sub8 = tid & 7;
                S part2 = zero<S>();
                if (c < nc) {
                    for (int i = s + sub8; i < m; i += 8) {
                        const S vi = (i == s) ? one<S>() : P[s * bm + i];
                        part2 = add(part2, cmul(vi, P[c * bm + i]));
                    }
                }
                const S dot = mul(conj_(t), group_sum<8>(part2));
                if (c < nc) {
                    for (int i = s + sub8; i < m; i += 8) {
                        const S vi = (i == s) ? one<S>() : P[s * bm + i];
                        P[c * bm + i] = sub(P[c * bm + i], mul(dot, vi));
                    }
                }
            }
            __syncthreads();
        }
        // R and exact zeros back to X
        for (int e = tid; e < m * nc; e += 256) {
            const int i = e % m, s = e / m;
            X[r0 + i + (c0 + s) * ld] = (i <= s) ? P[s * bm + i] : zero<S>();
        }
        __syncthreads();
    }
}

// Stage block k's reflectors (m x nc, column s at s*bm) and taus into LDS;
// 64 threads, fixed trip counts so that the loads are in flight together.
template <class S>
__device__ inline void stage_refl(S *vs, S *ts, const S *V, const S *tau, int64_t k, int bm, int nc, int t)
{
    const S *Vk = V + k * bm * nc;
    constexpr int CH = 16;
    const int tot = bm * nc;
    for (int e0 = 0; e0 < tot; e0 += 64 * CH) {
        S buf[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + u * 64 + t;
            buf[u] = e < tot ? Vk[e] : zero<S>();
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + u * 64 + t;
            if (e < tot) vs[e] = buf[u];
        }
    }
    if (t < nc) ts[t] = tau[k * nc + t];
}

// ------------------------------------------------------ left chain (columns)
// For k = nblk-1 .. 0: X(block k rows, c) <- Q_k^H X(block k rows, c) for the
// columns c in [cfirst, clast] with c >= (cfrom_block ? r0(k) : cfirst).
// 64 columns per workgroup; the block rows of the columns and the block's
// reflectors are staged in LDS.
template <class S>
__global__ __launch_bounds__(64) void k_s1_left_chain(S *X, int64_t ld, Blocks bl, int nc, const S *V, const S *tau,
                                                      int64_t cfirst, int64_t clast, int cfrom_block)
{
    __shared__ S xs[kS1MaxBM * 65];
    __shared__ S vs[kS1MaxBM * kS1MaxNB];
    __shared__ S ts[kS1MaxNB];
    const int t = threadIdx.x;
    const int64_t cb = cfirst + (int64_t)blockIdx.x * 64;
    const int64_t c = cb + t;
    const int bm = (int)bl.bm;
    constexpr int CH = 16;
    for (int64_t k = bl.nblk - 1; k >= 0; --k) {
        const int64_t r0 = bl.r0(k);
        const int m = (int)(bl.r1(k) - r0 + 1);
        const int64_t clo = cfrom_block ? i64max(cfirst, r0) : cfirst;
        if (cb + 63 < clo) continue;                        // uniform: the workgroup has no column here
        stage_refl(vs, ts, V, tau, k, bm, nc, t);
        // tile: thread t loads row t of the block for 64 columns (coalesced along rows)
        for (int c0 = 0; c0 < 64; c0 += CH) {
            S buf[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int64_t col = cb + c0 + u;
                buf[u] = (t < m && col <= clast) ? X[r0 + t + col * ld] : zero<S>();
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) xs[t * 65 + c0 + u] = buf[u];
        }
        __syncthreads();
        if (c <= clast && c >= clo) {
            const int ns = m < nc ? m : nc;
            for (int s = 0; s < ns; ++s) {
                const S tsv = ts[s];
                if (iszero(tsv)) continue;
                const S *v = vs + s * bm;
                S d0 = zero<S>(), d1 = zero<S>();
                int i = s;
                for (; i + 1 < m; i += 2) { d0 = add(d0, cmul(v[i], xs[i * 65 + t])); d1 = add(d1, cmul(v[i + 1], xs[(i + 1) * 65 + t])); }
                if (i < m) d0 = add(d0, cmul(v[i], xs[i * 65 + t]));
                const S d = mul(conj_(tsv), add(d0, d1));
                for (int ii = s; ii < m; ++ii) xs[ii * 65 + t] = sub(xs[ii * 65 + t], mul(d, v[ii]));
            }
        }
        __syncthreads();
        for (int c0 = 0; c0 < 64; c0 += CH) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int64_t col = cb + c0 + u;
                if (t < m && col <= clast && col >= clo) X[r0 + t + col * ld] = xs[t * 65 + c0 + u];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ right chain (rows)
// For k = nblk-1 .. 0: X(rho, block k columns) <- X(rho, block k columns) G_0
// ... G_{nc-1} for rows rho in [0, rlast]; the block's columns are the block's
// rows (r0(k) .. r1(k)).  64 rows per workgroup, reflectors staged in LDS.
template <class S>
__global__ __launch_bounds__(64) void k_s1_right_chain(S *X, int64_t ld, Blocks bl, int nc, const S *V, const S *tau,
                                                       int64_t rlast)
{
    __shared__ S xs[64 * (kS1MaxBM + 1)];
    __shared__ S vs[kS1MaxBM * kS1MaxNB];
    __shared__ S ts[kS1MaxNB];
    const int t = threadIdx.x;
    const int64_t rho = (int64_t)blockIdx.x * 64 + t;
    const bool ok = rho <= rlast;
    const int bm = (int)bl.bm;
    constexpr int CH = 16;
    S *x = xs + t * (kS1MaxBM + 1);
    for (int64_t k = bl.nblk - 1; k >= 0; --k) {
        const int64_t c0 = bl.r0(k);
        const int m = (int)(bl.r1(k) - c0 + 1);
        __syncthreads();
        stage_refl(vs, ts, V, tau, k, bm, nc, t);
        for (int cc0 = 0; cc0 < kS1MaxBM; cc0 += CH) {
            S buf[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int cc = cc0 + u;
                buf[u] = (ok && cc < m) ? X[rho + (c0 + cc) * ld] : zero<S>();
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) x[cc0 + u] = buf[u];
        }
        __syncthreads();
        if (ok) {
            const int ns = m < nc ? m : nc;
            for (int s = 0; s < ns; ++s) {
                const S tsv = ts[s];
                if (iszero(tsv)) continue;
                const S *v = vs + s * bm;
                S d0 = zero<S>(), d1 = zero<S>();
                int i = s;
                for (; i + 1 < m; i += 2) { d0 = add(d0, mul(x[i], v[i])); d1 = add(d1, mul(x[i + 1], v[i + 1])); }
                if (i < m) d0 = add(d0, mul(x[i], v[i]));
                const S d = mul(add(d0, d1), tsv);
                for (int ii = s; ii < m; ++ii) x[ii] = sub(x[ii], mul(d, conj_(v[ii])));
            }
            for (int cc = 0; cc < m; ++cc) X[rho + (c0 + cc) * ld] = x[cc];
        }
    }
}

// ------------------------------------------------ right factor (one block)
// RQ of B(block k, block k) = Rt Qt (Householder, last row first, the
// reflector vectors kept in the annihilated part of the row), the first nr
// rows of Qt, and their LQ factorisation: reflectors P_t (acting on local
// columns t..m-1, zeros above) into VR[k*bm*nc + t*bm + i], tau into
// tauR[k*nc + t].
template <class S>
__global__ __launch_bounds__(256) void k_s1_right_factor(const S *B, int64_t ld, Blocks bl, int64_t k, int nb,
                                                         S *VR, S *tauR)
{
    __shared__ S W[kS1MaxBM * (kS1MaxBM + 1)];       // W[i*(bm+1) + c] row-major
    __shared__ S Yc[kS1MaxBM * kS1MaxNB];            // Yc[c*bm + i] = Y(i, c), c < nr
    __shared__ S ut[kS1MaxBM];                       // tau of the RQ reflectors
    __shared__ S M[kS1MaxNB * (kS1MaxBM + 1)];       // M[t*(bm+1) + c]
    __shared__ double red[4];
    __shared__ S sc[3];
    __shared__ S dots[kS1MaxNB];
    const int tid = threadIdx.x;
    const int bm = (int)bl.bm, LW = bm + 1;
    const int64_t r0 = bl.r0(k);
    const int m = (int)(bl.r1(k) - r0 + 1);
    const int nr = m < nb ? m : nb;
    {
        constexpr int NT = kS1MaxBM * kS1MaxBM / 256;      // fixed trip count: loads in flight together
        S buf[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int e = tid + 256 * u, i = e % m, c = e / m;
            buf[u] = e < m * m ? B[r0 + i + (r0 + c) * ld] : zero<S>();
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int e = tid + 256 * u, i = e % m, c = e / m;
            if (e < m * m) W[i * LW + c] = buf[u];
        }
    }
    __syncthreads();
    // RQ, rows m-1 .. 1: u = conj(row i)(0..i), larfg with alpha = u_i
    for (int i = m - 1; i >= 1; --i) {
        double part = 0.0;
        for (int c = tid; c < i; c += 256) part += abs2(W[i * LW + c]);
        const double ss = block_sum256(part, red);
        if (tid == 0) {
            S t, b, f;
            bool triv;
            larfg_scalars(conj_(W[i * LW + i]), ss, t, b, f, triv);
            sc[0] = t; sc[1] = b; sc[2] = f;
            ut[i] = t;
        }
        __syncthreads();
        const S t = sc[0], f = sc[2];
        // u_c = conj(W[i][c]) * f (c < i), stored in place; u_i = 1
        for (int c = tid; c < i; c += 256) W[i * LW + c] = iszero(t) ? zero<S>() : mul(conj_(W[i * LW + c]), f);
        __syncthreads();
        if (!iszero(t)) {
            // rows 0..i-1: W(r, 0:i) <- W(r, 0:i) (I - t u u^H); 4 threads per row
            for (int rb = 0; rb < i; rb += 64) {
                const int r = rb + (tid >> 2), sub4 = tid & 3;
                S part2 = zero<S>();
                if (r < i)
                    for (int c = sub4; c <= i; c += 4) {
                        const S uc = (c == i) ? one<S>() : W[i * LW + c];
                        part2 = add(part2, mul(W[r * LW + c], uc));
                    }
                const S d = mul(group_sum<4>(part2), t);
                if (r < i)
                    for (int c = sub4; c <= i; c += 4) {
                        const S uc = (c == i) ? one<S>() : W[i * LW + c];
                        W[r * LW + c] = sub(W[r * LW + c], mul(d, conj_(uc)));
                    }
            }
        }
        __syncthreads();
    }
    // Yc = U_{m-1} ... U_1 [e_0 .. e_{nr-1}]
    for (int e = tid; e < m * nr; e += 256) {
        const int i = e % m, c = e / m;
        Yc[c * bm + i] = (i == c) ? one<S>() : zero<S>();
    }
    __syncthreads();
    for (int i = 1; i < m; ++i) {
        const S t = ut[i];
        if (iszero(t)) continue;
        // dots_c = u^H Yc(0:i, c), 8 threads per column
        {
            const int c = tid >> 3, sub8 = tid & 7;
            S part2 = zero<S>();
            if (c < nr)
                for (int ii = sub8; ii <= i; ii += 8) {
                    const S uc = (ii == i) ? one<S>() : W[i * LW + ii];
                    part2 = add(part2, cmul(uc, Yc[c * bm + ii]));
                }
            const S d = mul(group_sum<8>(part2), t);
            if (c < nr && sub8 == 0) dots[c] = d;
        }
        __syncthreads();
        for (int e = tid; e < (i + 1) * nr; e += 256) {
            const int ii = e % (i + 1), c = e / (i + 1);
            const S uc = (ii == i) ? one<S>() : W[i * LW + ii];
            Yc[c * bm + ii] = sub(Yc[c * bm + ii], mul(dots[c], uc));
        }
        __syncthreads();
    }
    // M = Qt(0:nr, :) = Yc^H
    for (int e = tid; e < m * nr; e += 256) {
        const int c = e % m, tt = e / m;
        M[tt * LW + c] = conj_(Yc[tt * bm + c]);
    }
    __syncthreads();
    // LQ of M: for row t, reflector from conj(M(t, t:m)); M(t+1:nr, t:m) <- M P_t
    for (int t = 0; t < nr; ++t) {
        const int len = m - t;
        double part = 0.0;
        for (int c = 1 + tid; c < len; c += 256) part += abs2(M[t * LW + t + c]);
        const double ss = block_sum256(part, red);
        if (tid == 0) {
            S ta, b, f;
            bool triv;
            larfg_scalars(conj_(M[t * LW + t]), ss, ta, b, f, triv);
            sc[0] = ta; sc[1] = b; sc[2] = f;
            tauR[k * nb + t] = ta;
        }
        __syncthreads();
        const S ta = sc[0], f = sc[2];
        // v = [1, conj(M(t, t+1:m)) f]; stored in VR (and kept in M's row t)
        for (int c = tid; c < bm; c += 256) {
            S v = zero<S>();
            if (c == t) v = one<S>();
            else if (c > t && c < m) v = iszero(ta) ? zero<S>() : mul(conj_(M[t * LW + c]), f);
            VR[(k * bm) * nb + t * bm + c] = v;
            if (c > t && c < m) M[t * LW + c] = v;
        }
        __syncthreads();
        if (!iszero(ta)) {
            // rows t+1..nr-1 (at most 31): 8 threads per row
            const int rr = t + 1 + (tid >> 3), sub8 = tid & 7;
            S part2 = zero<S>();
            if (rr < nr)
                for (int c = t + sub8; c < m; c += 8) {
                    const S vc = (c == t) ? one<S>() : M[t * LW + c];
                    part2 = add(part2, mul(M[rr * LW + c], vc));
                }
            const S d = mul(group_sum<8>(part2), ta);
            if (rr < nr)
                for (int c = t + sub8; c < m; c += 8) {
                    const S vc = (c == t) ? one<S>() : M[t * LW + c];
                    M[rr * LW + c] = sub(M[rr * LW + c], mul(d, conj_(vc)));
                }
        }
        __syncthreads();
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

template <class S>
static int left_phase(S *X, S *A2, S *B2, S *Q, int64_t ld, int64_t n, const Blocks &bl, int64_t c0, int nc,
                      S *V, S *tau, int64_t a2first, int64_t b2first, int b2from_block, hipStream_t st)
{
    int rc;
    hipLaunchKernelGGL(k_s1_block_qr<S>, dim3(1), dim3(256), 0, st, X, ld, bl, c0, nc, V, tau);
    if ((rc = launch_check("k_s1_block_qr"))) return rc;
    // X's own columns right of the panel (or A for the QR of B)
    if (A2 && a2first <= n - 1) {
        const int64_t ncols = n - a2first;
        hipLaunchKernelGGL(k_s1_left_chain<S>, dim3((unsigned)((ncols + 63) / 64)), dim3(64), 0, st, A2, ld, bl, nc,
                           (const S *)V, (const S *)tau, a2first, n - 1, 0);
        if ((rc = launch_check("k_s1_left_chain"))) return rc;
    }
    if (B2 && b2first <= n - 1) {
        const int64_t ncols = n - b2first;
        hipLaunchKernelGGL(k_s1_left_chain<S>, dim3((unsigned)((ncols + 63) / 64)), dim3(64), 0, st, B2, ld, bl, nc,
                           (const S *)V, (const S *)tau, b2first, n - 1, b2from_block);
        if ((rc = launch_check("k_s1_left_chain"))) return rc;
    }
    if (Q) {
        hipLaunchKernelGGL(k_s1_right_chain<S>, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, Q, ld, bl, nc,
                           (const S *)V, (const S *)tau, n - 1);
        if ((rc = launch_check("k_s1_right_chain"))) return rc;
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
    unsigned char *ws = (unsigned char *)workspace_get(2 * (vb + tb) + 1024, st, &rc);
    if (!ws) return rc;
    S *VL = (S *)ws, *TL = (S *)(ws + vb), *VR = (S *)(ws + vb + tb), *TR = (S *)(ws + 2 * vb + tb);
    // 1. QR of B (panels of nb columns, blocks from the panel's first row)
    for (int64_t c0 = 0; c0 + 1 < n; c0 += nb) {
        const int nc = (int)i64min(nb, n - c0);
        const int64_t rows = n - c0;
        const int64_t nblk = rows <= bm ? 1 : 1 + (rows - bm + (p - 1) * nb - 1) / ((p - 1) * nb);
        const Blocks bl{c0, (p - 1) * nb, bm, nblk, n};
        // B is dense here: every block's reflectors reach all trailing columns
        if ((rc = left_phase<S>(B, A, B, Q, ld, n, bl, c0, nc, VL, TL, 0, c0 + nc, 0, st))) return rc;
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
        if ((rc = left_phase<S>(A, A, B, Q, ld, n, bl, j - 1, nc, VL, TL, j2, bl.r0(0), 1, st))) return rc;
        // right: per block from the bottom
        for (int64_t k = nblk - 1; k >= 0; --k) {
            hipLaunchKernelGGL(k_s1_right_factor<S>, dim3(1), dim3(256), 0, st, (const S *)B, ld, bl, k, (int)nb, VR, TR);
            if ((rc = launch_check("k_s1_right_factor"))) return rc;
            // B(0:i2, block k columns) <- B P_0 ... P_{nb-1}: the row chain with this block only
            const int64_t rows = bl.r1(k) + 1;
            const Blocks one_blk{bl.r0(k), bl.step, bm, 1, n};
            hipLaunchKernelGGL(k_s1_right_chain<S>, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0, st, B, ld, one_blk,
                               (int)nb, (const S *)(VR + k * bm * nb), (const S *)(TR + k * nb), rows - 1);
            if ((rc = launch_check("k_s1_right_chain"))) return rc;
            hipLaunchKernelGGL(k_s1_zero_block<S>, dim3(1), dim3(256), 0, st, B, ld, bl, k, (int)nb);
            if ((rc = launch_check("k_s1_zero_block"))) return rc;
        }
        hipLaunchKernelGGL(k_s1_right_chain<S>, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, A, ld, bl, (int)nb,
                           (const S *)VR, (const S *)TR, n - 1);
        if ((rc = launch_check("k_s1_right_chain"))) return rc;
        if (Z) {
            hipLaunchKernelGGL(k_s1_right_chain<S>, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, Z, ld, bl, (int)nb,
                               (const S *)VR, (const S *)TR, n - 1);
            if ((rc = launch_check("k_s1_right_chain"))) return rc;
        }
    }
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
