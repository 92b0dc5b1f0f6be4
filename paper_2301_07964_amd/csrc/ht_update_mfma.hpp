// ht_update_mfma.hpp -- application phase of blocked stage two on the FP64
// matrix cores (Section 3.2, "Applying the reflectors"; application algorithm
// of the appendix), r in {4, 8, 16, 32}; real arithmetic first, the complex
// variant at the end.
//
// The q reflectors of window k (local indices 0 .. W-1, W = q+r-1, the w-th
// reflector acting on w .. w+r-1) are first accumulated into the window's
// orthogonal factor U_k = G_0 G_1 ... G_{q-1}, embedded in the identity of
// order KW = max(16, 2r) (k_form_factors).  Right updates then compute
// X(:, window) <- X(:, window) U_k and left updates X(window, :) <-
// U_k^H X(window, :), as the paper's delayed updates do with its window
// factors, windows from the bottom (k = kmax-1) to the top.
//
// MFMA formulation (v_mfma_f64_16x16x4f64: D = A B + C with A 16x4, B 4x16;
// lane l holds A[l%16][l/16], B[l/16][l%16] and D[4v + l/16][l%16], v < 4):
//   right:  D^T = U^T X^T  for a tile of 16 rows of X,
//   left:   D   = U^T X    for a tile of 16 columns (real case: U^H = U^T),
// so in both cases A is a fragment of U^T and B holds the tile with lane l
// on row/column l%16 and window index 4kk + l/16 in register kk.  The result
// lands with window index 16mb + 4v + l/16 in register (mb, v) of lane l,
// which is exactly where the B operand of the next step wants index
// 4(4mb+v) + l/16: the window ring stays in registers without any exchange.
// Consecutive windows overlap in q-1 indices (local c of window k is local
// c + r of window k-1), so the carried registers shift by r/4.
#pragma once
#include "ht_common.hpp"
#include "ht_update.hpp"

namespace ht {

// Store of a finished entry of the real update kernels: a relaxed store at
// system scope, which writes through the L2 instead of leaving the line dirty
// there.  The generation kernel runs beside these kernels (lookahead) and
// writes back its XCD's whole L2 at every step's release; with fewer dirty
// lines from the updates, those write-backs are shorter (n = 16384, r = 32:
// 5.37 s to 5.27 s per reduction; nontemporal stores: 5.32 s).  No ordering
// is implied: the kernels' results are ordered by stream order and the
// lookahead flags as before.
__device__ __forceinline__ void st_out(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// order of the embedded window factor for block size R
template <int R> struct KWOf { static constexpr int value = (2 * R < 16) ? 16 : 2 * R; };

// Window factors.  Grid (kmax, 2): blockIdx.y = 0 uses the left reflectors,
// 1 the right reflectors; one wavefront per window, lane i computes row i of
// U_k.  Output: F[(side*kext + k)*KW*KW + (mb*KK + kk)*64 + l]
//             = U_k[4kk + l/16][16mb + l%16]   (the A fragments of U_k^T).
template <int R, int KW>
__global__ __launch_bounds__(64) void k_form_factors(int64_t q, int64_t kext, const double *VL, const double *TL,
                                                     const double *VR, const double *TR, double *F)
{
    constexpr int MB = KW / 16, KK = KW / 4;
    const int64_t k = blockIdx.x;
    const int side = blockIdx.y;
    const int lane = threadIdx.x;
    const double *V = side ? VR : VL;
    const double *Tv = side ? TR : TL;
    double u[KW];
#pragma unroll
    for (int c = 0; c < KW; ++c) u[c] = (c == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int w = 0; w < R; ++w) {
        if (w < q) {
            const double tau = Tv[w * kext + k];
            if (tau != 0.0) {
                const double *v = V + (w * kext + k) * R;
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int c = 0; c < R; c += 2) {
                    s0 += u[w + c] * v[c];
                    s1 += u[w + c + 1] * v[c + 1];
                }
                const double s = (s0 + s1) * tau;
#pragma unroll
                for (int c = 0; c < R; ++c) u[w + c] -= s * v[c];
            }
        }
    }
    __shared__ double tr[KW][KW + 1];
    if (lane < KW) {
#pragma unroll
        for (int c = 0; c < KW; ++c) tr[lane][c] = u[c];
    }
    __syncthreads();
    double *out = F + ((int64_t)side * kext + k) * (KW * KW);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
            out[(mb * KK + kk) * 64 + lane] = tr[4 * kk + (lane >> 4)][16 * mb + (lane & 15)];
}

// Delayed updates on the matrix cores.  256 threads = 4 independent
// wavefronts; each owns TRW tiles of 16 rows (right) or 16 columns (left) of
// one job's matrix and streams them through the windows.  Jobs: as for the
// vector kernels (UpdJob), with npanels counted in wavefront tiles of 16*TRW.
template <int R, int TRW, bool LEFT>
__global__ __launch_bounds__(256) void k_update_mfma(UpdArgs<double> a, const double *F)
{
    constexpr int KW = KWOf<R>::value;
    constexpr int MB = KW / 16, KK = KW / 4, RS = R / 4;
    const int lane = threadIdx.x & 63;
    int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int jid = 0;
    while (jid < a.njobs - 1 && b >= a.job[jid].npanels) { b -= a.job[jid].npanels; ++jid; }
    UpdJob<double> J = a.job[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) if (jid == i) J = a.job[i];
    if (b >= J.npanels) return;
    const int64_t n = a.n, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    // left with lookahead epilogues: from the first tile the next group's
    // generation reads rightwards, the tiles left of it last
    const bool epi = LEFT && a.epi.flags != nullptr;
    if (epi) b = (b + (a.epi.c0 < n ? a.epi.c0 / (16 * TRW) : 0)) % J.npanels;
    const int64_t W = q + R - 1;
    const int g = lane >> 4, li = lane & 15;
    const int64_t p0 = b * (16 * TRW);              // first row (right) / column (left) of the tiles
    const double *Fs = F + (LEFT ? 0 : (int64_t)J.side * kext * (KW * KW));
    double *X = J.X;
    const int64_t ld = J.ld;

    // windows this wavefront has to apply (same limits as the vector kernels)
    int64_t kfirst = kmax - 1, klast = 0;
    if (J.lim >= 0) {
        if (!LEFT) {
            while (klast < kmax && !(p0 < i64min(j1 + klast * R + W - 1, n - 1) + 1 + J.lim)) ++klast;
            if (klast >= kmax) return;
        } else {
            while (kfirst >= 0 && !(p0 + 16 * TRW > j1 + kfirst * R - J.lim)) --kfirst;
            if (kfirst < 0 && !epi) return;
        }
    }
    if (kfirst >= klast) {                         // the tiles take part in at least one window
        // element (tile t, window index c) of window starting at lo
        auto addr = [&](int t, int64_t lo, int c, bool &ok) -> int64_t {
            const int64_t fixed = p0 + 16 * t + li, idx = lo + c;
            ok = fixed < n && idx < n;
            return LEFT ? idx + fixed * ld : fixed + idx * ld;
        };

        double xb[TRW][KK];
        {
            const int64_t lo = j1 + kfirst * R;
#pragma unroll
            for (int t = 0; t < TRW; ++t)
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int c = 4 * kk + g;
                    bool ok;
                    const int64_t ad = addr(t, lo, c, ok);
                    double v = 0.0;
                    if (ok && c < W) v = X[ad];
                    xb[t][kk] = v;
                }
        }
        for (int64_t k = kfirst; k >= klast; --k) {
            const int64_t lo = j1 + k * R;
            const double *Fk = Fs + k * (KW * KW);
            f64x4 acc[TRW][MB];
#pragma unroll
            for (int t = 0; t < TRW; ++t)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                double af[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) af[mb] = Fk[(mb * KK + kk) * 64 + lane];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int t = 0; t < TRW; ++t)
                        acc[t][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mb], xb[t][kk], acc[t][mb], 0, 0, 0);
            }
            // finished indices go back to HBM
            const int64_t f0 = (k == klast) ? 0 : q - 1;
#pragma unroll
            for (int t = 0; t < TRW; ++t)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int c = 16 * mb + 4 * v + g;
                        bool ok;
                        const int64_t ad = addr(t, lo, c, ok);
                        if (ok && c >= f0 && c < W) st_out(X + ad, acc[t][mb][v]);
                    }
            if (k == klast) break;
            // carry local 0 .. q-2 to local r .. W-1 of window k-1, load its new
            // indices 0 .. r-1
            const int64_t lon = lo - R;
#pragma unroll
            for (int t = 0; t < TRW; ++t) {
#pragma unroll
                for (int kk = 0; kk < RS; ++kk) {
                    const int c = 4 * kk + g;
                    xb[t][kk + RS] = (c < q - 1) ? acc[t][kk >> 2][kk & 3] : 0.0;
                }
#pragma unroll
                for (int kk = 0; kk < RS; ++kk) {
                    const int c = 4 * kk + g;
                    bool ok;
                    const int64_t ad = addr(t, lon, c, ok);
                    double v = 0.0;
                    if (ok) v = X[ad];
                    xb[t][kk] = v;
                }
            }
        }
    }
    if (epi) {
        // the wavefront's last window is in memory; the epilogue's loads may
        // read what other lanes stored
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        left_epilogue<double>(a, J, p0, 16 * TRW, lane, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) {
#pragma unroll
            for (int t = 0; t < TRW; ++t)            // flags of the tiles of 16 columns that exist
                if (b * TRW + t < (n + 15) / 16)
                    __hip_atomic_fetch_add(a.epi.flags + b * TRW + t, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace ht

namespace ht {

// ---------------------------------------------------------------- complex
// Complex128 variant.  A complex product on the FP64 matrix cores takes four
// real ones: Re D += Re A Re B - Im A Im B, Im D += Re A Im B + Im A Re B.
// The window factor is stored as two real planes of fragments of U^T; right
// updates use A = U^T, left updates A = U^H, whose imaginary plane is the
// stored one negated (the left reflectors' factor serves both: the left
// updates of H and T, and the right update of Q).

// Window factors, complex.  Grid (kmax, 2) as for the real kernel; lane i
// forms row i of U_k in LDS.  Output plane p (0 real, 1 imaginary):
//   F[((side*kext + k)*2 + p)*KW*KW + (mb*KK + kk)*64 + l]
//     = (Re, Im) U_k[4kk + l/16][16mb + l%16].
template <int R, int KW>
__global__ __launch_bounds__(64) void k_form_factors_z(int64_t q, int64_t kext, const zd *VL, const zd *TL,
                                                       const zd *VR, const zd *TR, double *F)
{
    constexpr int MB = KW / 16, KK = KW / 4, LU = KW + 1;
    const int64_t k = blockIdx.x;
    const int side = blockIdx.y;
    const int lane = threadIdx.x;
    const zd *V = side ? VR : VL;
    const zd *Tv = side ? TR : TL;
    __shared__ zd us[KW * LU];                      // row i of U_k at us[i*LU + c]
    __shared__ zd vs[R];
    zd *u = us + lane * LU;
    if (lane < KW) {
        for (int c = 0; c < KW; ++c) u[c] = (c == lane) ? one<zd>() : zero<zd>();
    }
    for (int w = 0; w < R; ++w) {
        if (w >= q) break;                          // uniform
        const zd tau = Tv[w * kext + k];
        if (iszero(tau)) continue;                  // uniform
        __syncthreads();
        if (lane < R) vs[lane] = V[(w * kext + k) * R + lane];
        __syncthreads();
        if (lane < KW) {                            // row <- row (I - tau v v^H)
            zd s = zero<zd>();
            for (int c = 0; c < R; ++c) s = add(s, mul(u[w + c], vs[c]));
            s = mul(s, tau);
            for (int c = 0; c < R; ++c) u[w + c] = sub(u[w + c], mul(s, conj_(vs[c])));
        }
    }
    __syncthreads();
    double *out = F + ((int64_t)side * kext + k) * 2 * (KW * KW);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const zd e = us[(4 * kk + (lane >> 4)) * LU + 16 * mb + (lane & 15)];
            out[(mb * KK + kk) * 64 + lane] = e.re;
            out[KW * KW + (mb * KK + kk) * 64 + lane] = e.im;
        }
}

// Delayed updates on the matrix cores, complex.  Same tiling, window ring and
// job handling as the real kernel (one tile of 16 rows / columns per
// wavefront), with the real and imaginary parts of the tile and of the
// accumulators in separate registers.
template <int R, bool LEFT>
__global__ __launch_bounds__(256) void k_update_mfma_z(UpdArgs<zd> a, const double *F)
{
    constexpr int KW = KWOf<R>::value;
    constexpr int MB = KW / 16, KK = KW / 4, RS = R / 4;
    const int lane = threadIdx.x & 63;
    int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int jid = 0;
    while (jid < a.njobs - 1 && b >= a.job[jid].npanels) { b -= a.job[jid].npanels; ++jid; }
    UpdJob<zd> J = a.job[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) if (jid == i) J = a.job[i];
    if (b >= J.npanels) return;
    const int64_t n = a.n, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    // left with lookahead epilogues: from the first tile the next group's
    // generation reads rightwards, the tiles left of it last
    const bool epi = LEFT && a.epi.flags != nullptr;
    if (epi) b = (b + (a.epi.c0 < n ? a.epi.c0 / 16 : 0)) % J.npanels;
    const int64_t W = q + R - 1;
    const int g = lane >> 4, li = lane & 15;
    const int64_t p0 = b * 16;                      // first row (right) / column (left) of the tile
    const double *Fs = F + (LEFT ? 0 : (int64_t)J.side * kext * 2 * (KW * KW));
    zd *X = J.X;
    const int64_t ld = J.ld;

    int64_t kfirst = kmax - 1, klast = 0;
    if (J.lim >= 0) {
        if (!LEFT) {
            while (klast < kmax && !(p0 < i64min(j1 + klast * R + W - 1, n - 1) + 1 + J.lim)) ++klast;
            if (klast >= kmax) return;
        } else {
            while (kfirst >= 0 && !(p0 + 16 > j1 + kfirst * R - J.lim)) --kfirst;
            if (kfirst < 0 && !epi) return;
        }
    }
    if (kfirst >= klast) {                         // the tile takes part in at least one window
        auto addr = [&](int64_t lo, int c, bool &ok) -> int64_t {
            const int64_t fixed = p0 + li, idx = lo + c;
            ok = fixed < n && idx < n;
            return LEFT ? idx + fixed * ld : fixed + idx * ld;
        };

        double xr[KK], xi[KK];
        {
            const int64_t lo = j1 + kfirst * R;
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const int c = 4 * kk + g;
                bool ok;
                const int64_t ad = addr(lo, c, ok);
                zd v = zero<zd>();
                if (ok && c < W) v = X[ad];
                xr[kk] = v.re;
                xi[kk] = v.im;
            }
        }
        for (int64_t k = kfirst; k >= klast; --k) {
            const int64_t lo = j1 + k * R;
            const double *Fr = Fs + k * 2 * (KW * KW), *Fi = Fr + KW * KW;
            // the next window's new indices (lo-r .. lo-1) are not written by this
            // window: load them now so that their latency overlaps the products
            double nr[RS], ni[RS];
#pragma unroll
            for (int kk = 0; kk < RS; ++kk) {
                const int c = 4 * kk + g;
                bool ok;
                const int64_t ad = addr(lo - R, c, ok);
                zd v = zero<zd>();
                if (ok && k > klast) v = X[ad];
                nr[kk] = v.re;
                ni[kk] = v.im;
            }
            f64x4 ar[MB], ai[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) { ar[mb] = f64x4{0.0, 0.0, 0.0, 0.0}; ai[mb] = f64x4{0.0, 0.0, 0.0, 0.0}; }
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                double fr[MB], fi[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    fr[mb] = Fr[(mb * KK + kk) * 64 + lane];
                    fi[mb] = LEFT ? -Fi[(mb * KK + kk) * 64 + lane] : Fi[(mb * KK + kk) * 64 + lane];
                }
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    ar[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[mb], xr[kk], ar[mb], 0, 0, 0);
                    ar[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fi[mb], xi[kk], ar[mb], 0, 0, 0);
                    ai[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[mb], xi[kk], ai[mb], 0, 0, 0);
                    ai[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fi[mb], xr[kk], ai[mb], 0, 0, 0);
                }
            }
            const int64_t f0 = (k == klast) ? 0 : q - 1;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = 16 * mb + 4 * v + g;
                    bool ok;
                    const int64_t ad = addr(lo, c, ok);
                    if (ok && c >= f0 && c < W) X[ad] = mk<zd>(ar[mb][v], ai[mb][v]);
                }
            if (k == klast) break;
#pragma unroll
            for (int kk = 0; kk < RS; ++kk) {
                const int c = 4 * kk + g;
                const bool keep = c < q - 1;
                xr[kk + RS] = keep ? ar[kk >> 2][kk & 3] : 0.0;
                xi[kk + RS] = keep ? ai[kk >> 2][kk & 3] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < RS; ++kk) { xr[kk] = nr[kk]; xi[kk] = ni[kk]; }
        }
    }
    if (epi) {
        // the wavefront's last window is in memory; the epilogue's loads may
        // read what other lanes stored
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        left_epilogue<zd>(a, J, p0, 16, lane, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_fetch_add(a.epi.flags + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace ht

namespace ht {

// Delayed updates, real, r = 32, one tile of NL = 16 TC rows (right) or
// columns (left) per workgroup.  The four wavefronts split each window's
// product by output index (wavefront v forms indices 16v .. 16v+15 of the
// window for all NL lines, with its quarter of the factor), so a tile's
// sequence of windows advances at a quarter of the matrix-core time per
// window and each factor fragment serves TC line blocks.  The tile's window
// lives in LDS (the current window and the next); finished indices leave
// through a staging buffer with stores that run along the contiguous
// dimension; the next window's new indices and factor fragments are loaded
// before the current window's products.  Tiles with the longest sequences of
// windows (top rows for right updates, rightmost columns for left updates)
// are dispatched first, jobs interleaved.  The library launches both forms
// with TC = 1: the left form always at r = 32, the right form for H and T in
// the lookahead schedule (where no Q, Z update runs beside it; beside one, it
// was no faster over a whole reduction).  TC = 2 was no faster.
template <int R, bool LEFT, int TC>
__global__ __launch_bounds__(256) void k_update_mfma_coop(UpdArgs<double> a, const double *F)
{
    static_assert(R == 32, "one 16-index block of the window factor per wavefront");
    constexpr int KW = KWOf<R>::value, KK = KW / 4, LT = KW + 1, NL = 16 * TC;
    __shared__ double buf[2][NL * LT];             // tile line j, window index c at [j*LT + c]
    __shared__ double ob[2][NL * LT];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jid = (int)(blockIdx.x % a.njobs);
    UpdJob<double> J = a.job[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) if (jid == i) J = a.job[i];
    const int64_t bi = (int64_t)(blockIdx.x / a.njobs), n_ = a.n;
    // left: rightmost tiles (most windows) first, unless the next group's
    // generation waits for the tiles' epilogues: then from the first tile it
    // reads rightwards, the tiles left of it last
    const bool epi = LEFT && a.epi.flags != nullptr;
    const int64_t b = !LEFT ? bi : !epi ? J.npanels - 1 - bi : (bi + (a.epi.c0 < n_ ? a.epi.c0 / NL : 0)) % J.npanels;
    if (b < 0 || b >= J.npanels) return;
    const int64_t n = a.n, q = a.q, j1 = a.j1, kmax = a.kmax, kext = a.kext;
    const int W = (int)(q + R - 1);
    const int g = lane >> 4, li = lane & 15;
    const int64_t p0 = b * NL;
    const double *Fs = F + (LEFT ? 0 : (int64_t)J.side * kext * (KW * KW));
    double *X = J.X;
    const int64_t ld = J.ld;

    int64_t kfirst = kmax - 1, klast = 0;
    if (J.lim >= 0) {
        if (!LEFT) {
            while (klast < kmax && !(p0 < i64min(j1 + klast * R + W - 1, n - 1) + 1 + J.lim)) ++klast;
            if (klast >= kmax) return;
        } else {
            while (kfirst >= 0 && !(p0 + NL > j1 + kfirst * R - J.lim)) --kfirst;
            if (kfirst < 0 && !epi) return;
        }
    }
    if (kfirst >= klast) {                         // the tile takes part in at least one window
        // element (tile line j, window index c) of the window starting at lo
        auto at = [&](int j, int64_t lo, int c, bool &ok) -> int64_t {
            const int64_t fixed = p0 + j, idx = lo + c;
            ok = fixed < n && idx < n;
            return LEFT ? idx + fixed * ld : fixed + idx * ld;
        };
        // element e of a whole window (NL x 64) or of the new indices (NL x R),
        // the contiguous dimension fastest
        auto wmap = [&](int e, int &j, int &c) { if (LEFT) { c = e & 63; j = e >> 6; } else { j = e % NL; c = e / NL; } };
        auto nmap = [&](int e, int &j, int &c) { if (LEFT) { c = e % R; j = e / R; } else { j = e % NL; c = e / NL; } };
        {
            const int64_t lo = j1 + kfirst * R;
#pragma unroll
            for (int i = 0; i < 4 * TC; ++i) {
                int j, c;
                wmap(tid + 256 * i, j, c);
                bool ok;
                const int64_t ad = at(j, lo, c, ok);
                buf[0][j * LT + c] = (ok && c < W) ? X[ad] : 0.0;
                buf[1][j * LT + c] = 0.0;              // indices >= W of the other buffer stay zero
            }
        }
        double pre[2 * TC];
        auto load_new = [&](int64_t kn) {
            const int64_t lo = j1 + kn * R;
#pragma unroll
            for (int i = 0; i < 2 * TC; ++i) {
                int j, c;
                nmap(tid + 256 * i, j, c);
                bool ok;
                const int64_t ad = at(j, lo, c, ok);
                pre[i] = ok ? X[ad] : 0.0;
            }
        };
        if (kfirst > klast) load_new(kfirst - 1);
        double af[KK];
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) af[kk] = Fs[kfirst * (KW * KW) + (wv * KK + kk) * 64 + lane];
        __syncthreads();
        int cur = 0;
        for (int64_t k = kfirst; k >= klast; --k) {
            const int64_t lo = j1 + k * R;
            const bool more = k > klast;
            double afn[KK];
            if (more) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) afn[kk] = Fs[(k - 1) * (KW * KW) + (wv * KK + kk) * 64 + lane];
            }
            f64x4 acc[TC];
#pragma unroll
            for (int t = 0; t < TC; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk)
#pragma unroll
                for (int t = 0; t < TC; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk], buf[cur][(16 * t + li) * LT + 4 * kk + g], acc[t],
                                                                  0, 0, 0);
            const int f0 = more ? (int)(q - 1) : 0;
            const int nxt = cur ^ 1;
            double *ow = ob[k & 1];
#pragma unroll
            for (int t = 0; t < TC; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = 16 * wv + 4 * v + g, j = 16 * t + li;
                    if (c >= f0 && c < W) ow[j * LT + c] = acc[t][v];
                    if (more && c < q - 1) buf[nxt][j * LT + c + R] = acc[t][v];    // index c + R of window k-1
                }
            if (more) {
#pragma unroll
                for (int i = 0; i < 2 * TC; ++i) {
                    int j, c;
                    nmap(tid + 256 * i, j, c);
                    buf[nxt][j * LT + c] = pre[i];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4 * TC; ++i) {
                int j, c;
                wmap(tid + 256 * i, j, c);
                bool ok;
                const int64_t ad = at(j, lo, c, ok);
                if (ok && c >= f0 && c < W) st_out(X + ad, ow[j * LT + c]);
            }
            if (!more) break;
            if (k - 1 > klast) load_new(k - 2);
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) af[kk] = afn[kk];
            cur = nxt;
        }
    }
    if (epi) {
        __syncthreads();                           // the tile's last window is in memory
        left_epilogue<double>(a, J, p0, NL, tid, 256);
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
            for (int t = 0; t < TC; ++t)
                __hip_atomic_fetch_add(a.epi.flags + b * TC + t, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Left updates, complex, r = 32: the four-wavefront tile scheme of
// k_update_mfma_coop (left form, TC = 1) for complex data (four real products
// per complex one, A = U^H).  One finished-row staging buffer, so two
// barriers per window.
template <int R>
__global__ __launch_bounds__(256) void k_update_mfma_z_coop_left(UpdArgs<zd> a, const double *F)
{
    static_assert(R == 32, "one 16-index block of the window factor per wavefront");
    constexpr int KW = KWOf<R>::value, KK = KW / 4, LT = KW + 1;
    __shared__ zd buf[2][16 * LT];                 // column j, window index c at [j*LT + c]
    __shared__ zd ob[16 * LT];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jid = (int)(blockIdx.x % a.njobs);
    UpdJob<zd> J = a.job[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) if (jid == i) J = a.job[i];
    // rightmost tiles (most windows) first, unless the next group's
    // generation waits for the tiles' epilogues: then from the first tile it
    // reads rightwards, the tiles left of it last
    const bool epi = a.epi.flags != nullptr;
    const int64_t bi = (int64_t)(blockIdx.x / a.njobs);
    if (bi >= J.npanels) return;
    const int64_t n = a.n, q = a.q, j1 = a.j1, kmax = a.kmax;
    const int64_t b = !epi ? J.npanels - 1 - bi : (bi + (a.epi.c0 < n ? a.epi.c0 / 16 : 0)) % J.npanels;
    const int W = (int)(q + R - 1);
    const int g = lane >> 4, li = lane & 15;
    const int64_t p0 = b * 16;
    zd *X = J.X;
    const int64_t ld = J.ld;

    int64_t kfirst = kmax - 1;
    const int64_t klast = 0;
    if (J.lim >= 0) {
        while (kfirst >= 0 && !(p0 + 16 > j1 + kfirst * R - J.lim)) --kfirst;
        if (kfirst < 0 && !epi) return;
    }
    if (kfirst >= klast) {                         // the tile takes part in at least one window
        // whole window: row tid % 64 of columns tid / 64 + 4i; new rows: row
        // tid % 32 of columns tid / 32 + 8i
        const int wr = tid & 63, wc = tid >> 6, nr = tid & 31, nc = tid >> 5;
        {
            const int64_t lo = j1 + kfirst * R;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = wc + 4 * i;
                const int64_t col = p0 + j, row = lo + wr;
                zd v = zero<zd>();
                if (wr < W && col < n && row < n) v = X[row + col * ld];
                buf[0][j * LT + wr] = v;
                buf[1][j * LT + wr] = zero<zd>();      // indices >= W of the other buffer stay zero
            }
        }
        zd pre[2];
        auto load_new = [&](int64_t kn) {
            const int64_t lo = j1 + kn * R;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int64_t col = p0 + nc + 8 * i, row = lo + nr;
                pre[i] = (col < n && row < n) ? X[row + col * ld] : zero<zd>();
            }
        };
        if (kfirst > 0) load_new(kfirst - 1);
        double fr[KK], fi[KK];
        auto load_f = [&](int64_t k, double (&r_)[KK], double (&i_)[KK]) {
            const double *Fr = F + k * 2 * (KW * KW), *Fi = Fr + KW * KW;
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                r_[kk] = Fr[(wv * KK + kk) * 64 + lane];
                i_[kk] = -Fi[(wv * KK + kk) * 64 + lane];          // U^H: conjugate
            }
        };
        load_f(kfirst, fr, fi);
        __syncthreads();
        int cur = 0;
        for (int64_t k = kfirst; k >= 0; --k) {
            const int64_t lo = j1 + k * R;
            double frn[KK], fin[KK];
            if (k > 0) load_f(k - 1, frn, fin);
            f64x4 ar = f64x4{0.0, 0.0, 0.0, 0.0}, ai = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const zd v = buf[cur][li * LT + 4 * kk + g];
                ar = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[kk], v.re, ar, 0, 0, 0);
                ar = __builtin_amdgcn_mfma_f64_16x16x4f64(-fi[kk], v.im, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[kk], v.im, ai, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f64_16x16x4f64(fi[kk], v.re, ai, 0, 0, 0);
            }
            const int f0 = (k == 0) ? 0 : (int)(q - 1);
            const int nxt = cur ^ 1;
            __syncthreads();                            // the previous window's stores have read ob
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 16 * wv + 4 * v + g;
                const zd z = mk<zd>(ar[v], ai[v]);
                if (c >= f0 && c < W) ob[li * LT + c] = z;
                if (k > 0 && c < q - 1) buf[nxt][li * LT + c + R] = z;   // index c + R of window k-1
            }
            if (k > 0) {
#pragma unroll
                for (int i = 0; i < 2; ++i) buf[nxt][(nc + 8 * i) * LT + nr] = pre[i];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = wc + 4 * i;
                const int64_t col = p0 + j, row = lo + wr;
                if (wr >= f0 && wr < W && col < n && row < n) X[row + col * ld] = ob[j * LT + wr];
            }
            if (k == 0) break;
            if (k > 1) load_new(k - 2);
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) { fr[kk] = frn[kk]; fi[kk] = fin[kk]; }
            cur = nxt;
        }
    }
    if (epi) {
        __syncthreads();                           // the tile's last window is in memory
        left_epilogue<zd>(a, J, p0, 16, tid, 256);
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(a.epi.flags + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace ht
