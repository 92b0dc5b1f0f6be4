// ht_batched.hip -- batched stage two: many independent r-HT pencils of
// uneven n and r reduced to Hessenberg-triangular form in ONE persistent
// launch (the C ABI ht_stage2_batched / ht_stage2_batched_z).
//
// Small pencils (the batched workloads have n of a few hundred) are bound by
// the latency of the ~n^2/(2r) dependent steps of the sweep chase, not by
// flops, so a launch per group and phase (the blocked single-pencil path) is
// the wrong shape for them.  Here the workgroups of one launch pull whole
// pencils from two device-side queues (vector atomics on counters) and run
// the unblocked stage-two algorithm of the appendix on each (Section 3.1),
// every reflector applied at once to its full range, so the results agree
// with ht_stage2 up to rounding.  A pencil is reduced either by a whole
// workgroup of 256 threads (larger n: more rows and columns per reflector)
// or by a single wavefront, four pencils per workgroup at a time (small n:
// the wavefront needs no barrier between the phases of a step); the choice
// per (n, r) comes from a tuning table (ht_batched_set_tuning, filled by the
// autotuner).  Each queue is ordered longest first, so that the pencils that
// take longest start first.
#include "ht_common.hpp"
#include "ht_generate.hpp"
#include "ht_workspace.hpp"
#include "ht.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <mutex>
#include <vector>
#include <string.h>
#include <stdio.h>

namespace ht {

extern thread_local char g_errmsg[256];
int launch_check(const char *what);
bool profiling_enabled();

// per-pencil start/finish stamps of the last batched call made with kernel
// timing enabled (device wall clock), per calling thread
struct BatchStamps { unsigned long long *dev = nullptr; int64_t count = 0; hipStream_t st = nullptr; };
static thread_local BatchStamps g_stamps;

template <class S>
struct Pencil {
    S *H, *T, *Q, *Z;
    int64_t n, r, ld;
};

constexpr int kBatThreads = 256;

__global__ void k_reset_counters(int *c) { if (threadIdx.x < 2 && blockIdx.x == 0) c[threadIdx.x] = 0; }

// Synchronisation of the NT threads that reduce one pencil: the workgroup
// (NT = 256: a barrier, which also completes the waves' memory operations)
// or one wavefront (NT = 64: its lanes run in lockstep, so completing the
// wavefront's own memory operations before the next phase reads them is
// enough).
template <int NT>
__device__ __forceinline__ void pencil_sync()
{
    if constexpr (NT == kBatThreads) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// X(rows a..a+m-1, cols c0..c1) <- G^H X, one column per thread
template <class S, int NT>
__device__ inline void left_cols(S *X, int64_t ld, int64_t a, int m, int64_t c0, int64_t c1,
                                 const S *v, S tau, int tid)
{
    const S ct = conj_(tau);
    for (int64_t c = c0 + tid; c <= c1; c += NT) {
        S *col = X + a + c * ld;
        S s0 = zero<S>(), s1 = zero<S>();
        int i = 0;
        for (; i + 1 < m; i += 2) { s0 = add(s0, cmul(v[i], col[i])); s1 = add(s1, cmul(v[i + 1], col[i + 1])); }
        if (i < m) s0 = add(s0, cmul(v[i], col[i]));
        const S s = mul(ct, add(s0, s1));
        for (int ii = 0; ii < m; ++ii) col[ii] = sub(col[ii], mul(s, v[ii]));
    }
}

// X(rows r0..r1, cols a..a+m-1) <- X G, one row per thread; with zfirst the
// entry of column a is written as an exact zero for rows > a
template <class S, int NT>
__device__ inline void right_rows_b(S *X, int64_t ld, int64_t a, int m, int64_t r0, int64_t r1,
                                    const S *v, S tau, int tid, bool zfirst)
{
    for (int64_t row = r0 + tid; row <= r1; row += NT) {
        S *p = X + row + a * ld;
        S s0 = zero<S>(), s1 = zero<S>();
        int c = 0;
        for (; c + 1 < m; c += 2) { s0 = add(s0, mul(p[c * ld], v[c])); s1 = add(s1, mul(p[(c + 1) * ld], v[c + 1])); }
        if (c < m) s0 = add(s0, mul(p[c * ld], v[c]));
        const S s = mul(add(s0, s1), tau);
        for (int cc = 0; cc < m; ++cc)
            p[cc * ld] = (zfirst && cc == 0 && row > a) ? zero<S>() : sub(p[cc * ld], mul(s, conj_(v[cc])));
    }
}

// The unblocked stage-two algorithm of the appendix (Section 3.1) on one
// pencil, by NT threads (tid = 0..NT-1; the first 64 of them form the
// wavefront that generates the reflectors): for every sweep j and block k,
//   left reflector from H(i1:i2, jb) (xLARFG),
//   G^H applied to rows i1..i2 of H (columns jb+1..n) and T (columns i1..n),
//   Q <- Q G on columns i1..i2,
//   RQ of the updated T block in registers, opposite reflector,
//   W applied to columns i1..i2 of H (rows 1..i3), T (rows 1..i2) and Z (all
//   rows); T(i1+1:i2, i1) <- 0 exactly.
// sv, sw: 64 entries of LDS each, stau: 2.
template <class S, int RM, int NT>
__device__ void reduce_pencil(const Pencil<S> &P, int tid, S *sv, S *sw, S *stau)
{
    const int lane = tid & 63;
    const bool gen = tid < 64;                     // the generating wavefront
    const int64_t n = P.n, ld = P.ld;
    S *H = P.H, *T = P.T, *Q = P.Q, *Z = P.Z;
    const int64_t r = i64min(P.r, i64max(n - 1, 1));
    // entries outside the r-HT pattern are not read: they become exact zeros
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + r + 1 + tid; i < n; i += NT) H[i + c * ld] = zero<S>();
        for (int64_t i = c + 1 + tid; i < n; i += NT) T[i + c * ld] = zero<S>();
    }
    pencil_sync<NT>();
    if (n > 2 && r > 1) {
        for (int64_t j = 1; j <= n - 2; ++j) {
            const int64_t nbj = nblocks(n, r, j);
            for (int64_t k = 0; k < nbj; ++k) {
                const int64_t jb = j + i64max(0, (k - 1) * r + 1);
                const int64_t i1 = j + k * r + 1;
                const int64_t i2 = i64min(j + (k + 1) * r, n);
                const int64_t i3 = i64min(j + (k + 2) * r, n);
                const int m = (int)(i2 - i1 + 1);
                const int64_t a = i1 - 1, cb = jb - 1;
                // left reflector
                if (gen) {
                    const S x = lane < m ? H[a + lane + cb * ld] : zero<S>();
                    S v, tau, beta;
                    wave_larfg(x, lane, m, v, tau, beta);
                    sv[lane] = lane < m ? v : zero<S>();
                    if (lane == 0) { stau[0] = tau; H[a + cb * ld] = beta; }
                    else if (lane < m) H[a + lane + cb * ld] = zero<S>();
                }
                pencil_sync<NT>();
                {
                    const S tau = stau[0];
                    if (!iszero(tau)) {
                        left_cols<S, NT>(H, ld, a, m, cb + 1, n - 1, sv, tau, tid);
                        left_cols<S, NT>(T, ld, a, m, a, n - 1, sv, tau, tid);
                        if (Q) right_rows_b<S, NT>(Q, ld, a, m, 0, n - 1, sv, tau, tid, false);
                    }
                }
                pencil_sync<NT>();
                // RQ of the T block and the opposite reflector
                if (gen) {
                    S x[RM];
#pragma unroll
                    for (int c = 0; c < RM; ++c) {
                        S v = zero<S>();
                        if (lane < m && c < m) v = T[a + lane + (a + c) * ld];
                        if (lane == 32 + c && c < m) v = one<S>();
                        x[c] = v;
                    }
                    rq_rows<S, RM>(x, m);
                    S y = shfl_(x[0], 32 + (lane & 31));
                    if (lane >= m) y = zero<S>();
                    const unsigned long long mask = __ballot(lane < m && !iszero(y));
                    const int p = mask ? (__ffsll((long long)mask) - 1) : 0;
                    const S yp = bcast(y, p);
                    if (!iszero(yp)) {
                        const double ra = 1.0 / sqrt(abs2(yp));
                        if (im(yp) == 0.0) {
                            if (re(yp) < 0.0) y = mk<S>(-re(y), -im(y));
                        } else {
                            const S ph = mk<S>(re(yp) * ra, -im(yp) * ra);
                            y = mul(y, ph);
                            if (lane == p) y = mk<S>(re(y), 0.0);
                        }
                    }
                    S v, tau, beta;
                    wave_larfg(y, lane, m, v, tau, beta);
                    sw[lane] = lane < m ? v : zero<S>();
                    if (lane == 0) stau[1] = tau;
                }
                pencil_sync<NT>();
                {
                    const S sig = stau[1];
                    if (!iszero(sig)) {
                        right_rows_b<S, NT>(H, ld, a, m, 0, i3 - 1, sw, sig, tid, false);
                        right_rows_b<S, NT>(T, ld, a, m, 0, i2 - 1, sw, sig, tid, true);
                        if (Z) right_rows_b<S, NT>(Z, ld, a, m, 0, n - 1, sw, sig, tid, false);
                    } else {
                        for (int64_t i = a + 1 + tid; i < a + m; i += NT) T[i + a * ld] = zero<S>();
                    }
                }
                pencil_sync<NT>();
            }
        }
    }
    // exact zeros of the output contract
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c + 2 + tid; i < n; i += NT) H[i + c * ld] = zero<S>();
        for (int64_t i = c + 1 + tid; i < n; i += NT) T[i + c * ld] = zero<S>();
    }
    pencil_sync<NT>();
}

// One persistent launch over two queues of pencils (indices into `pen`,
// each in decreasing order of work): the workgroup queue (a pencil per
// workgroup of 256 threads), drained first, then the wavefront queue, from
// which each of a workgroup's four wavefronts takes pencils on its own.
// Positions are taken with vector atomics on counters[0] / counters[1].
template <class S, int RM>
__global__ __launch_bounds__(kBatThreads) void k_stage2_persistent(const Pencil<S> *pen, const int *order, int ngroup,
                                                                   int nwave, int *counters,
                                                                   unsigned long long *stamps)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ S sv[4][64], sw[4][64];
    __shared__ S stau[4][2];
    __shared__ int s_idx;
    for (;;) {
        if (tid == 0) s_idx = __hip_atomic_fetch_add(counters, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int i = s_idx;
        __syncthreads();
        if (i >= ngroup) break;
        const int b = order[i];
        if (stamps && tid == 0) stamps[2 * b] = wall_clock64();
        reduce_pencil<S, RM, kBatThreads>(pen[b], tid, sv[0], sw[0], stau[0]);
        if (stamps && tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            stamps[2 * b + 1] = wall_clock64();
        }
    }
    for (;;) {
        int i = 0;
        if (lane == 0) i = __hip_atomic_fetch_add(counters + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        i = __shfl(i, 0, 64);
        if (i >= nwave) break;
        const int b = order[ngroup + i];
        if (stamps && lane == 0) stamps[2 * b] = wall_clock64();
        reduce_pencil<S, RM, 64>(pen[b], lane, sv[wid], sw[wid], stau[wid]);
        if (stamps && lane == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            stamps[2 * b + 1] = wall_clock64();
        }
    }
}

// ------------------------------------------------------------ tuning table
// Which pencils a batched call reduces with one wavefront instead of a
// workgroup of 256 threads: the first entry with n <= n_max and r == r_e
// decides (r_e = 0 matches any r); without a match, pencils with
// n <= kDefaultWaveN take a wavefront.
struct BatTune { int64_t n_max, r, threads; };
static std::mutex g_tune_mu;
static std::vector<BatTune> g_tune;
constexpr int64_t kDefaultWaveN = 128;

static int threads_for(int64_t n, int64_t r)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const BatTune &t : g_tune)
        if (n <= t.n_max && (t.r == 0 || t.r == r)) return (int)t.threads;
    return n <= kDefaultWaveN ? 64 : kBatThreads;
}

template <class S>
static int batched_impl(int64_t count, S *const *H, S *const *T, S *const *Q, S *const *Z, const int64_t *n,
                        const int64_t *r, const int64_t *ld, const int64_t *q, void *stream)
{
    if (count < 0) return -1;
    if (count > 0 && !H) return -2;
    if (count > 0 && !T) return -3;
    if (count > 0 && !Q) return -4;
    if (count > 0 && !Z) return -5;
    if (count > 0 && !n) return -6;
    if (count > 0 && !r) return -7;
    if (count > 0 && !ld) return -8;
    if (count == 0) return 0;
    if (count > (int64_t)(1 << 30)) return -1;
    std::vector<Pencil<S>> hp((size_t)count);
    int64_t rmax = 1;
    for (int64_t b = 0; b < count; ++b) {
        if (n[b] < 0) return -6;
        if (r[b] < 1) return -7;
        if (ld[b] < (n[b] > 1 ? n[b] : 1)) return -8;
        if (n[b] > 0 && (!H[b] || !T[b])) return -2;
        if (q && (q[b] < 0 || (n[b] > 2 && q[b] > i64min(r[b], n[b] - 1)))) return -9;
        hp[b] = Pencil<S>{H[b], T[b], Q[b], Z[b], n[b], r[b], ld[b]};
        if (n[b] > 2) rmax = i64max(rmax, i64min(r[b], n[b] - 1));
    }
    if (rmax > kMaxR) return HT_ERR_NOTSUP;
    // the two queues, each longest first (the chase of a pencil takes about
    // n^2 / (2r) dependent steps of about n work each)
    std::vector<int> grp, wav;
    for (int64_t b = 0; b < count; ++b) {
        const int64_t rr = i64min(r[b], i64max(n[b] - 1, 1));
        (threads_for(n[b], rr) == 64 ? wav : grp).push_back((int)b);
    }
    auto work = [&](int b) { return (double)n[b] * (double)n[b] * (double)n[b] / (double)i64max(1, r[b]); };
    auto longest_first = [&](int x, int y) { return work(x) > work(y); };
    std::stable_sort(grp.begin(), grp.end(), longest_first);
    std::stable_sort(wav.begin(), wav.end(), longest_first);
    std::vector<int> order(grp);
    order.insert(order.end(), wav.begin(), wav.end());

    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    g_errmsg[0] = 0;
    int rc = 0;
    const size_t dbytes = (size_t)count * sizeof(Pencil<S>);
    const size_t obytes = (size_t)count * sizeof(int);
    const size_t dal = (dbytes + 255) & ~(size_t)255, oal = (obytes + 255) & ~(size_t)255;
    const bool timed = profiling_enabled();
    const size_t sbytes = timed ? (size_t)count * 2 * sizeof(unsigned long long) : 0;
    unsigned char *ws = (unsigned char *)workspace_get(dal + oal + 256 + sbytes, st, &rc);
    if (!ws) return rc;
    Pencil<S> *dp = (Pencil<S> *)ws;
    int *dorder = (int *)(ws + dal);
    int *counters = (int *)(ws + dal + oal);            // positions in the two queues
    unsigned long long *stamps = timed ? (unsigned long long *)(ws + dal + oal + 256) : nullptr;
    g_stamps = BatchStamps{stamps, timed ? count : 0, st};
    // the descriptors and the order go through this stream's pinned staging
    // buffer, so the call does not wait for the stream; the host arrays are
    // read before return
    PinnedEntry *pe = pinned_get(dal + obytes, st);
    if (!pe) { snprintf(g_errmsg, sizeof(g_errmsg), "pinned staging buffer"); return HT_ERR_HIP; }
    memcpy(pe->ptr, hp.data(), dbytes);
    memcpy((unsigned char *)pe->ptr + dal, order.data(), obytes);
    if (hipMemcpyAsync(ws, pe->ptr, dal + obytes, hipMemcpyHostToDevice, st) != hipSuccess) return HT_ERR_HIP;
    if (hipEventRecord(pe->done, st) != hipSuccess) return HT_ERR_HIP;
    pe->pending = true;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, st, counters);
    if ((rc = launch_check("k_reset_counters"))) return rc;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) ncu = pr.multiProcessorCount;
    }
    const int64_t need = (int64_t)grp.size() + ((int64_t)wav.size() + 3) / 4;
    const int64_t wgs = i64max(1, i64min(need, (int64_t)ncu * (rmax <= 16 ? 2 : 1)));
    const dim3 grid((unsigned)wgs), blk(kBatThreads);
    const int ng = (int)grp.size(), nw = (int)wav.size();
    if (rmax <= 16)
        hipLaunchKernelGGL((k_stage2_persistent<S, 16>), grid, blk, 0, st, dp, dorder, ng, nw, counters, stamps);
    else
        hipLaunchKernelGGL((k_stage2_persistent<S, 32>), grid, blk, 0, st, dp, dorder, ng, nw, counters, stamps);
    return launch_check("k_stage2_persistent");
}

}  // namespace ht

extern "C" {
int ht_batched_set_tuning(int64_t entries, const int64_t *n_max, const int64_t *r, const int64_t *threads)
{
    if (entries < 0) return -1;
    if (entries > 0 && (!n_max || !r || !threads)) return -2;
    std::vector<ht::BatTune> t((size_t)entries);
    for (int64_t e = 0; e < entries; ++e) {
        if (threads[e] != 64 && threads[e] != ht::kBatThreads) return -4;
        if (r[e] < 0) return -3;
        t[(size_t)e] = ht::BatTune{n_max[e], r[e], threads[e]};
    }
    std::lock_guard<std::mutex> lk(ht::g_tune_mu);
    ht::g_tune.swap(t);
    return 0;
}

int ht_stage2_batched(int64_t count, double *const *H, double *const *T, double *const *Q, double *const *Z,
                      const int64_t *n, const int64_t *r, const int64_t *ld, const int64_t *q, void *stream)
{
    return ht::batched_impl<double>(count, H, T, Q, Z, n, r, ld, q, stream);
}
int ht_batched_completion_ms(double *ms, int64_t count)
{
    const ht::BatchStamps b = ht::g_stamps;
    if (!ms || count != b.count || !b.dev) return -1;
    if (count == 0) return 0;
    std::vector<unsigned long long> h((size_t)count * 2);
    if (hipStreamSynchronize(b.st) != hipSuccess) return HT_ERR_HIP;
    if (hipMemcpy(h.data(), b.dev, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
        return HT_ERR_HIP;
    int dev = 0, rate_khz = 100000;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    unsigned long long t0 = h[0];
    for (int64_t i = 0; i < count; ++i) t0 = h[2 * i] < t0 ? h[2 * i] : t0;
    for (int64_t i = 0; i < count; ++i) ms[i] = (double)(h[2 * i + 1] - t0) / (double)rate_khz;
    return 0;
}
int ht_stage2_batched_z(int64_t count, void *const *H, void *const *T, void *const *Q, void *const *Z,
                        const int64_t *n, const int64_t *r, const int64_t *ld, const int64_t *q, void *stream)
{
    return ht::batched_impl<ht::zd>(count, (ht::zd *const *)H, (ht::zd *const *)T, (ht::zd *const *)Q,
                                    (ht::zd *const *)Z, n, r, ld, q, stream);
}
}
