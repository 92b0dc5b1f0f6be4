// ht_stage2.hip -- stage two of the two-stage Hessenberg-triangular reduction
// (Steel & Vandebril, Section 3) on gfx950, and the C ABI declared in ht.h.
//
// Per group of q sweeps (Section 3.2):
//   1. copy the diagonal band of H and T that the generate phase touches into
//      a scratch band (the delayed updates later recompute every entry of H
//      and T from the pre-group values, so generation works on a copy);
//   2. generate phase (ht_generate.hpp): reflectors of the q sweeps;
//   3. application phase (ht_update.hpp): right updates of H, T, Z and Q,
//      then left updates of H and T.
// The Q and Z updates of a group run on an auxiliary stream, beside the next
// group's work on the caller's stream.  With lookahead (r in {4, 8, 16, 32})
// the left pass of group g and then group g's Q and Z updates run on a
// second stream, while group g+1's generation runs on the caller's stream,
// reading each tile of its scratch band once the left pass has written it.
// Every call joins its streams into the caller's stream before it returns.
#include "ht_common.hpp"
#include "ht_generate.hpp"
#include "ht_update.hpp"
#include "ht_update_reg.hpp"
#include "ht_update_mfma.hpp"
#include "ht_workspace.hpp"
#include "ht.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <map>
#include <mutex>
#include <vector>

namespace ht {

// ------------------------------------------------------- error reporting
thread_local char g_errmsg[256] = "";

int launch_check(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return 0;
    snprintf(g_errmsg, sizeof(g_errmsg), "%s: %s", what, hipGetErrorString(e));
    return HT_ERR_LAUNCH;
}

// ------------------------------------------------------------ profiling
// When enabled, every kernel launch of stage two is bracketed by HIP events
// recorded on the caller's stream; ht_profile_read() sums the elapsed times
// per kernel class.  Classes: 0 band copy, 1 generate, 2 right update of H
// and T, 3 left update, 4 exact zeros, 5 right update of Q and Z, 6 window
// factors.
constexpr int kProfClasses = 7;
struct ProfRec { int cls; hipEvent_t a, b; };
static std::mutex g_prof_mu;
static bool g_prof_on = false;
bool profiling_enabled() { std::lock_guard<std::mutex> lk(g_prof_mu); return g_prof_on; }
static std::vector<ProfRec> g_prof;

struct ProfScope {
    bool on = false;
    int cls = 0;
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int c, hipStream_t s) : cls(c), st(s) {       // c < 0: no timing
        if (c < 0) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        on = hipEventRecord(a, st) == hipSuccess;
    }
    ~ProfScope() {
        if (!on) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back({cls, a, b});
    }
};

// --------------------------------------------------------------- helpers
template <class S>
__global__ __launch_bounds__(256) void k_band_copy(const S *__restrict__ H, const S *__restrict__ T, int64_t ld,
                                                   S *SH, S *ST, Band B, int64_t n, int64_t c0,
                                                   int *progress, int nprog, int *flags, int nflags)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < nprog) progress[threadIdx.x] = 0;
    if (threadIdx.x == 0 && (int)blockIdx.x < nflags) flags[blockIdx.x] = 0;
    const int64_t c = c0 + blockIdx.x;
    if (c >= n) return;
    const int64_t ilo = i64max(0, c - B.BU), ihi = i64min(n - 1, c + B.BL);
    for (int64_t i = ilo + threadIdx.x; i <= ihi; i += blockDim.x) {
        SH[B.idx(i, c)] = H[i + c * ld];
        ST[B.idx(i, c)] = T[i + c * ld];
    }
}

// X(i, c) = 0 for i > c + off  (the exact zeros of the output contract, and the
// "not read" entries of the input contract)
template <class S>
__global__ __launch_bounds__(256) void k_zero_lower(S *X, int64_t ld, int64_t n, int64_t off)
{
    const int64_t c = blockIdx.x;
    for (int64_t i = c + off + 1 + threadIdx.x; i < n; i += blockDim.x) X[i + c * ld] = zero<S>();
}

// Exact zeros of the structure after the last sweep j2 of a group (the rule
// of CleanCol), rows c+1 .. c+depth of the columns c >= c0.
template <class S>
__global__ __launch_bounds__(256) void k_clean(S *H, S *T, int64_t ld, int64_t n, int64_t r, int64_t j2,
                                               int64_t c0, int64_t depth)
{
    const int64_t c = c0 + blockIdx.x;              // 0-based column
    if (c >= n) return;
    const CleanCol cc(c, r, n, j2);
    const int64_t rend = i64min(n, c + 1 + depth);   // 1-based last row examined
    for (int64_t i1b = c + 2 + threadIdx.x; i1b <= rend; i1b += blockDim.x) {
        if (!cc.keepT(i1b)) T[(i1b - 1) + c * ld] = zero<S>();
        if (!cc.keepH(i1b)) H[(i1b - 1) + c * ld] = zero<S>();
    }
}

// Progress counters of the generate phase to zero (when no band copy runs
// before it)
__global__ void k_zero_ints(int *p, int cnt)
{
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) p[i] = 0;
}

template <class S>
static int zero_lower(S *X, int64_t ld, int64_t n, int64_t off, hipStream_t st, bool prof = true)
{
    if (n <= 0 || !X) return 0;
    ProfScope ps(prof ? 4 : -1, st);
    hipLaunchKernelGGL(k_zero_lower<S>, dim3((unsigned)n), dim3(256), 0, st, X, ld, n, off);
    return launch_check("k_zero_lower");
}

inline int64_t default_q(int64_t n, int64_t r) { (void)n; return r; }

// A short pause on the left stream before each left pass of the lookahead
// schedule.  The left pass and the next group's generation become ready
// together (when the right pass ends); the generation's workgroups each need a
// whole compute unit (their register use allows one wavefront per SIMD), and
// the left pass's small workgroups, if dispatched first, would take every
// unit.  The pause lets the generation be dispatched first (measured at
// n = 16384, r = 32: 5.30 s a reduction with a pause of 10 us to 80 us,
// 5.61 s without).  Bounded by the device's constant-rate clock.
constexpr int kLaDelayUs = 10;
constexpr int64_t kLaMinN = 1024;              // automatic lookahead from this order on
__global__ void k_delay(int64_t ticks)
{
    if (threadIdx.x == 0) {
        const uint64_t t0 = wall_clock64();
        while (wall_clock64() - t0 < (uint64_t)ticks) __builtin_amdgcn_s_sleep(8);
    }
}

// Reflector buffers: the Q/Z updates of group g run on an auxiliary stream
// while the caller's stream goes on with group g+1, so consecutive groups use
// different buffers.
constexpr int kNBuf = 2;

// Auxiliary stream and events per (device, caller stream).
struct AuxCtx {
    hipStream_t aux = nullptr;
    hipEvent_t gen[kNBuf] = {}, qz[kNBuf] = {}, join = nullptr;
    // lookahead: the left pass of group g, then the Q and Z updates of group
    // g, run on `left` once the right pass (event rdone) is done; the caller's
    // stream waits for the left pass (ldone) before the right pass of group g+1
    hipStream_t left = nullptr;
    hipEvent_t rdone = nullptr, ldone = nullptr;
    int64_t delay_ticks = 0;      // kLaDelayUs in ticks of the device's constant-rate clock
    // lookahead calls in flight: one being enqueued (pending), or the end of
    // the last one enqueued on this stream (la_end, once recorded)
    hipEvent_t la_end = nullptr;
    bool la_pending = false, la_recorded = false;
    int dev = 0;
    bool ok = false;
};
static std::mutex g_aux_mu;
static std::map<std::pair<int, hipStream_t>, AuxCtx> g_aux;

static AuxCtx *aux_ctx(hipStream_t st)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_aux_mu);
    AuxCtx &c = g_aux[{dev, st}];
    if (c.ok) return &c;
    if (hipStreamCreateWithFlags(&c.aux, hipStreamNonBlocking) != hipSuccess) return nullptr;
    for (int b = 0; b < kNBuf; ++b) {
        if (hipEventCreateWithFlags(&c.gen[b], hipEventDisableTiming) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&c.qz[b], hipEventDisableTiming) != hipSuccess) return nullptr;
    }
    if (hipEventCreateWithFlags(&c.join, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (hipStreamCreateWithFlags(&c.left, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&c.rdone, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&c.ldone, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&c.la_end, hipEventDisableTiming) != hipSuccess) return nullptr;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    c.delay_ticks = (int64_t)khz * kLaDelayUs / 1000;
    c.dev = dev;
    c.ok = true;
    return &c;
}

// Lookahead makes the first sweep of a generation wait for the left pass of
// the same call, which runs on another stream; a generation workgroup takes a
// whole compute unit, so the generations of several calls running at once
// on one device could hold every unit while their left passes wait for one.
// A call therefore takes the lookahead schedule only while no other stream's
// lookahead call is in flight on the device (being enqueued, or its end
// event not yet reached); otherwise it runs its groups in sequence.  The
// claim ends when the call has enqueued its work (LaClaim's destructor).
struct LaClaim {
    AuxCtx *c = nullptr;
    ~LaClaim()
    {
        if (!c) return;
        std::lock_guard<std::mutex> lk(g_aux_mu);
        c->la_pending = false;
    }
};

static bool claim_lookahead(AuxCtx *self, LaClaim &cl)
{
    std::lock_guard<std::mutex> lk(g_aux_mu);
    bool busy = false;
    for (auto &kv : g_aux) {
        AuxCtx &o = kv.second;
        if (busy || &o == self || !o.ok || o.dev != self->dev) continue;
        busy = o.la_pending || (o.la_recorded && hipEventQuery(o.la_end) == hipErrorNotReady);
    }
    (void)hipGetLastError();                          // a query that returned not-ready leaves no error behind
    if (busy) return false;
    self->la_pending = true;
    cl.c = self;
    return true;
}

// Launch the application-phase kernels: register-ring variants for r in
// {4, 8, 16, 32} (complex: up to 16), the LDS-ring kernels otherwise.
template <class S>
static int launch_update(bool right, const UpdArgs<S> &ua, int64_t panels, hipStream_t st)
{
    const int64_t r = ua.r;
    const bool cplx = sizeof(S) > 8;
    const dim3 g((unsigned)panels), blk(64);
#define HT_REG_CASE(RR)                                                                               \
    case RR:                                                                                          \
        if (right) hipLaunchKernelGGL((k_update_right_reg<S, RR>), g, blk, 0, st, ua);               \
        else hipLaunchKernelGGL((k_update_left_reg<S, RR>), g, blk, 0, st, ua);                      \
        return launch_check(right ? "k_update_right_reg" : "k_update_left_reg");
    if (!(cplx && r > 16)) {
        switch (r) {
            HT_REG_CASE(4)
            HT_REG_CASE(8)
            HT_REG_CASE(16)
            HT_REG_CASE(32)
            default: break;
        }
    }
#undef HT_REG_CASE
    const size_t lds_right = (size_t)(2 * r) * 64 * sizeof(S);
    const size_t lds_left = lds_right + (size_t)64 * 65 * sizeof(S);
    if (right) hipLaunchKernelGGL(k_update_right<S>, g, blk, lds_right, st, ua);
    else hipLaunchKernelGGL(k_update_left<S>, g, blk, lds_left, st, ua);
    return launch_check(right ? "k_update_right" : "k_update_left");
}

// Matrix-core application kernels (real, r in {4, 8, 16, 32}).  Each job's
// npanels counts wavefront tiles of 16*TRW rows (right) / columns (left).
// coop: the H/T right pass of the lookahead schedule at r = 32, which has
// the device to itself (the Q/Z update runs after the left pass): one tile of
// 16 rows per workgroup, the window's product split over its four wavefronts
// (n = 8192: 209 ms to 121 ms per reduction, the same arithmetic, bitwise;
// n = 16384: 864 ms to 848 ms)
template <int R>
static int launch_update_mfma_r(bool left, UpdArgs<double> ua, const double *F, hipStream_t st, bool coop = false)
{
    if constexpr (R == 32) {
        if (!left && coop) {
            int64_t tot = 0;
            for (int i = 0; i < ua.njobs; ++i) { ua.job[i].npanels = (ua.n + 15) / 16; tot += ua.job[i].npanels; }
            hipLaunchKernelGGL((k_update_mfma_coop<R, false, 1>), dim3((unsigned)tot), dim3(256), 0, st, ua, F);
            return launch_check("k_update_mfma_coop(right)");
        }
        if (left) {
            // left updates at r = 32: one tile of 16 columns per workgroup, the window's product split
            // over its four wavefronts (measured: n = 8192 87 ms against 224 ms for one LDS-staged tile
            // per wavefront; n = 16384 1120 ms against 1463 ms for two direct tiles per wavefront)
            int64_t tot = 0;
            for (int i = 0; i < ua.njobs; ++i) { ua.job[i].npanels = (ua.n + 15) / 16; tot += ua.job[i].npanels; }
            hipLaunchKernelGGL((k_update_mfma_coop<R, true, 1>), dim3((unsigned)tot), dim3(256), 0, st, ua, F);
            return launch_check("k_update_mfma_coop(left)");
        }
    }
    const int64_t kt = knob(HT_KNOB_UPDATE_TILE_ROWS);
    const int trw = kt == 1 || kt == 2 ? (int)kt : (ua.n >= 8192 ? 2 : 1);
    const int64_t tile = 16 * trw;
    int64_t tot = 0;
    for (int i = 0; i < ua.njobs; ++i) { ua.job[i].npanels = (ua.n + tile - 1) / tile; tot += ua.job[i].npanels; }
    const dim3 grid((unsigned)((tot + 3) / 4)), blk(256);
    if (trw == 2) {
        if (left) hipLaunchKernelGGL((k_update_mfma<R, 2, true>), grid, blk, 0, st, ua, F);
        else hipLaunchKernelGGL((k_update_mfma<R, 2, false>), grid, blk, 0, st, ua, F);
    } else {
        if (left) hipLaunchKernelGGL((k_update_mfma<R, 1, true>), grid, blk, 0, st, ua, F);
        else hipLaunchKernelGGL((k_update_mfma<R, 1, false>), grid, blk, 0, st, ua, F);
    }
    return launch_check(left ? "k_update_mfma(left)" : "k_update_mfma(right)");
}

static int launch_update_mfma(bool left, const UpdArgs<double> &ua, const double *F, hipStream_t st, bool coop)
{
    switch (ua.r) {
    case 4: return launch_update_mfma_r<4>(left, ua, F, st);
    case 8: return launch_update_mfma_r<8>(left, ua, F, st);
    case 16: return launch_update_mfma_r<16>(left, ua, F, st);
    case 32: return launch_update_mfma_r<32>(left, ua, F, st, coop);
    default: return HT_ERR_NOTSUP;
    }
}

// Complex matrix-core application kernels (tiles of 16 rows / columns).
template <int R>
static int launch_update_mfma_z_r(bool left, UpdArgs<zd> ua, const double *F, hipStream_t st)
{
    int64_t tot = 0;
    for (int i = 0; i < ua.njobs; ++i) { ua.job[i].npanels = (ua.n + 15) / 16; tot += ua.job[i].npanels; }
    const dim3 grid((unsigned)((tot + 3) / 4)), blk(256);
    // left updates at r = 32: one column tile per workgroup, the window product split over its four
    // wavefronts (n = 8192: 613 ms against 800 ms for one LDS-staged tile per wavefront, 1.63 s for
    // direct loads); at r <= 16 the direct loads are faster (narrower tiles, more of them resident)
    if constexpr (R == 32) {
        if (left) {
            hipLaunchKernelGGL((k_update_mfma_z_coop_left<R>), dim3((unsigned)tot), blk, 0, st, ua, F);
            return launch_check("k_update_mfma_z_coop_left");
        }
    }
    if (left) hipLaunchKernelGGL((k_update_mfma_z<R, true>), grid, blk, 0, st, ua, F);
    else hipLaunchKernelGGL((k_update_mfma_z<R, false>), grid, blk, 0, st, ua, F);
    return launch_check(left ? "k_update_mfma_z(left)" : "k_update_mfma_z(right)");
}

static int launch_update_mfma_z(bool left, const UpdArgs<zd> &ua, const double *F, hipStream_t st)
{
    switch (ua.r) {
    case 4: return launch_update_mfma_z_r<4>(left, ua, F, st);
    case 8: return launch_update_mfma_z_r<8>(left, ua, F, st);
    case 16: return launch_update_mfma_z_r<16>(left, ua, F, st);
    case 32: return launch_update_mfma_z_r<32>(left, ua, F, st);
    default: return HT_ERR_NOTSUP;
    }
}

static int launch_form_factors_z(int64_t r, int64_t q, int64_t kmax, int64_t kext, const zd *VL, const zd *TL,
                                 const zd *VR, const zd *TR, double *F, hipStream_t st)
{
    const dim3 grid((unsigned)kmax, 2), blk(64);
    switch (r) {
    case 4: hipLaunchKernelGGL((k_form_factors_z<4, 16>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    case 8: hipLaunchKernelGGL((k_form_factors_z<8, 16>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    case 16: hipLaunchKernelGGL((k_form_factors_z<16, 32>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    case 32: hipLaunchKernelGGL((k_form_factors_z<32, 64>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    default: return HT_ERR_NOTSUP;
    }
    return launch_check("k_form_factors_z");
}

static int launch_form_factors(int64_t r, int64_t q, int64_t kmax, int64_t kext, const double *VL, const double *TL,
                               const double *VR, const double *TR, double *F, hipStream_t st)
{
    const dim3 grid((unsigned)kmax, 2), blk(64);
    switch (r) {
    case 4: hipLaunchKernelGGL((k_form_factors<4, 16>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    case 8: hipLaunchKernelGGL((k_form_factors<8, 16>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    case 16: hipLaunchKernelGGL((k_form_factors<16, 32>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    case 32: hipLaunchKernelGGL((k_form_factors<32, 64>), grid, blk, 0, st, q, kext, VL, TL, VR, TR, F); break;
    default: return HT_ERR_NOTSUP;
    }
    return launch_check("k_form_factors");
}

// dispatch of one update pass: matrix cores for r in {4, 8, 16, 32}, the
// vector kernels otherwise
template <class S>
static int launch_pass(bool right, const UpdArgs<S> &ua, int64_t panels, const S *F, hipStream_t st, bool coop = false)
{
    if constexpr (sizeof(S) == 8) {
        if (F) return launch_update_mfma(!right, ua, (const double *)F, st, coop);
    } else {
        if (F) return launch_update_mfma_z(!right, ua, (const double *)F, st);
    }
    return launch_update<S>(right, ua, panels, st);
}

struct Geometry {
    int64_t n, r, q, kext, BU, BL, ldb;
    size_t esz;
    size_t off_SH, off_ST, off_refl, refl_bytes, vbytes, tbytes, fbytes, tfbytes, off_prog, off_flags, total;
};

// The matrix-core application path: real and complex, r in {4, 8, 16, 32}.
static bool use_mfma(int64_t r, size_t) { return r == 4 || r == 8 || r == 16 || r == 32; }
static int64_t kw_of(int64_t r) { return 2 * r < 16 ? 16 : 2 * r; }

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static Geometry geometry(int64_t n, int64_t r, int64_t q, size_t esz, int nbuf = kNBuf)
{
    Geometry g{};
    g.n = n; g.r = r; g.q = q; g.esz = esz;
    g.kext = nblocks(n, r, 1) + 1;
    g.BU = (q + 1) * r;
    g.BL = 2 * r;
    g.ldb = g.BU + g.BL + 1;
    size_t o = 0;
    g.off_SH = o; o += al((size_t)n * g.ldb * esz);
    g.off_ST = o; o += al((size_t)n * g.ldb * esz);
    // per buffer: V_L, V_R, tau_L, tau_R and, on the matrix-core path, the
    // window factors of both sides
    g.vbytes = al((size_t)q * g.kext * r * esz);
    g.tbytes = al((size_t)q * g.kext * esz);
    g.fbytes = use_mfma(r, esz) ? al((size_t)2 * g.kext * kw_of(r) * kw_of(r) * esz) : 0;
    g.tfbytes = al((size_t)q * g.kext * kMaxR * esz);          // WY factors of the lazy left updates
    g.refl_bytes = g.vbytes * 2 + g.tbytes * 2 + g.fbytes + g.tfbytes;
    g.off_refl = o; o += g.refl_bytes * nbuf;
    g.off_prog = o; o += al((size_t)3 * q * sizeof(int));          // progress, far-row helpers' progress (H, T)
    g.off_flags = o; o += al((size_t)((n + 15) / 16) * sizeof(int));  // lookahead: tiles of the band ready
    g.total = o;
    return g;
}

// A caller-provided workspace for calls that must not allocate: `ws` holds
// `cap` bytes of device memory, `status` is the device status word.  Such a
// call runs every kernel on the caller's stream (no auxiliary stream, events
// or kernel timing) with one reflector buffer.
struct FixedWs {
    unsigned char *ws;
    size_t cap;
    int *status;
};

// Stage two, sweeps 1..jmax (jmax < 0 or >= n-2: all of them; the exact
// zeros of the final form are written only when all sweeps are done).
template <class S>
static int stage2_impl(S *H, S *T, S *Q, S *Z, int64_t n, int64_t r, int64_t ld, int64_t q, int64_t jmax,
                       void *stream, const FixedWs *fx = nullptr)
{
    if (n < 0) return -5;
    if (r < 1) return -6;
    if (ld < (n > 1 ? n : 1)) return -7;
    if (n > 0 && !H) return -1;
    if (n > 0 && !T) return -2;
    if (n == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    int rc;
    (void)hipGetLastError();           // clear a stale error left by earlier HIP calls
    g_errmsg[0] = 0;
    // every check that can fail comes before the first launch, so that a call
    // that returns an error has enqueued nothing
    const int64_t re_ = i64min(r, i64max(n - 1, 1));
    const bool trivial = n <= 2 || re_ <= 1;
    const int nbuf = fx ? 1 : kNBuf;
    Geometry g{};
    if (!trivial) {
        if (re_ > kMaxR) return HT_ERR_NOTSUP;
        if (q == 0) q = default_q(n, re_);
        if (q < 1 || q > re_) return -8;
        g = geometry(n, re_, q, sizeof(S), nbuf);
        if (fx && g.total > fx->cap) {
            snprintf(g_errmsg, sizeof(g_errmsg), "workspace of %zu bytes exceeds the fixed scratch of %zu bytes",
                     g.total, fx->cap);
            return HT_ERR_SCRATCH;
        }
    }
    // entries outside the r-HT pattern are not read: they are overwritten by 0
    if ((rc = zero_lower(H, ld, n, r, st, !fx)) || (rc = zero_lower(T, ld, n, 0, st, !fx))) return rc;
    if (trivial) {
        if ((rc = zero_lower(H, ld, n, 1, st, !fx))) return rc;
        return 0;
    }
    unsigned char *ws = nullptr;
    int *status = nullptr;
    if (fx) {
        ws = fx->ws;
        status = fx->status;
    } else {
        ws = (unsigned char *)workspace_get(g.total, st, &rc);
        if (!ws) return rc;
        StatusEntry *se = status_get(st);
        if (!se) { snprintf(g_errmsg, sizeof(g_errmsg), "status word allocation failed"); return HT_ERR_NOMEM; }
        status = se->dev;
    }
    const int64_t jlast = (jmax < 0 || jmax > n - 2) ? n - 2 : jmax;
    const int64_t wait_limit = knob(HT_KNOB_WAIT_POLLS);
    S *SH = (S *)(ws + g.off_SH), *ST = (S *)(ws + g.off_ST);
    int *prog = (int *)(ws + g.off_prog);
    const Band B{g.BU, g.BL, g.ldb};
    const int64_t rr = re_;
    const bool qz = (Q != nullptr) || (Z != nullptr);
    const bool mf = use_mfma(rr, sizeof(S));
    // lookahead: the left pass of group g (with the exact zeros and the next
    // group's band copy in its per-tile epilogue), then group g's Q and Z
    // updates, on a second stream; the generation of group g+1 waits for the
    // tiles of the band it reads
    // knob 1 (automatic): from n = 1024 on; for small pencils the pause and the
    // stream hand-offs of every group cost more than the overlap saves (a loop
    // of 2048 single calls with n up to 512: 30.2 s without, 32.6 s with)
    const int64_t la_knob = knob(HT_KNOB_LOOKAHEAD);
    const bool want_la = !fx && mf && (la_knob == 2 || (la_knob == 1 && n >= kLaMinN));
    const bool need_ctx = (qz && !fx) || want_la;
    AuxCtx *ax = need_ctx ? aux_ctx(st) : nullptr;
    if (need_ctx && !ax) { snprintf(g_errmsg, sizeof(g_errmsg), "auxiliary stream creation failed"); return HT_ERR_HIP; }
    LaClaim claim;
    const bool la = want_la && claim_lookahead(ax, claim);
    const bool aux = qz && !fx && !la;               // otherwise Q and Z on the auxiliary stream
    const bool prof = !fx;                           // kernel timing creates events: not for fixed scratch
    const int64_t np = (n + 63) / 64;
    int *flags = la ? (int *)(ws + g.off_flags) : nullptr;
    const int ntiles = (int)((n + 15) / 16);

    int64_t grp = 0;
    for (int64_t j1 = 1; j1 <= jlast; j1 += q, ++grp) {
        const int64_t j2 = i64min(j1 + q - 1, jlast);
        const int64_t qg = j2 - j1 + 1;
        const int64_t kmax = nblocks(n, rr, j1);
        const int64_t kext = kmax + 1;
        const int buf = (int)(grp % nbuf);
        unsigned char *rb = ws + g.off_refl + g.refl_bytes * buf;
        const size_t vbytes = g.vbytes, tbytes = g.tbytes;
        S *VL = (S *)rb, *VR = (S *)(rb + vbytes), *TL = (S *)(rb + 2 * vbytes), *TR = (S *)(rb + 2 * vbytes + tbytes);
        S *F = mf ? (S *)(rb + 2 * vbytes + 2 * tbytes) : nullptr;    // window factors
        S *TF = (S *)(rb + 2 * vbytes + 2 * tbytes + g.fbytes);        // WY factors of generation
        // the Q and Z updates of group grp - kNBuf must be done with this buffer
        if ((aux || (la && qz)) && grp >= kNBuf && hipStreamWaitEvent(st, ax->qz[buf], 0) != hipSuccess)
            return HT_ERR_HIP;
        // 1. scratch band (lookahead: from the second group on, written by the
        // previous group's left pass)
        if (!la || grp == 0) {
            ProfScope ps(prof ? 0 : -1, st);
            hipLaunchKernelGGL(k_band_copy<S>, dim3((unsigned)(n - (j1 - 1))), dim3(256), 0, st,
                               (const S *)H, (const S *)T, ld, SH, ST, B, n, j1 - 1, prog, (int)(3 * qg),
                               flags, la ? ntiles : 0);
            if ((rc = launch_check("k_band_copy"))) return rc;
        } else {
            hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(256), 0, st, prog, (int)(3 * qg));
            if ((rc = launch_check("k_zero_ints"))) return rc;
        }
        // 2. generate
        GenArgs<S> ga{};
        ga.n = n; ga.r = rr; ga.j1 = j1; ga.j2 = j2; ga.kext = kext; ga.band = B;
        ga.SH = SH; ga.ST = ST; ga.VL = VL; ga.TL = TL; ga.VR = VR; ga.TR = TR; ga.TF = TF; ga.progress = prog;
        ga.hdone = prog + qg;
        ga.status = status; ga.wait_limit = wait_limit;
        ga.flags = la && grp > 0 ? flags : nullptr;
        ga.flag_need = (int)(2 * grp);
        ga.ntiles = ntiles;
        { ProfScope ps(prof ? 1 : -1, st);
        if (rr <= 8) hipLaunchKernelGGL((k_generate<S, 8>), dim3((unsigned)(3 * qg)), dim3(256), 0, st, ga);
        else if (rr <= 16) hipLaunchKernelGGL((k_generate<S, 16>), dim3((unsigned)(3 * qg)), dim3(256), 0, st, ga);
        else hipLaunchKernelGGL((k_generate<S, 32>), dim3((unsigned)(3 * qg)), dim3(256), 0, st, ga);
        if ((rc = launch_check("k_generate"))) return rc; }
        if (mf) {
            ProfScope ps(prof ? 6 : -1, st);
            if constexpr (sizeof(S) == 8) {
                if ((rc = launch_form_factors(rr, qg, kmax, kext, VL, TL, VR, TR, F, st))) return rc;
            } else {
                if ((rc = launch_form_factors_z(rr, qg, kmax, kext, VL, TL, VR, TR, (double *)F, st))) return rc;
            }
        }
        UpdArgs<S> ua{};
        ua.n = n; ua.r = rr; ua.q = qg; ua.j1 = j1; ua.kmax = kmax; ua.kext = kext;
        ua.VL = VL; ua.TL = TL; ua.VR = VR; ua.TR = TR;
        int nj = 0;
        int64_t tot = 0;
        auto addjob = [&](S *X, int side, int64_t lim, int mat) {
            if (!X) return;
            ua.job[nj].X = X; ua.job[nj].ld = ld; ua.job[nj].lim = lim; ua.job[nj].npanels = np; ua.job[nj].side = side;
            ua.job[nj].mat = mat;
            ++nj; tot += np;
        };
        // 3a. Q and Z (right updates) on the auxiliary stream (fixed scratch:
        // on the caller's stream; lookahead: after the left pass, below)
        if (qz && !la) {
            hipStream_t qs = st;
            if (aux) {
                if (hipEventRecord(ax->gen[buf], st) != hipSuccess) return HT_ERR_HIP;
                if (hipStreamWaitEvent(ax->aux, ax->gen[buf], 0) != hipSuccess) return HT_ERR_HIP;
                qs = ax->aux;
            }
            addjob(Z, 1, -1, 2);
            addjob(Q, 0, -1, 2);
            ua.njobs = nj;
            { ProfScope ps(prof ? 5 : -1, qs);
            if ((rc = launch_pass<S>(true, ua, tot, F, qs))) return rc; }
            if (aux && hipEventRecord(ax->qz[buf], ax->aux) != hipSuccess) return HT_ERR_HIP;
        }
        // 3b. H and T: right updates, then left updates, then the exact zeros
        // (lookahead: the right pass waits for the previous group's left pass)
        if (la && grp > 0 && hipStreamWaitEvent(st, ax->ldone, 0) != hipSuccess) return HT_ERR_HIP;
        nj = 0; tot = 0;
        addjob(H, 1, (q + 2) * rr, 0);
        addjob(T, 1, (q + 1) * rr, 1);
        ua.njobs = nj;
        { ProfScope ps(prof ? 2 : -1, st);
        if ((rc = launch_pass<S>(true, ua, tot, F, st, la))) return rc; }
        nj = 0; tot = 0;
        addjob(H, 0, (q + 1) * rr, 0);
        addjob(T, 0, (q + 1) * rr, 1);
        ua.njobs = nj;
        const int64_t cc0 = i64max(0, j1 - 1 - (q + 2) * rr), depth = (q + 4) * rr;
        if (la) {
            if (hipEventRecord(ax->rdone, st) != hipSuccess) return HT_ERR_HIP;
            if (hipStreamWaitEvent(ax->left, ax->rdone, 0) != hipSuccess) return HT_ERR_HIP;
            hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, ax->left, ax->delay_ticks);
            if ((rc = launch_check("k_delay"))) return rc;
            LeftEpi<S> &e = ua.epi;
            e.SH = SH; e.ST = ST; e.band = B;
            e.c0 = j2 < jlast ? j2 : n;              // the next group's first column j2+1 (1-based)
            e.j2 = j2; e.cc0 = cc0; e.depth = depth; e.flags = flags;
            { ProfScope ps(prof ? 3 : -1, ax->left);
            if ((rc = launch_pass<S>(false, ua, tot, F, ax->left))) return rc; }
            if (hipEventRecord(ax->ldone, ax->left) != hipSuccess) return HT_ERR_HIP;
            if (qz) {
                ua.epi.flags = nullptr;
                nj = 0; tot = 0;
                addjob(Z, 1, -1, 2);
                addjob(Q, 0, -1, 2);
                ua.njobs = nj;
                { ProfScope ps(prof ? 5 : -1, ax->left);
                if ((rc = launch_pass<S>(true, ua, tot, F, ax->left))) return rc; }
                if (hipEventRecord(ax->qz[buf], ax->left) != hipSuccess) return HT_ERR_HIP;
            }
            continue;
        }
        { ProfScope ps(prof ? 3 : -1, st);
        if ((rc = launch_pass<S>(false, ua, tot, F, st))) return rc; }
        { ProfScope ps(prof ? 4 : -1, st);
        hipLaunchKernelGGL(k_clean<S>, dim3((unsigned)(n - cc0)), dim3(256), 0, st, H, T, ld, n, rr, j2, cc0, depth);
        if ((rc = launch_check("k_clean"))) return rc; }
    }
    if (la) {    // join the left stream; the call's end is what other streams' calls check
        if (hipEventRecord(ax->ldone, ax->left) != hipSuccess) return HT_ERR_HIP;
        if (hipStreamWaitEvent(st, ax->ldone, 0) != hipSuccess) return HT_ERR_HIP;
        if (hipEventRecord(ax->la_end, st) != hipSuccess) return HT_ERR_HIP;
        std::lock_guard<std::mutex> lk(g_aux_mu);
        ax->la_recorded = true;
    }
    if (aux) {   // join the auxiliary stream
        if (hipEventRecord(ax->join, ax->aux) != hipSuccess) return HT_ERR_HIP;
        if (hipStreamWaitEvent(st, ax->join, 0) != hipSuccess) return HT_ERR_HIP;
    }
    if (jlast == n - 2 && ((rc = zero_lower(H, ld, n, 1, st, prof)) || (rc = zero_lower(T, ld, n, 0, st, prof))))
        return rc;
    return 0;
}

// ------------------------------------------------ fixed scratch (no allocation)
// ht_stage2_noalloc takes its workspace from this array instead of the
// per-stream cache.  Each device that runs the library holds its own copy
// until the process ends.  Host code must not pass the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address of each copy is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.  The first 256 bytes hold a
// status word for calls that pass no status pointer of their own.
constexpr size_t kScratchBytes = size_t(HT_NOALLOC_SCRATCH_BYTES);
constexpr size_t kScratchStatus = 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first call
// on that device), or nullptr with *rc set.
static unsigned char *scratch_of_current_device(int *rc)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { *rc = HT_ERR_HIP; return nullptr; }
    if (dev < 0 || dev >= kMaxDevices) { *rc = HT_ERR_NOTSUP; return nullptr; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            snprintf(g_errmsg, sizeof(g_errmsg), "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            *rc = HT_ERR_HIP;
            return nullptr;
        }
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    return g_scratch_ptr[dev];
}

// Device status word of the stream -> pinned host int, and cleared.
__global__ void k_status_take(int *dev, int *host)
{
    if (threadIdx.x == 0) { *host = *dev; *dev = 0; }
}

}  // namespace ht

// =================================================================== C ABI
extern "C" {

int ht_stage2(double *H, double *T, double *Q, double *Z, int64_t n, int64_t r, int64_t ld, void *stream)
{
    return ht::stage2_impl<double>(H, T, Q, Z, n, r, ld, 0, -1, stream);
}

int ht_stage2_q(double *H, double *T, double *Q, double *Z, int64_t n, int64_t r, int64_t ld, int64_t q,
                void *stream)
{
    return ht::stage2_impl<double>(H, T, Q, Z, n, r, ld, q, -1, stream);
}

int ht_stage2_noalloc(double *H, double *T, double *Q, double *Z, int64_t n, int64_t r, int64_t ld, int *status,
                      void *stream)
{
    // argument checks first (they need no device)
    if (n < 0) return -5;
    if (r < 1) return -6;
    if (ld < (n > 1 ? n : 1)) return -7;
    if (n > 0 && !H) return -1;
    if (n > 0 && !T) return -2;
    int rc = 0;
    unsigned char *base = ht::scratch_of_current_device(&rc);
    if (!base) return rc;
    ht::FixedWs fx;
    fx.ws = base + ht::kScratchStatus;
    fx.cap = ht::kScratchBytes - ht::kScratchStatus;
    fx.status = status ? status : (int *)base;
    return ht::stage2_impl<double>(H, T, Q, Z, n, r, ld, 0, -1, stream, &fx);
}

int ht_stage2_sweeps(double *H, double *T, double *Q, double *Z, int64_t n, int64_t r, int64_t ld, int64_t q,
                     int64_t jmax, void *stream)
{
    return ht::stage2_impl<double>(H, T, Q, Z, n, r, ld, q, jmax, stream);
}

int ht_stage2_z_sweeps(void *H, void *T, void *Q, void *Z, int64_t n, int64_t r, int64_t ld, int64_t q,
                       int64_t jmax, void *stream)
{
    return ht::stage2_impl<ht::zd>((ht::zd *)H, (ht::zd *)T, (ht::zd *)Q, (ht::zd *)Z, n, r, ld, q, jmax, stream);
}

int ht_stage2_z(void *H, void *T, void *Q, void *Z, int64_t n, int64_t r, int64_t ld, void *stream)
{
    return ht::stage2_impl<ht::zd>((ht::zd *)H, (ht::zd *)T, (ht::zd *)Q, (ht::zd *)Z, n, r, ld, 0, -1, stream);
}

int ht_stage2_z_q(void *H, void *T, void *Q, void *Z, int64_t n, int64_t r, int64_t ld, int64_t q, void *stream)
{
    return ht::stage2_impl<ht::zd>((ht::zd *)H, (ht::zd *)T, (ht::zd *)Q, (ht::zd *)Z, n, r, ld, q, -1, stream);
}

int64_t ht_workspace_bytes(int64_t n, int64_t r, int64_t q, int is_complex)
{
    if (n < 0 || r < 1 || q < 0) return -1;
    if (n <= 2) return 0;
    const int64_t re_ = ht::i64min(r, n - 1);
    if (re_ <= 1) return 0;
    if (q == 0) q = ht::default_q(n, re_);
    if (q > re_) return -1;
    return (int64_t)ht::geometry(n, re_, q, is_complex ? 16 : 8).total;
}

int ht_reserve_workspace(int64_t bytes, void *stream)
{
    if (bytes < 0) return -1;
    return ht::workspace_reserve((size_t)bytes, (hipStream_t)stream);
}

int64_t ht_default_q(int64_t n, int64_t r)
{
    if (n <= 2 || r <= 1) return 1;
    return ht::default_q(n, ht::i64min(r, n - 1));
}

const char *ht_strerror(int code)
{
    if (code == 0) return "success";
    if (code < 0) return "invalid argument";
    switch (code) {
    case HT_ERR_HIP: return "HIP runtime error";
    case HT_ERR_NOMEM: return "device workspace allocation failed";
    case HT_ERR_LAUNCH: return "kernel launch failed";
    case HT_ERR_NOTSUP: return "configuration not supported (r > 32 on the GPU path)";
    case HT_ERR_TIMEOUT: return "a bounded device-side wait gave up: the output of a call on this stream is invalid";
    case HT_ERR_SCRATCH: return "the call needs more workspace than the fixed no-allocation scratch holds";
    default: return "unknown error";
    }
}

const char *ht_version(void) { return "libht 0.2 (gfx950)"; }

int ht_stream_status(void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    ht::StatusEntry *se = ht::status_get(st);
    if (!se) return HT_ERR_NOMEM;
    hipLaunchKernelGGL(ht::k_status_take, dim3(1), dim3(64), 0, st, se->dev, se->host);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return HT_ERR_HIP;
    const int v = *(volatile int *)se->host;
    return (v & ht::kStatusWaitTimeout) ? HT_ERR_TIMEOUT : 0;
}

int ht_set_knob(int knob, int64_t value)
{
    if (knob < 1 || knob > ht::kNumKnobs) return -1;
    switch (knob) {
    case HT_KNOB_WAIT_POLLS: if (value < 0) return -2; break;
    case HT_KNOB_UPDATE_TILE_ROWS: if (value < 0 || value > 2) return -2; break;
    case HT_KNOB_LOOKAHEAD: if (value < 0 || value > 2) return -2; break;
    default: break;
    }
    ht::knobs()[knob - 1].store(value, std::memory_order_relaxed);
    return 0;
}

int64_t ht_get_knob(int knob)
{
    if (knob < 1 || knob > ht::kNumKnobs) return -1;
    return ht::knob(knob);
}

const char *ht_last_error_message(void) { return ht::g_errmsg; }

int ht_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(ht::g_prof_mu);
    ht::g_prof_on = on != 0;
    return 0;
}

int ht_profile_read(double *ms, int64_t *count, int nclasses)
{
    std::vector<ht::ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(ht::g_prof_mu);
        recs.swap(ht::g_prof);
    }
    for (int c = 0; c < nclasses; ++c) { if (ms) ms[c] = 0.0; if (count) count[c] = 0; }
    int rc = 0;
    for (auto &p : recs) {
        float t = 0.f;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&t, p.a, p.b) != hipSuccess) rc = HT_ERR_HIP;
        if (p.cls < nclasses) { if (ms) ms[p.cls] += t; if (count) count[p.cls] += 1; }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    return rc;
}

}  // extern "C"

extern "C" void ht_release_workspace(void) { ht::workspace_release_all_current_device(); }
