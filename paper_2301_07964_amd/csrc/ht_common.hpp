// ht_common.hpp -- scalar helpers, index map and launch geometry shared by the
// HIP kernels of libht (gfx950 only).
//
// Index notation follows the paper (Steel & Vandebril, Section 3 and the
// stage-two algorithms of the appendix): sweeps j and matrix rows/columns are
// 1-based in the index formulas, converted to 0-based only at memory access.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ht {

// ------------------------------------------------------------------ scalars
struct zd { double re, im; };

// branch-free choice, component-wise for complex values
__host__ __device__ inline double sel(bool c, double a, double b) { return c ? a : b; }
__host__ __device__ inline zd sel(bool c, zd a, zd b) { zd z; z.re = c ? a.re : b.re; z.im = c ? a.im : b.im; return z; }

__host__ __device__ inline double re(double a) { return a; }
__host__ __device__ inline double re(zd a) { return a.re; }
__host__ __device__ inline double im(double) { return 0.0; }
__host__ __device__ inline double im(zd a) { return a.im; }
template <class S> __host__ __device__ inline S mk(double r, double i);
template <> __host__ __device__ inline double mk<double>(double r, double) { return r; }
template <> __host__ __device__ inline zd mk<zd>(double r, double i) { zd z; z.re = r; z.im = i; return z; }
template <class S> __host__ __device__ inline S zero() { return mk<S>(0.0, 0.0); }
template <class S> __host__ __device__ inline S one() { return mk<S>(1.0, 0.0); }

__host__ __device__ inline double conj_(double a) { return a; }
__host__ __device__ inline zd conj_(zd a) { return mk<zd>(a.re, -a.im); }
__host__ __device__ inline double add(double a, double b) { return a + b; }
__host__ __device__ inline zd add(zd a, zd b) { return mk<zd>(a.re + b.re, a.im + b.im); }
__host__ __device__ inline double sub(double a, double b) { return a - b; }
__host__ __device__ inline zd sub(zd a, zd b) { return mk<zd>(a.re - b.re, a.im - b.im); }
__host__ __device__ inline double mul(double a, double b) { return a * b; }
__host__ __device__ inline zd mul(zd a, zd b) { return mk<zd>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
// conj(a) * b
__host__ __device__ inline double cmul(double a, double b) { return a * b; }
__host__ __device__ inline zd cmul(zd a, zd b) { return mk<zd>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re); }
__host__ __device__ inline double scal(double a, double s) { return a * s; }
__host__ __device__ inline zd scal(zd a, double s) { return mk<zd>(a.re * s, a.im * s); }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline double abs2(zd a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline bool iszero(double a) { return a == 0.0; }
__host__ __device__ inline bool iszero(zd a) { return a.re == 0.0 && a.im == 0.0; }
// 1 / (c + i d), Smith's method
__host__ __device__ inline double recip(double a) { return 1.0 / a; }
__host__ __device__ inline zd recip(zd z) {
    double c = z.re, d = z.im;
    if (fabs(c) >= fabs(d)) { double e = d / c, f = c + d * e; return mk<zd>(1.0 / f, -e / f); }
    double e = c / d, f = d + c * e; return mk<zd>(e / f, -1.0 / f);
}

// Square root and reciprocal of positive normal doubles with a short chain of
// dependent operations (the reflector scalars sit on the critical path of
// the generate phase): the hardware estimates refined by Newton's method --
// for the square root Goldschmidt's coupled iteration on g ~ sqrt(s),
// h ~ 1/(2 sqrt(s)), two steps and a final residual correction; for the
// reciprocal two Newton-Raphson steps y <- y + y (1 - d y).  Accurate to about
// an ulp, not correctly rounded; the inputs here are O(1) (entries of the
// pencil), far from overflow, underflow and zero.
__device__ __forceinline__ double sqrt_nr(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, s);
    return fma(d, h, g);
}
__device__ __forceinline__ double rcp_nr(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}

// xLARFG scalars for a non-trivial reflector (ss = ||x||^2 > 0 or alpha not
// real): beta = -sign(Re alpha) sqrt(|alpha|^2 + ss), tau = (beta - alpha) /
// beta and sc = 1 / (alpha - beta), with a single reciprocal: 1 / beta and
// 1 / |alpha - beta|^2 both come from q = 1 / (beta |alpha - beta|^2).
// |Re(alpha - beta)| = |Re alpha| + |beta| >= |beta| > 0, so q is finite.
template <class S>
__device__ __forceinline__ void larfg_core(S alpha, double ss, S &tau, double &beta, S &sc)
{
    const double b = -(re(alpha) >= 0.0 ? 1.0 : -1.0) * sqrt_nr(abs2(alpha) + ss);
    const S amb = sub(alpha, mk<S>(b, 0.0));
    const double n2 = abs2(amb);
    const double q = rcp_nr(b * n2);
    const double rb = n2 * q;                     // 1 / beta
    tau = mk<S>((b - re(alpha)) * rb, -im(alpha) * rb);
    sc = scal(conj_(amb), b * q);                 // conj(amb) / |amb|^2
    beta = b;
}

// ------------------------------------------------------- wave reductions
// Cross-lane data movement with DPP (in-row permutations, no LDS round trip)
// and v_readlane (broadcast of one lane into scalar registers).
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffu), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// value of lane l in every lane (l wave-uniform)
__device__ __forceinline__ double bcast(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ zd bcast(zd v, int l) { return mk<zd>(bcast(v.re, l), bcast(v.im, l)); }

// sum over aligned groups of G lanes (G in {2, 4, 8, 16}), result in every
// lane of the group: quad permutations, then half-row and row mirrors
template <int G> __device__ inline double group_sum(double v) {
    v += dpp_d<0xB1>(v);                              // quad_perm [1,0,3,2]
    if (G >= 4) v += dpp_d<0x4E>(v);                  // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_d<0x141>(v);                 // row_half_mirror
    if (G >= 16) v += dpp_d<0x140>(v);                // row_mirror
    return v;
}
template <int G> __device__ inline zd group_sum(zd v) { return mk<zd>(group_sum<G>(v.re), group_sum<G>(v.im)); }
// sum over the 64 lanes, result in every lane
__device__ inline double wave_sum(double v) {
    v = group_sum<16>(v);
    return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}
__device__ inline zd wave_sum(zd v) { return mk<zd>(wave_sum(v.re), wave_sum(v.im)); }

// ------------------------------------------------------- stage-two index map
// 1-based formulas of the unblocked stage-two algorithm.
__host__ __device__ inline int64_t nblocks(int64_t n, int64_t r, int64_t j) {  // blocks with >= 2 rows
    return n - j - 2 < 0 ? 0 : 1 + (n - j - 2) / r;
}
__host__ __device__ inline int64_t i64min(int64_t a, int64_t b) { return a < b ? a : b; }
__host__ __device__ inline int64_t i64max(int64_t a, int64_t b) { return a > b ? a : b; }

// Band storage of a scratch copy: element (i,c) (0-based) with
// -BU <= i - c <= BL lives at B[(i - c + BU) + c * ldb], ldb = BU + BL + 1.
struct Band {
    int64_t BU, BL, ldb;
    __host__ __device__ inline int64_t idx(int64_t i0, int64_t c0) const { return (i0 - c0 + BU) + c0 * ldb; }
};

// Maximum supported r on the GPU path: a lazy update column segment
// (q + r - 1 <= 63 rows) must fit one 64-lane wavefront.
constexpr int kMaxR = 32;
constexpr int kWin = 64;     // padded window-factor order (>= q + r - 1)

}  // namespace ht
