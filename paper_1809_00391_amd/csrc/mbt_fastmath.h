// mbt_fastmath.h -- FP64 sine, cosine and exponential used per particle by
// the tracker kernels (host-callable too, so their accuracy is tested on the
// CPU against extended-precision references).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mbt {

// ---------------------------------------------------------------------------
// FP64 sine/cosine/exponential for the per-particle map.
//
// sincos_poly: sin and cos of |r| <= pi/4 as r + r z P(z) and
// 1 - z/2 + z^2 Q(z), z = r^2, with P and Q of degree 5 minimising the largest
// error of sin and cos on the interval (Remez exchange in 60-digit
// arithmetic, gen_sincos_minimax.py beside this file: 3.4e-18 relative for
// sin, 4.7e-20 for cos before rounding), in Horner form with FMAs.
// sincos_cw: argument reduction by pi/2 after Cody and Waite (1980): with
// k = rint(2x/pi), r = x - k*P1 - k*P2 where P1 is the double nearest pi/2
// and P2 = pi/2 - P1, each step one FMA, then a quadrant swap.  Arguments
// beyond 1e5 (never reached by particles near a bucket) use the library.
// ---------------------------------------------------------------------------
// One Horner step p*z + c, rounded once.  On the device it is spelled as a
// single three-operand v_fma_f64 whose coefficient operand is a scalar
// register pair (a VOP3 instruction may read one): the coefficients are
// loop-invariant, stay in scalar registers, and no vector register or copy
// is spent on them, where the compiler's own choice copies each coefficient
// into a vector register first.  The result is the same correctly rounded
// FMA either way.
__host__ __device__ __forceinline__ double horner(double p, double z, double c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r;
    __asm__("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(z), "s"(c));
    return r;
#else
    return fma(p, z, c);
#endif
}

constexpr double kPio2Hi = 1.5707963267948966;     // double nearest pi/2
constexpr double kPio2Lo = 6.123233995736766e-17;  // pi/2 - kPio2Hi
constexpr double kTwoOverPi = 0.6366197723675814;

__host__ __device__ __forceinline__ void sincos_poly(double r, double &s, double &c)
{
    const double z = r * r;
    double ps = 1.5896827930152048e-10;           // S5
    ps = horner(ps, z, -2.505075865328765e-08);   // S4
    ps = horner(ps, z, 2.7557313695226595e-06);   // S3
    ps = horner(ps, z, -0.0001984126982981695);   // S2
    ps = horner(ps, z, 0.008333333333322425);     // S1
    ps = horner(ps, z, -0.16666666666666632);     // S0
    s = fma(r * z, ps, r);
    double pc = -1.1359669889814536e-11;          // C5
    pc = horner(pc, z, 2.0875723684860718e-09);   // C4
    pc = horner(pc, z, -2.7557314355245e-07);     // C3
    pc = horner(pc, z, 2.4801587289491837e-05);   // C2
    pc = horner(pc, z, -0.0013888888888874138);   // C1
    pc = horner(pc, z, 0.0416666666666666);       // C0
    pc = fma(pc, z, -0.5);                        // -1/2 (inline constant)
    c = fma(z, pc, 1.0);
}

// x = q*pi/2 + r: rotate (sin r, cos r) into quadrant q.  The sine changes
// sign where bit 1 of q is set, the cosine where bit 1 of q + 1 is; each
// negation is that bit moved into the sign bit and XORed in (exact, and the
// same value as a negation, signed zeros included).
__host__ __device__ __forceinline__ void quadrant(int q, double sr, double cr, double &s, double &c)
{
    const double s0 = (q & 1) ? cr : sr;
    const double c0 = (q & 1) ? sr : cr;
    const uint64_t sign_s = (uint64_t)(((uint32_t)q << 30) & 0x80000000u) << 32;
    const uint64_t sign_c = (uint64_t)(((uint32_t)q + 1u) << 30 & 0x80000000u) << 32;
    s = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, s0) ^ sign_s);
    c = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, c0) ^ sign_c);
}

// Library sine and cosine for the rare huge argument, kept out of line so
// the per-particle loop stays small.
// Returned by value: an out-parameter of a call that is not inlined would
// force the caller's results through scratch memory on every path.
struct SinCos {
    double s, c;
};
__host__ __device__ __noinline__ SinCos sincos_libm(double x)
{
    return SinCos{sin(x), cos(x)};
}

__host__ __device__ __forceinline__ void sincos_cw(double x, double &s, double &c)
{
    if (!(fabs(x) < 1e5)) {
        const SinCos r = sincos_libm(x);
        s = r.s;
        c = r.c;
        return;
    }
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kPio2Hi, x);
    r = fma(-k, kPio2Lo, r);
    double sr, cr;
    sincos_poly(r, sr, cr);
    quadrant((int)k, sr, cr, s, c);
}

// sin and cos of 2*pi*u for u in (0, 1]: 4u = k + f exactly (|f| <= 1/2),
// angle f*pi/2 in [-pi/4, pi/4], quadrant k.
__host__ __device__ __forceinline__ void sincos_2pi(double u, double &s, double &c)
{
    const double t = 4.0 * u;
    const double k = rint(t);
    double sr, cr;
    sincos_poly((t - k) * kPio2Hi, sr, cr);
    quadrant((int)k, sr, cr, s, c);
}

__host__ __device__ __noinline__ double exp_libm(double y) { return exp(y); }

// exp(y) for the long-range decay across a bunch (alpha*tau ~ 1e-5): the
// Taylor polynomial of degree 3 for |y| < 1e-4 (truncation y^4/24 < 4.2e-18,
// under 0.04 ulp of 1), of degree 4 for |y| < 1e-3 (y^5/120 < 8.4e-18),
// otherwise the library.
__host__ __device__ __forceinline__ double exp_taylor3(double y)
{
    double p = 1.0 / 6.0;
    p = fma(p, y, 0.5);
    p = fma(p, y, 1.0);
    return fma(p, y, 1.0);
}

__host__ __device__ __forceinline__ double exp_taylor4(double y)
{
    double p = 1.0 / 24.0;
    p = horner(p, y, 1.0 / 6.0);
    p = fma(p, y, 0.5);
    p = fma(p, y, 1.0);
    return fma(p, y, 1.0);
}

__host__ __device__ __forceinline__ double exp_small(double y)
{
    const double a = fabs(y);
    if (a < 1e-4)
        return exp_taylor3(y);
    if (a < 1e-3)
        return exp_taylor4(y);
    return exp_libm(y);
}

// (cos(n x), sin(n x)) from (cos x, sin x): the triple-angle identities for
// n = 3 (sin 3x = sin x (3 - 4 sin^2 x), cos 3x = cos x (4 cos^2 x - 3)),
// repeated complex products otherwise.
__host__ __device__ __forceinline__ void multiple_angle(int n, double s1, double c1, double &sn, double &cn)
{
    if (n == 3) {
        sn = s1 * fma(-4.0 * s1, s1, 3.0);
        cn = c1 * fma(4.0 * c1, c1, -3.0);
        return;
    }
    double s = s1, c = c1;
    for (int i = 1; i < n; ++i) {
        const double cs = fma(c, c1, -s * s1);
        const double ss = fma(s, c1, c * s1);
        c = cs;
        s = ss;
    }
    sn = s;
    cn = c;
}

#ifndef MBT_FAST_NOISE_MATH
#define MBT_FAST_NOISE_MATH 1
#endif

// (m - 1) / (m + 1) for m in [sqrt(1/2), sqrt(2)).  On the device with the
// fast noise arithmetic: the hardware reciprocal refined by two Newton steps
// and a final residual correction (within an ulp of the quotient).
__host__ __device__ __forceinline__ double atanh_arg(double m)
{
#if defined(__HIP_DEVICE_COMPILE__) && MBT_FAST_NOISE_MATH
    const double d = m + 1.0, n = m - 1.0;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
#else
    return (m - 1.0) / (m + 1.0);
#endif
}

// sqrt(x) for the Box-Muller radius (x > 0).  On the device with the fast
// noise arithmetic: the hardware reciprocal square root refined by one
// coupled Newton step for sqrt(x) and 1/(2 sqrt(x)), then a residual
// correction (within an ulp).
__host__ __device__ __forceinline__ double sqrt_pos(double x)
{
#if defined(__HIP_DEVICE_COMPILE__) && MBT_FAST_NOISE_MATH
    const double y = __builtin_amdgcn_rsq(x);
    double r = x * y, h = 0.5 * y;
    const double e = fma(-r, h, 0.5);
    r = fma(r, e, r);
    h = fma(h, e, h);
    return fma(fma(-r, r, x), h, r);
#else
    return sqrt(x);
#endif
}

// Natural logarithm of u in (0, 1] (the Box-Muller uniform).  u = m 2^e
// with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s), s = (m - 1)/(m + 1),
// |s| <= 3 - 2 sqrt(2) = 0.1716, with atanh(s) = s + s z L(z), z = s^2, L the
// degree-6 polynomial minimising the relative error on that interval (Remez,
// gen_sincos_minimax.py: 1.2e-18 before rounding; the series
// s + s^3/3 + s^5/5 + ... would need terms to s^19); e ln 2 is added with
// ln 2 split into a 32-bit head and a tail so that e * head is exact.
__host__ __device__ __forceinline__ double log_unit(double u)
{
    int e;
    double m = frexp(u, &e);  // m in [1/2, 1)
    if (m < 0.7071067811865476) {
        m = m + m;
        e -= 1;
    }
    const double s = atanh_arg(m);
    const double z = s * s;
    double p = 0.07397974850291429;               // L6
    p = horner(p, z, 0.07657025276056356);        // L5
    p = horner(p, z, 0.09091782163059837);        // L4
    p = horner(p, z, 0.11111099286592262);        // L3
    p = horner(p, z, 0.1428571437119381);         // L2
    p = horner(p, z, 0.19999999999707338);        // L1
    p = horner(p, z, 0.3333333333333367);         // L0
    const double lm = fma(2.0 * s * z, p, 2.0 * s);
    const double ln2_hi = 0.693147180369123816490;    // ln 2 to 32 bits
    const double ln2_lo = 1.90821492927058770002e-10; // ln 2 - ln2_hi
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, lm));
}

}  // namespace mbt
