// Host-side accuracy check of the tracker's FP64 sin/cos/exp routines
// (paper_1809_00391_amd/csrc/mbt_fastmath.h) against long-double libm.
// Prints: name max_abs_err max_rel_err
#include "mbt_fastmath.h"

#include <cmath>
#include <cstdio>
#include <random>

int main()
{
    std::mt19937_64 rng(12345);
    auto report = [](const char *name, long double ea, long double er) {
        std::printf("%s %.3Le %.3Le\n", name, ea, er);
    };
    // sincos_cw over the ranges the kernels use: RF phase (|x| < ~4),
    // long-range phases (|x| < ~50) and wide arguments up to the 1e5 cut.
    const double ranges[] = {1e-6, 0.3, 0.785, 4.0, 60.0, 1e3, 9.9e4, 3e5};
    for (double R : ranges) {
        std::uniform_real_distribution<double> U(-R, R);
        long double ea = 0, er = 0;
        for (int i = 0; i < 200000; ++i) {
            double x = U(rng), s, c;
            mbt::sincos_cw(x, s, c);
            long double ts = sinl((long double)x), tc = cosl((long double)x);
            long double d1 = fabsl((long double)s - ts), d2 = fabsl((long double)c - tc);
            ea = fmaxl(ea, fmaxl(d1, d2));
            if (fabsl(ts) > 0) er = fmaxl(er, d1 / fabsl(ts));
        }
        char name[64];
        std::snprintf(name, sizeof name, "sincos_cw_%g", R);
        report(name, ea, er);
    }
    {
        // 2*pi*u on the 53-bit grid of the noise uniforms
        long double ea = 0;
        for (int i = 0; i < 400000; ++i) {
            uint64_t w = rng();
            double u = (double)(w >> 11) * 0x1.0p-53 + 0x1.0p-54;
            double s, c;
            mbt::sincos_2pi(u, s, c);
            long double th = 2.0L * 3.14159265358979323846264338327950288L * (long double)u;
            ea = fmaxl(ea, fmaxl(fabsl((long double)s - sinl(th)), fabsl((long double)c - cosl(th))));
        }
        report("sincos_2pi", ea, 0);
    }
    {
        std::uniform_real_distribution<double> U(-2e-3, 2e-3);
        long double er = 0;
        for (int i = 0; i < 200000; ++i) {
            double y = U(rng);
            long double t = expl((long double)y);
            er = fmaxl(er, fabsl((long double)mbt::exp_small(y) - t) / t);
        }
        report("exp_small", 0, er);
    }
    {
        // the degree-3 range alone, densely
        std::uniform_real_distribution<double> U(-1.2e-4, 1.2e-4);
        long double er = 0;
        for (int i = 0; i < 200000; ++i) {
            double y = U(rng);
            long double t = expl((long double)y);
            er = fmaxl(er, fabsl((long double)mbt::exp_small(y) - t) / t);
        }
        report("exp_small_1e-4", 0, er);
    }
    {
        // log on the 53-bit uniform grid of (0, 1], including the extremes
        long double er = 0;
        for (int i = 0; i < 400000; ++i) {
            uint64_t w = rng();
            if (i == 0) w = 0;
            if (i == 1) w = ~0ull;
            if (i < 2000) w >>= (i % 60);  // small u: large |log|
            double u = (double)(w >> 11) * 0x1.0p-53 + 0x1.0p-54;
            long double t = logl((long double)u);
            long double d = fabsl((long double)mbt::log_unit(u) - t);
            er = fmaxl(er, t != 0 ? d / fabsl(t) : d);
        }
        report("log_unit", 0, er);
    }
    for (int n = 2; n <= 6; ++n) {
        std::uniform_real_distribution<double> U(-1.0, 1.0);
        long double ea = 0;
        for (int i = 0; i < 100000; ++i) {
            double x = U(rng), s1, c1, sn, cn;
            mbt::sincos_cw(x, s1, c1);
            mbt::multiple_angle(n, s1, c1, sn, cn);
            ea = fmaxl(ea, fmaxl(fabsl((long double)sn - sinl((long double)n * x)),
                                 fabsl((long double)cn - cosl((long double)n * x))));
        }
        char name[64];
        std::snprintf(name, sizeof name, "multiple_angle_%d", n);
        report(name, ea, 0);
    }
    return 0;
}
