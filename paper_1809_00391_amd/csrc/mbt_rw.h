// mbt_rw.h -- short-range resistive-wall wake of a round pipe (host code,
// evaluated once per table when a job is bound).
//
// For a pipe of radius b, DC conductivity sigma and length L, with z = c t and
// the characteristic distance s0 = (2 b^2 / (Z0 sigma))^(1/3), the wake of
// Bane and Sands ("The short-range resistive wall wakefields", 1995) in SI
// units is
//   W(t) = (4 Z0 c L / (pi b^2)) [ exp(-z/s0) cos(sqrt(3) z/s0) / 3
//           - (sqrt(2)/pi) I(z/s0) ],  I(a) = int_0^inf x^2 exp(-a x^2) / (x^6 + 8) dx,
// the transform of the impedance (L / (2 pi b)) / (1/Z_s + i w eps0 b / 2) with
// the surface impedance Z_s = (1 + i) sqrt(w mu0 / (2 sigma)).  W(0+) =
// Z0 c L / (pi b^2) for any conductivity; far behind the charge it tends to
// the thick-wall -(c L / (4 pi b)) sqrt(Z0 / (pi sigma)) z^(-3/2).
#pragma once

#include <cmath>
#include <vector>

namespace mbt {

struct ResistiveWall {
    double radius_m, conductivity_S_m, length_m;
};

// Gauss-Legendre nodes and weights on [-1, 1]: roots of P_n by Newton's
// method from the Chebyshev guesses, P_n and P_n' from the three-term
// recurrence; w = 2 / ((1 - x^2) P_n'(x)^2).
inline void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.141592653589793;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16)
                break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Composite Gauss-Legendre (panels x nodes) of f over [lo, hi].
template <class F>
double gl_integrate(F f, double lo, double hi, int panels, const std::vector<double> &x,
                    const std::vector<double> &w)
{
    const double h = (hi - lo) / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double c = lo + (p + 0.5) * h;
        double s = 0.0;
        for (size_t i = 0; i < x.size(); ++i)
            s += w[i] * f(c + 0.5 * h * x[i]);
        sum += 0.5 * h * s;
    }
    return sum;
}

// I(a) for a > 0.  a >= 1: x = s / sqrt(a) leaves s^2 exp(-s^2) / (8 + s^6/a^3)
// over s in [0, 7]; a < 1: [0, 1] in x and [0, 1] in y = 1/x, the latter in
// fine panels to follow exp(-a / y^2).
inline double rw_integral(double a, const std::vector<double> &x, const std::vector<double> &w)
{
    if (a >= 1.0) {
        const double a3 = a * a * a;
        auto f = [a3](double s) {
            const double s2 = s * s;
            return s2 * std::exp(-s2) / (8.0 + s2 * s2 * s2 / a3);
        };
        return gl_integrate(f, 0.0, 7.0, 16, x, w) / (a * std::sqrt(a));
    }
    auto fx = [a](double t) {
        const double t2 = t * t;
        return t2 * std::exp(-a * t2) / (t2 * t2 * t2 + 8.0);
    };
    auto fy = [a](double y) {
        const double y2 = y * y;
        return y2 * std::exp(-a / y2) / (1.0 + 8.0 * y2 * y2 * y2);
    };
    return gl_integrate(fx, 0.0, 1.0, 8, x, w) + gl_integrate(fy, 0.0, 1.0, 128, x, w);
}

// W(t) in V/C for t >= 0 (W(0+) at t = 0).
inline double rw_wake(const ResistiveWall &rw, double t, const std::vector<double> &x,
                      const std::vector<double> &w)
{
    const double c = 299792458.0, z0 = 376.730313668, pi = 3.141592653589793;
    const double b = rw.radius_m;
    const double amp = 4.0 * z0 * c * rw.length_m / (pi * b * b);
    if (t <= 0.0)
        return 0.25 * amp;  // 1/3 - (sqrt(2)/pi) I(0), I(0) = pi / (12 sqrt(2))
    const double s0 = std::cbrt(2.0 * b * b / (z0 * rw.conductivity_S_m));
    const double u = c * t / s0;
    return amp * (std::exp(-u) * std::cos(std::sqrt(3.0) * u) / 3.0 -
                  (std::sqrt(2.0) / pi) * rw_integral(u, x, w));
}

}  // namespace mbt
