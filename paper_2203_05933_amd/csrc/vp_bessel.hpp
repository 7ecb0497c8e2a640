// Modified Bessel functions I_n and K_n of integer order on the host, in
// long double, for the modified Helmholtz translation operators and
// near-field matrices built at plan time.
//
//   I_n(x) = sum_{k>=0} (x/2)^(2k+n) / (k! (n+k)!)                (power series;
//            every term is positive, so it converges without cancellation)
//   K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt,  v = 0, 1     (integral
//            representation, by the trapezoidal rule: the integrand is analytic
//            in the strip |Im t| < pi/2, where it grows to about e^x times its
//            size on the real line, so the rule's relative error is about
//            exp(x - pi^2 / step); step = min(1/8, pi^2 / (x + 50)) keeps it
//            below e^-45, under long-double rounding)
//   K_{n+1}(x) = K_{n-1}(x) + (2n / x) K_n(x)                     (upward
//            recurrence, stable for K)
#pragma once

#include <cmath>

namespace vp {

// out[n] = I_n(x), n = 0..nmax, x >= 0
inline void bessel_i_all(long double x, int nmax, long double *out) {
    const long double h = x / 2, h2 = h * h;
    long double lead = 1.0L;  // (x/2)^n / n!
    for (int n = 0; n <= nmax; ++n) {
        if (n > 0) lead *= h / n;
        long double term = lead, sum = lead;
        for (int k = 1; k < 400; ++k) {
            term *= h2 / ((long double)k * (k + n));
            sum += term;
            if (term <= sum * 1e-24L) break;
        }
        out[n] = sum;
    }
}

// K_v(x) for v = 0 and 1, x > 0
inline void bessel_k01(long double x, long double &k0, long double &k1) {
    const long double pi2 = 9.869604401089358618834490999876151L;
    const long double step = std::fmin(0.125L, pi2 / (x + 50.0L));
    long double s0 = 0.5L * std::exp(-x), s1 = 0.0L;  // t = 0 carries half weight; cosh(0) = 1, the K_1 term
    s1 = 0.5L * std::exp(-x);
    for (int i = 1; i < 100000; ++i) {
        const long double t = i * step;
        const long double e = std::exp(-x * std::cosh(t));
        s0 += e;
        const long double e1 = e * std::cosh(t);
        s1 += e1;
        if (e1 <= s1 * 1e-26L && e <= s0 * 1e-26L) break;
    }
    k0 = step * s0;
    k1 = step * s1;
}

// out[n] = K_n(x), n = 0..nmax, x > 0
inline void bessel_k_all(long double x, int nmax, long double *out) {
    long double k0, k1;
    bessel_k01(x, k0, k1);
    out[0] = k0;
    if (nmax >= 1) out[1] = k1;
    for (int n = 1; n < nmax; ++n) out[n + 1] = out[n - 1] + (2.0L * n / x) * out[n];
}

}  // namespace vp
