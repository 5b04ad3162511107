// Demagnetisation factors of an ellipsoid (the body E of Sec. 2.1, whose
// factor N_d scales the far field -Ms N_d mbar), from Carlson's symmetric
// elliptic integral R_D:  N_a = (abc/3) R_D(b^2, c^2, a^2) and cyclically.
// R_D is evaluated by Carlson's duplication algorithm (B. C. Carlson,
// "Numerical computation of real or complex elliptic integrals", Numerical
// Algorithms 10, 1995), with its fifth-order series for the final step.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace gspm {

double carlson_rd(double x, double y, double z) {
    double A0 = (x + y + 3.0 * z) / 5.0, A = A0;
    double Q = std::pow(0.25 * 1e-16, -1.0 / 6.0) * std::max({std::fabs(A0 - x), std::fabs(A0 - y), std::fabs(A0 - z)});
    double sum = 0.0, fac = 1.0, pow4 = 1.0;
    for (int it = 0; it < 100 && pow4 * Q >= std::fabs(A); ++it) {
        const double sx = std::sqrt(x), sy = std::sqrt(y), sz = std::sqrt(z);
        const double lam = sx * sy + sx * sz + sy * sz;
        sum += fac / (sz * (z + lam));
        fac *= 0.25;
        pow4 *= 0.25;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        A = 0.25 * (A + lam);
    }
    // A - x after m duplications equals 4^-m (A0 - x0)
    const double X = (A - x) / A, Y = (A - y) / A, Z = -(X + Y) / 3.0;
    const double XY = X * Y, Z2 = Z * Z;
    const double E2 = XY - 6.0 * Z2, E3 = (3.0 * XY - 8.0 * Z2) * Z, E4 = 3.0 * (XY - Z2) * Z2, E5 = XY * Z2 * Z;
    const double series = 1.0 - 3.0 * E2 / 14.0 + E3 / 6.0 + 9.0 * E2 * E2 / 88.0 - 3.0 * E4 / 22.0 -
                          9.0 * E2 * E3 / 52.0 + 3.0 * E5 / 26.0;
    return pow4 * series / (A * std::sqrt(A)) + 3.0 * sum;
}

void demag_factors(double a, double b, double c, double N[3]) {
    const double v = a * b * c / 3.0;
    N[0] = v * carlson_rd(b * b, c * c, a * a);
    N[1] = v * carlson_rd(c * c, a * a, b * b);
    N[2] = v * carlson_rd(a * a, b * b, c * c);
}

}  // namespace gspm
