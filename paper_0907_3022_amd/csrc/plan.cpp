// Host-side plan of one Chebyshev time step (Sect. 2.2 of arXiv:0907.3022):
// spectral shift and scale, Bessel-function weights c_k = (-i)^k J_k(a dt)
// and the truncation order from the decay of J_k (eq. (dec_Bessel)).
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace chebtd {

// log J_nu(z) for nu > z from the Debye expansion's leading term,
// J_nu(nu sech(alpha)) ~ exp(-nu (alpha - tanh alpha)) / sqrt(2 pi nu tanh alpha).
static double log_bessel_debye(double nu, double z)
{
    double alpha = std::acosh(nu / z);
    double th = std::tanh(alpha);
    return -nu * (alpha - th) - 0.5 * std::log(2.0 * M_PI * nu * th);
}

// Order at which Miller's backward recurrence starts: beyond max(kmax, z)
// far enough that J there is below 1e-40 of the values wanted.
static int miller_start(double z, int kmax)
{
    double base = std::max((double)kmax, z);
    int n = (int)std::ceil(base) + 16;
    if (z > 0.0) {
        while (n < 10 * (int)base + 64) {
            if ((double)n > 1.05 * z + 8.0 && log_bessel_debye((double)n, z) < -92.0) break;
            n += 8;
        }
    }
    return n + (n & 1);  // even
}

// J_0(z)..J_kmax(z) by Miller's backward recurrence J_{k-1} = (2k/z) J_k -
// J_{k+1}, normalised with J_0 + 2 sum J_{2k} = 1 (compensated summation).
int bessel_miller(double z, int kmax, std::vector<double> &J)
{
    if (kmax < 0 || !(z >= 0.0) || !std::isfinite(z)) return -1;
    J.assign((size_t)kmax + 1, 0.0);
    if (z == 0.0) {
        J[0] = 1.0;
        return 0;
    }
    if (z < 1e-10) {
        // J_k(z) = (z/2)^k / k! * (1 - (z/2)^2/(k+1) + ...)
        double t = 1.0, q = 0.25 * z * z;
        for (int k = 0; k <= kmax; ++k) {
            if (k) t *= 0.5 * z / k;
            J[(size_t)k] = t * (1.0 - q / (k + 1));
        }
        return 0;
    }
    const int ns = miller_start(z, kmax);
    std::vector<double> w((size_t)ns + 2, 0.0);
    w[(size_t)ns] = 1e-280;
    const double two_over_z = 2.0 / z;
    for (int k = ns; k >= 1; --k) {
        w[(size_t)k - 1] = (k * two_over_z) * w[(size_t)k] - w[(size_t)k + 1];
        if (std::fabs(w[(size_t)k - 1]) > 1e240) {
            for (size_t j = (size_t)k - 1; j <= (size_t)ns + 1; ++j) w[j] *= 1e-240;
        }
    }
    // Neumann sum with Kahan compensation
    double s = w[0], c = 0.0;
    for (int k = 2; k <= ns; k += 2) {
        double y = 2.0 * w[(size_t)k] - c;
        double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    for (int k = 0; k <= kmax; ++k) J[(size_t)k] = w[(size_t)k] / s;
    return 0;
}

// Last order kept: every |J_k(z)| with k > M lies below tol.  J_k(z) is
// monotone for k > z, so M + 1 is the first such k beyond z.
int truncation_order(double z, double tol)
{
    if (!(tol > 0.0) || !(z >= 0.0) || !std::isfinite(z)) return -1;
    int kmax = (int)std::ceil(z) + 32;
    // widen the search with the Debye estimate before computing
    while (z > 0.0 && log_bessel_debye((double)kmax, z) > std::log(tol) - 4.0) kmax += 16;
    std::vector<double> J;
    for (;;) {
        if (bessel_miller(z, kmax, J)) return -1;
        for (int k = (int)std::floor(z) + 1; k <= kmax; ++k) {
            if (k >= 1 && std::fabs(J[(size_t)k]) < tol) return k - 1;
        }
        kmax = 2 * kmax + 16;
    }
}

void shift_scale(double emin, double emax, double alpha, double *a, double *b)
{
    const double eps = alpha * (emax - emin);
    *b = 0.5 * (emax + emin);
    *a = 0.5 * (emax - emin + eps);
}

// gamma_0 = e^{-i b dt} J_0(a dt), gamma_k = 2 e^{-i b dt} (-i)^k J_k(a dt).
void step_weights(double a, double b, double dt, int M, std::vector<double> &gamma)
{
    std::vector<double> J;
    bessel_miller(a * dt, M, J);
    const std::complex<double> phase(std::cos(b * dt), -std::sin(b * dt));
    static const std::complex<double> minus_i_pow[4] = {
        {1.0, 0.0}, {0.0, -1.0}, {-1.0, 0.0}, {0.0, 1.0}};
    gamma.assign(2 * ((size_t)M + 1), 0.0);
    for (int k = 0; k <= M; ++k) {
        std::complex<double> g = phase * minus_i_pow[k & 3] * J[(size_t)k];
        if (k) g *= 2.0;
        gamma[2 * (size_t)k] = g.real();
        gamma[2 * (size_t)k + 1] = g.imag();
    }
}

}  // namespace chebtd
