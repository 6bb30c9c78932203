// model.cpp -- substitution model set-up on the host.
//
// GTR (the paper supports GTR and runs JC69 + Gamma; Methods, "Phylogenetic
// Topographer"): Q_ij = r_ij pi_j for i != j, rows summing to zero, scaled to
// one expected substitution per unit time.  Because pi_i Q_ij is symmetric,
// S = Pi^1/2 Q Pi^-1/2 is symmetric; a cyclic Jacobi sweep diagonalises it,
// S = V diag(lam) V^T, which gives P(t) = U diag(exp(lam t)) Uinv with
// U = Pi^-1/2 V and Uinv = V^T Pi^1/2.  The kernels only ever need U, Uinv and
// lam: transition matrices, their derivatives and the per-edge eigenbasis
// tables all follow from them.  Both sides of an edge project onto the
// eigenbasis with the same matrix W = Pi^1/2 V (W_im = pi_i U_im = Uinv_mi).
//
// Discrete Gamma rate variation (Yang 1994, category means): K categories of
// probability 1/K cut at the quantiles of Gamma(alpha, rate alpha); the rate
// of a category is K times the partial first moment over its interval, which
// equals K [G(alpha+1, alpha x_hi) - G(alpha+1, alpha x_lo)] with G the
// regularised lower incomplete gamma function.
#include <cmath>
#include <cstring>

#include "pt_internal.hpp"

namespace pt {
namespace {

// Regularised lower incomplete gamma G(a, x).
double inc_gamma(double a, double x) {
    if (x <= 0.0) return 0.0;
    const double log_front = a * std::log(x) - x - std::lgamma(a);
    if (x <= a + 1.0) {
        // G = x^a e^-x / Gamma(a+1) * sum_n x^n / ((a+1)...(a+n))
        double term = 1.0, sum = 1.0;
        for (int n = 1; n < 100000; ++n) {
            term *= x / (a + n);
            sum += term;
            if (term <= sum * 1e-17) break;
        }
        return std::exp(log_front) * sum / a;
    }
    // 1 - G = x^a e^-x / Gamma(a) * CF, continued fraction evaluated from the
    // bottom up; the depth needed near x ~ a grows like sqrt(a).
    double f = 0.0;
    const int depth = 300 + int(30.0 * std::sqrt(a));
    for (int k = depth; k >= 1; --k) {
        f = k * (k - a) / (x + 2 * k + 1 - a - f);
    }
    double upper = std::exp(log_front) / (x + 1 - a - f);
    return 1.0 - upper;
}

// y with G(a, y) = q: Newton steps on G from a Wilson-Hilferty start, kept
// inside a shrinking bracket (bisection when Newton leaves it).
double inc_gamma_inv(double a, double q) {
    double lo = 0.0, hi = std::max(1.0, a);
    while (inc_gamma(a, hi) < q) { lo = hi; hi *= 2.0; }
    // Wilson-Hilferty approximation of the chi-square quantile, in gamma units
    double z;
    {
        // inverse standard normal by bisection on erfc (start value only)
        double zl = -10, zh = 10;
        for (int i = 0; i < 80; ++i) {
            double zm = 0.5 * (zl + zh);
            if (0.5 * std::erfc(-zm / std::sqrt(2.0)) < q) zl = zm; else zh = zm;
        }
        z = 0.5 * (zl + zh);
    }
    double c = 1.0 / (9.0 * a);
    double y = a * std::pow(1.0 - c + z * std::sqrt(c), 3);
    if (!(y > lo && y < hi)) y = 0.5 * (lo + hi);
    const double lga = std::lgamma(a);
    for (int it = 0; it < 200; ++it) {
        double g = inc_gamma(a, y) - q;
        if (g < 0) lo = y; else hi = y;
        double dens = std::exp((a - 1.0) * std::log(y) - y - lga);
        double yn = y - g / dens;
        if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
        if (std::fabs(yn - y) <= 1e-15 * y || hi - lo <= 1e-15 * hi) { y = yn; break; }
        y = yn;
    }
    return y;
}

// Cyclic Jacobi diagonalisation of a symmetric 4x4 matrix A (destroyed).
void jacobi4(double A[4][4], double V[4][4], double lam[4]) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) off += A[i][j] * A[i][j];
        if (off < 1e-300) break;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 4; ++k) {  // columns p, q
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {  // rows p, q
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < 4; ++i) lam[i] = A[i][i];
}

}  // namespace

pt_status gamma_category_rates(double alpha, int K, double *out, std::string &err) {
    if (K < 1 || K > kMaxCats) { err = "n_cats must be in 1..8"; return PT_EINVAL; }
    if (K == 1) { out[0] = 1.0; return PT_OK; }
    if (!(alpha > 0.0) || !std::isfinite(alpha)) { err = "alpha must be finite and > 0"; return PT_EINVAL; }
    double prev = 0.0;
    for (int i = 0; i < K; ++i) {
        double cum = 1.0;
        if (i + 1 < K) cum = inc_gamma(alpha + 1.0, inc_gamma_inv(alpha, double(i + 1) / K));
        out[i] = K * (cum - prev);
        prev = cum;
    }
    return PT_OK;
}

pt_status build_model(const pt_model &m, AlnDev &d, std::string &err) {
    double fsum = 0.0;
    for (int i = 0; i < 4; ++i) {
        if (!(m.freqs[i] > 0.0) || !std::isfinite(m.freqs[i])) { err = "freqs must be > 0"; return PT_EINVAL; }
        fsum += m.freqs[i];
    }
    if (std::fabs(fsum - 1.0) > 1e-9) { err = "freqs must sum to 1 (within 1e-9)"; return PT_EINVAL; }
    for (int x = 0; x < 6; ++x)
        if (!(m.rates[x] > 0.0) || !std::isfinite(m.rates[x])) { err = "rates must be finite and > 0"; return PT_EINVAL; }
    pt_status st = gamma_category_rates(m.alpha, m.n_cats, d.rate, err);
    if (st) return st;
    d.K = m.n_cats;
    d.Kp = 1;
    while (d.Kp < d.K) d.Kp *= 2;
    for (int k = d.K; k < kMaxCats; ++k) d.rate[k] = 0.0;

    static const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {1, 2, 3, 2, 3, 3};
    double R[4][4] = {};
    for (int x = 0; x < 6; ++x) { R[I[x]][J[x]] = m.rates[x]; R[J[x]][I[x]] = m.rates[x]; }
    double mu = 0.0;  // mean rate before normalisation
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            if (i != j) mu += m.freqs[i] * R[i][j] * m.freqs[j];
    double S[4][4], sq[4];
    for (int i = 0; i < 4; ++i) sq[i] = std::sqrt(m.freqs[i]);
    for (int i = 0; i < 4; ++i) {
        double row = 0.0;
        for (int j = 0; j < 4; ++j)
            if (j != i) { S[i][j] = R[i][j] * sq[i] * sq[j] / mu; row += R[i][j] * m.freqs[j] / mu; }
        S[i][i] = -row;
    }
    double V[4][4], lam[4];
    jacobi4(S, V, lam);
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k) {
            d.U[i * 4 + k] = V[i][k] / sq[i];
            d.Uinv[k * 4 + i] = V[i][k] * sq[i];
            d.W[i * 4 + k] = V[i][k] * sq[i];
        }
    for (int k = 0; k < 4; ++k) d.lam[k] = lam[k];
    for (int i = 0; i < 4; ++i) d.freqs[i] = m.freqs[i];
    return PT_OK;
}

}  // namespace pt
