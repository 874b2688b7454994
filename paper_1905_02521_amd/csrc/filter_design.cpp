// filter_design.cpp -- host FP64 design of the coloured-noise FIR filter.
//
//  theta(omega, T) = (hbar omega / 2) coth(hbar omega / 2 kT)        eq. (1)
//  kappa_P(omega, T): the solution of eq. (10) with eq. (11) that is
//    completely monotone in omega^2, written as a Laplace integral.
//    With kT = hbar = 1, X = omega:
//      kappa_P / kT = 1 + X^2 int_0^inf e^{-tau X^2} (Th_nu / Th_s - 1) dtau
//      Th_nu(tau) = sum_n exp(-4 pi^2 n^2 tau / P)       (Matsubara sum of coth)
//      Th_s(tau)  = sum_k exp(-4 P sin^2(pi k / P) tau)  (ring normal modes, eq. 11)
//    evaluated with the exp-sinh substitution tau = exp(t - e^-t) and the
//    trapezoid rule (double-exponential decay at both ends).
//  taps: h_k, k = -Nf .. Nf-1, the 2Nf-point inverse DFT of sqrt(S) sampled
//    at omega_j = pi j / (Nf dt) and extended evenly, so the noise spectrum
//    equals S exactly at the grid points (eq. 7 / eq. 12 after the O-step
//    scaling sqrt((1 - c1^2)/m)).
#include <cmath>
#include <vector>

namespace qtb {

namespace {
constexpr double kPi = 3.141592653589793238462643383;

double theta_red(double x)  // theta / kT as a function of x = hbar |omega| / kT
{
    x = std::fabs(x);
    if (x < 1e-4) {
        const double x2 = x * x;
        return 1.0 + x2 / 12.0 - x2 * x2 / 720.0;
    }
    return 0.5 * x / std::tanh(0.5 * x);
}

double theta_nu(double tau, int P)
{
    const double a = 4.0 * kPi * kPi * tau / P;
    if (a > 2.0) {
        double s = 0.0;
        for (int n = 12; n >= 1; --n) s += std::exp(-a * n * n);
        return 1.0 + 2.0 * s;
    }
    double s = 0.0;
    for (int m = 12; m >= 1; --m) s += std::exp(-kPi * kPi * m * m / a);
    return std::sqrt(kPi / a) * (1.0 + 2.0 * s);
}

double theta_s(double tau, int P)
{
    double s = 0.0;
    for (int k = P - 1; k >= 0; --k) {
        const double sn = std::sin(kPi * k / P);
        s += std::exp(-4.0 * P * sn * sn * tau);
    }
    return s;
}

struct KappaGrid {
    int P = 0;
    double h = 0.0;
    std::vector<double> tau, wg;  // nodes and weights (including Jacobian, g)
};

KappaGrid make_grid(int P)
{
    KappaGrid G;
    G.P = P;
    G.h = 1.0 / 48.0;
    for (double t = -5.5; t <= 7.0; t += G.h) {
        const double et = std::exp(-t);
        const double tau = std::exp(t - et);
        const double jac = tau * (1.0 + et);
        const double g = theta_nu(tau, P) / theta_s(tau, P) - 1.0;
        G.tau.push_back(tau);
        G.wg.push_back(jac * g * G.h);
    }
    return G;
}

double kappa_red(const KappaGrid& G, double X)  // kappa_P / kT at X = hbar omega / kT
{
    if (X == 0.0) return 1.0;
    const double X2 = X * X;
    double s = 0.0;
    for (size_t q = 0; q < G.tau.size(); ++q) {
        const double e = std::exp(-G.tau[q] * X2);
        if (e == 0.0) break;
        s += e * G.wg[q];
    }
    return 1.0 + X2 * s;
}
}  // namespace

double design_theta(double omega, double T, double hbar, double kB)
{
    const double kT = kB * T;
    return kT * theta_red(hbar * omega / kT);
}

double design_kappa(double omega, double T, int P, double hbar, double kB)
{
    const double kT = kB * T;
    if (P == 1) return design_theta(omega, T, hbar, kB);
    const KappaGrid G = make_grid(P);
    return kT * kappa_red(G, hbar * std::fabs(omega) / kT);
}

// The target spectrum S_j of the random force on the grid
// omega_j = pi j / (Nf dt), j = 0 .. Nf (2 Nf = two_nf): k_BT (kind 0),
// theta (eq. 1, kind 1) or kappa_P (eq. 10-12, kind 2).
void design_spectrum(int kind, double T, int P, double dt, int two_nf, double hbar, double kB,
                     double* S)
{
    const int Nf = two_nf / 2;
    const double kT = kB * T;
    KappaGrid G;
    if (kind == 2 && P > 1) G = make_grid(P);
    for (int j = 0; j <= Nf; ++j) {
        const double w = kPi * j / (Nf * dt);
        const double X = hbar * w / kT;
        S[j] = kind == 0 ? kT : ((kind == 2 && P > 1) ? kT * kappa_red(G, X) : kT * theta_red(X));
    }
}

// kind: 0 white (kT), 1 theta, 2 kappa_P.  out[k + Nf], k = -Nf .. Nf-1.
void design_taps(int kind, double T, int P, double dt, int two_nf, double hbar, double kB,
                 double* out)
{
    const int Nf = two_nf / 2;
    const double kT = kB * T;
    if (kind == 0) {
        for (int x = 0; x < two_nf; ++x) out[x] = 0.0;
        out[Nf] = std::sqrt(kT);
        return;
    }
    std::vector<double> H(Nf + 1);
    design_spectrum(kind, T, P, dt, two_nf, hbar, kB, H.data());
    for (int j = 0; j <= Nf; ++j) H[j] = std::sqrt(H[j]);
    std::vector<double> ctab(two_nf);
    for (int m = 0; m < two_nf; ++m) ctab[m] = std::cos(kPi * m / Nf);
    for (int k = -Nf; k < Nf; ++k) {
        double acc = 0.0;
        for (int j = 0; j < two_nf; ++j) {
            const int jj = j <= Nf ? j : two_nf - j;
            long long idx = ((long long)j * k) % two_nf;
            if (idx < 0) idx += two_nf;
            acc += H[jj] * ctab[idx];
        }
        out[k + Nf] = acc / two_nf;
    }
}

}  // namespace qtb
