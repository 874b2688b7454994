/*
 * qtb_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Loops are written in the order the paper states the method, with
 * no blocking or fusion.  OpenMP only splits independent atoms.
 *
 * Paper: Dammak et al., arXiv:1905.02521.
 *   eq. (1)  theta(omega,T)                       -> orc_theta
 *   eq. (3)  ring-polymer effective potential     -> spring terms, orc_sim_hamiltonian
 *   eq. (4)  PIMD equations of motion             -> orc_sim_run (B/A steps)
 *   eq. (5)  primitive energy estimator           -> orc_sim_observe
 *   eq. (6)-(7) noise PSD 2 m gamma theta         -> orc_taps (kind 1), O step
 *   eq. (8)  QTB Langevin equation                -> orc_sim_run (O step)
 *   eq. (10)-(12) kappa_P and its PSD             -> orc_kappa, orc_taps (kind 2)
 *   Sec. 2.3 orthogonal normal-mode transform     -> orc_nm_matrix
 */
#include "qtb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846

/* ------------------------------------------------------------------ eq. (1) */
double orc_theta(double omega, double T, const orc_units *u)
{
    double w = fabs(omega);
    double kT = u->kB * T;
    if (w == 0.0) return kT; /* limit of eq. (1) at omega -> 0 */
    double x = u->hbar * w / kT;
    /* hbar w [1/2 + 1/(exp(x) - 1)] */
    return u->hbar * w * (0.5 + 1.0 / expm1(x));
}

/* ------------------------------------------------------- eq. (10)-(11) */
/*
 * Reading of eq. (10): write G(x) = kappa_P(sqrt x)/x and y = omega^2/P.  With
 * eq. (11), eq. (10) reads sum_k G(y + s_k) = theta(sqrt(P y))/y, where
 * s_k = 4 omega_P^2 sin^2(k pi/P).  The Matsubara sum of coth turns the right
 * side into kT sum_n 1/(y + nu_n^2/P), nu_n = 2 pi n kT/hbar.  Taking G as a
 * Laplace transform G(x) = int_0^inf exp(-t x) phi(t) dt gives
 * phi = kT Theta_nu / Theta_s with Theta_nu(t) = sum_n exp(-t nu_n^2/P) and
 * Theta_s(t) = sum_k exp(-t s_k).  In units where kT = hbar = 1
 * (tau = t (kT/hbar)^2, X = hbar omega/kT):
 *   kappa_P/kT = 1 + X^2 int_0^inf exp(-tau X^2) [Theta_nu/Theta_s - 1] dtau.
 */
static double theta_nu_sum(double tau, int P)
{
    double a = 4.0 * PI_D * PI_D * tau / P; /* sum_n exp(-a n^2) */
    double s;
    if (a >= 1.0) {
        s = 1.0;
        for (int n = 1; n < 64; ++n) {
            double t = exp(-a * n * n);
            s += 2.0 * t;
            if (t < 1e-20) break;
        }
    } else {
        /* Poisson summation: sqrt(pi/a) sum_m exp(-pi^2 m^2 / a) */
        double r = 1.0;
        for (int m = 1; m < 64; ++m) {
            double t = exp(-PI_D * PI_D * m * m / a);
            r += 2.0 * t;
            if (t < 1e-20) break;
        }
        s = sqrt(PI_D / a) * r;
    }
    return s;
}

static double theta_s_sum(double tau, int P)
{
    double s = 0.0;
    for (int k = 0; k < P; ++k) {
        double sn = sin(PI_D * k / P);
        s += exp(-4.0 * P * sn * sn * tau);
    }
    return s;
}

double orc_kappa(double omega, double T, int P, const orc_units *u, double h_quad)
{
    double kT = u->kB * T;
    if (P == 1) return orc_theta(omega, T, u);
    double X = u->hbar * fabs(omega) / kT;
    if (X == 0.0) return kT;
    double h = (h_quad > 0.0) ? h_quad : 1.0 / 32.0;
    /* trapezoid in s = ln tau on [-80, 12]; both ends decay exponentially */
    double smin = -80.0, smax = 12.0;
    int n = (int)ceil((smax - smin) / h);
    double sum = 0.0;
    for (int i = 0; i <= n; ++i) {
        double s = smin + i * h;
        double tau = exp(s);
        double e = exp(-tau * X * X);
        if (e == 0.0 && s > 0.0) break;
        double g = theta_nu_sum(tau, P) / theta_s_sum(tau, P) - 1.0;
        double w = (i == 0 || i == n) ? 0.5 : 1.0;
        sum += w * e * g * tau;
    }
    return kT * (1.0 + X * X * sum * h);
}

/* -------------------------------------------------------- FIR taps (eq. 7, 12) */
/*
 * The noise zeta_n = sum_k h_k w_{n-k} has discrete spectrum |H(phi)|^2,
 * phi = omega dt.  The taps are the 2Nf-point inverse DFT of H_j = sqrt(S_j)
 * on omega_j = pi j/(Nf dt), j = 0..Nf, extended evenly, so that the realised
 * spectrum equals S exactly on the grid.  With the O step amplitude
 * sqrt((1-c1^2)/m) this gives the random-force PSD 2 m gamma S of eq. (7)/(12).
 */
int orc_taps(int kind, double T, int P, double dt, int two_nf,
             const orc_units *u, double *h_out)
{
    if (two_nf < 2 || (two_nf & 1)) return 1;
    int Nf = two_nf / 2;
    double kT = u->kB * T;
    if (kind == 0) {
        for (int i = 0; i < two_nf; ++i) h_out[i] = 0.0;
        h_out[Nf] = sqrt(kT);
        return 0;
    }
    double *H = (double *)malloc(sizeof(double) * (Nf + 1));
    for (int j = 0; j <= Nf; ++j) {
        double w = PI_D * j / (Nf * dt);
        double S = (kind == 1) ? orc_theta(w, T, u) : orc_kappa(w, T, P, u, 0.0);
        H[j] = sqrt(S);
    }
    for (int k = -Nf; k < Nf; ++k) {
        double acc = H[0];
        for (int j = 1; j < Nf; ++j) acc += 2.0 * H[j] * cos(PI_D * j * k / Nf);
        acc += H[Nf] * cos(PI_D * k);
        h_out[k + Nf] = acc / (2.0 * Nf);
    }
    free(H);
    return 0;
}

/* --------------------------------------------------------------- Philox4x32-10 */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------ Gaussian transform spec */
/*
 * Natural log of u in (0,1), written with +, -, *, / and fma only:
 * u = 2^e f, f in (sqrt(1/2), sqrt(2)];  ln f = 2 atanh(s), s = (f-1)/(f+1),
 * atanh(s) = s (1 + z/3 + z^2/5 + ... + z^11/23), z = s^2 (|s| <= 0.1716).
 * ln 2 is split in fdlibm's hi/lo pair so that e * ln2_hi is exact.
 */
static double u64_as_double(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t double_as_u64(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }

double orc_log_spec(double u)
{
    uint64_t bits = double_as_u64(u);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    double f = u64_as_double((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (f > 1.4142135623730951) { f = f * 0.5; e = e + 1; }
    double s = (f - 1.0) / (f + 1.0);
    double z = s * s;
    double q = 1.0 / 23.0;
    q = fma(q, z, 1.0 / 21.0);
    q = fma(q, z, 1.0 / 19.0);
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    q = fma(q, z, 1.0);
    double t = s * q;
    double lnf = t + t;
    double de = (double)e;
    double hi = de * 6.93147180369123816490e-01;
    double lo = fma(de, 1.90821492927058770002e-10, lnf);
    return hi + lo;
}

/*
 * cos(2 pi u) for u = N / 2^53 with N odd, N < 2^53.  Quadrant split done on
 * the integer: q = round(4u), r = 4u - q in [-1/2, 1/2] exactly; x = r pi/2
 * with pi/2 as a hi/lo pair; cos x and sin x by their Taylor series to
 * z^9 (|x| <= pi/4); then cos(q pi/2 + x) by quadrant.
 */
double orc_cos2pi_spec(uint64_t N)
{
    uint64_t q = (N + (1ull << 50)) >> 51;
    int64_t rem = (int64_t)N - (int64_t)(q << 51);
    double r = (double)rem * 4.4408920985006262e-16; /* 2^-51 */
    double xh = r * 1.5707963267948966;
    double x = fma(r, 6.123233995736766e-17, xh);
    double z = x * x;
    /* cos x = 1 + z*(-1/2! + z*(1/4! - ...)) */
    double c = -1.0 / 6402373705728000.0;   /* -1/18! */
    c = fma(c, z, 1.0 / 20922789888000.0);  /* 1/16! */
    c = fma(c, z, -1.0 / 87178291200.0);    /* -1/14! */
    c = fma(c, z, 1.0 / 479001600.0);       /* 1/12! */
    c = fma(c, z, -1.0 / 3628800.0);        /* -1/10! */
    c = fma(c, z, 1.0 / 40320.0);           /* 1/8! */
    c = fma(c, z, -1.0 / 720.0);            /* -1/6! */
    c = fma(c, z, 1.0 / 24.0);              /* 1/4! */
    c = fma(c, z, -1.0 / 2.0);              /* -1/2! */
    double cosx = fma(c, z, 1.0);
    /* sin x = x + x z (-1/3! + z (1/5! - ...)) */
    double p = -1.0 / 121645100408832000.0; /* -1/19! */
    p = fma(p, z, 1.0 / 355687428096000.0); /* 1/17! */
    p = fma(p, z, -1.0 / 1307674368000.0);  /* -1/15! */
    p = fma(p, z, 1.0 / 6227020800.0);      /* 1/13! */
    p = fma(p, z, -1.0 / 39916800.0);       /* -1/11! */
    p = fma(p, z, 1.0 / 362880.0);          /* 1/9! */
    p = fma(p, z, -1.0 / 5040.0);           /* -1/7! */
    p = fma(p, z, 1.0 / 120.0);             /* 1/5! */
    p = fma(p, z, -1.0 / 6.0);              /* -1/3! */
    double xz = x * z;
    double sinx = fma(xz, p, x);
    switch (q & 3u) {
    case 0: return cosx;
    case 1: return -sinx;
    case 2: return -cosx;
    default: return sinx;
    }
}

/*
 * w = sqrt(-2 ln u1) cos(2 pi u2).  The paper only asks for normally
 * distributed numbers (the a_j, b_j of eq. 9); the generator is our reading.
 * Counter = (n + 2^40 as two words, d, 16*stream + tag), key = seed words.
 * Uniforms: m = (x0>>6)*2^26 + (x1>>6) (52 bits), u = (2m+1) 2^-53.
 */
double orc_gauss(uint64_t seed, int64_t n, uint32_t d, uint32_t stream, uint32_t tag)
{
    uint64_t c = (uint64_t)(n + ((int64_t)1 << 40));
    uint32_t ctr[4] = {(uint32_t)c, (uint32_t)(c >> 32), d, stream * 16u + tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    uint64_t m1 = ((uint64_t)(x[0] >> 6) << 26) | (uint64_t)(x[1] >> 6);
    uint64_t m2 = ((uint64_t)(x[2] >> 6) << 26) | (uint64_t)(x[3] >> 6);
    double u1 = (double)(2 * m1 + 1) * 1.1102230246251565e-16; /* 2^-53 */
    double a = -2.0 * orc_log_spec(u1);
    double rad = sqrt(a);
    return rad * orc_cos2pi_spec(2 * m2 + 1);
}

void orc_gauss_fill(uint64_t seed, int64_t n0, int64_t n_rows, uint32_t d0, uint32_t n_dof,
                    uint32_t stream, uint32_t tag, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n_rows; ++r)
        for (uint32_t j = 0; j < n_dof; ++j)
            out[r * n_dof + j] = orc_gauss(seed, n0 + r, d0 + j, stream, tag);
}

double orc_zeta(const double *h, int two_nf, uint64_t seed, uint32_t stream,
                int64_t n, uint32_t d)
{
    int Nf = two_nf / 2;
    double acc = 0.0;
    for (int k = -Nf; k < Nf; ++k)
        acc += h[k + Nf] * orc_gauss(seed, n - k, d, stream, 0);
    return acc;
}

/* --------------------------------------------------------------- potential */
/*
 * Pair potential (not given by the paper; the workload's): Buckingham
 * A exp(-r/rho) - C/r^6 in shifted-force form at r_cut, plus damped shifted
 * force Coulomb (Fennell & Gezelter 2006):
 *   k qi qj [erfc(ar)/r - erfc(a rc)/rc + (erfc(a rc)/rc^2
 *            + 2a/sqrt(pi) exp(-a^2 rc^2)/rc)(r - rc)]
 * and the self term -(erfc(a rc)/(2 rc) + a/sqrt(pi)) k sum q_i^2.
 * pair_eval returns V(r) and writes -dV/dr.
 */
static double buck_V(double A, double rho, double C, double r)
{
    double v = 0.0;
    if (A != 0.0) v += A * exp(-r / rho);
    if (C != 0.0) v -= C / (r * r * r * r * r * r);
    return v;
}
static double buck_dV(double A, double rho, double C, double r)
{
    double d = 0.0;
    if (A != 0.0) d -= (A / rho) * exp(-r / rho);
    if (C != 0.0) d += 6.0 * C / (r * r * r * r * r * r * r);
    return d;
}

static double pair_eval(const orc_pot *p, const orc_units *u, int a, int b, double r,
                        double *fmag)
{
    int ab = a * p->n_species + b;
    double A = p->buck_A[ab], rho = p->buck_rho[ab], C = p->buck_C[ab];
    double rc = p->r_cut, al = p->dsf_alpha;
    double V = buck_V(A, rho, C, r) - buck_V(A, rho, C, rc) - (r - rc) * buck_dV(A, rho, C, rc);
    double F = -buck_dV(A, rho, C, r) + buck_dV(A, rho, C, rc);
    double qq = u->coulomb_k * p->charge[a] * p->charge[b];
    if (qq != 0.0) {
        double erc = erfc(al * rc);
        double grc = 2.0 * al / sqrt(PI_D) * exp(-al * al * rc * rc);
        double shiftF = erc / (rc * rc) + grc / rc;
        double er = erfc(al * r);
        double gr = 2.0 * al / sqrt(PI_D) * exp(-al * al * r * r);
        V += qq * (er / r - erc / rc + shiftF * (r - rc));
        F += qq * (er / (r * r) + gr / r - shiftF);
    }
    *fmag = F;
    return V;
}

static double self_energy(const orc_pot *p, const orc_units *u, int N, const int32_t *sp)
{
    double rc = p->r_cut, al = p->dsf_alpha;
    double q2 = 0.0;
    for (int i = 0; i < N; ++i) q2 += p->charge[sp[i]] * p->charge[sp[i]];
    return -(erfc(al * rc) / (2.0 * rc) + al / sqrt(PI_D)) * u->coulomb_k * q2;
}

double orc_pair_bruteforce(const orc_pot *pot, const orc_units *u, int N,
                           const double box[3], const int32_t *species,
                           const double *pos, double *f, double *virial)
{
    double rc = pot->r_cut;
    int m[3];
    for (int d = 0; d < 3; ++d) m[d] = (int)floor(rc / box[d] + 0.5) + 1;
    double *ei = (double *)calloc(N, sizeof(double));
    double *vi = (double *)calloc((size_t)9 * N, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < N; ++i) {
        double fx = 0, fy = 0, fz = 0, e = 0;
        double vir[9] = {0};
        for (int j = 0; j < N; ++j) {
            double d0[3];
            for (int d = 0; d < 3; ++d) {
                double x = pos[d * N + i] - pos[d * N + j];
                d0[d] = x - box[d] * nearbyint(x / box[d]);
            }
            for (int nx = -m[0]; nx <= m[0]; ++nx)
                for (int ny = -m[1]; ny <= m[1]; ++ny)
                    for (int nz = -m[2]; nz <= m[2]; ++nz) {
                        double dx = d0[0] + nx * box[0];
                        double dy = d0[1] + ny * box[1];
                        double dz = d0[2] + nz * box[2];
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 >= rc * rc) continue;
                        if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
                        double r = sqrt(r2), F;
                        double V = pair_eval(pot, u, species[i], species[j], r, &F);
                        e += 0.5 * V;
                        fx += F * dx / r; fy += F * dy / r; fz += F * dz / r;
                        double dd[3] = {dx, dy, dz};
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) vir[3 * a + b] += 0.5 * dd[a] * F * dd[b] / r;
                    }
        }
        f[i] = fx; f[N + i] = fy; f[2 * N + i] = fz;
        ei[i] = e;
        for (int k = 0; k < 9; ++k) vi[9 * i + k] = vir[k];
    }
    double E = 0.0;
    for (int i = 0; i < N; ++i) E += ei[i];
    if (virial) {
        for (int k = 0; k < 9; ++k) virial[k] = 0.0;
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < 9; ++k) virial[k] += vi[9 * i + k];
    }
    free(ei); free(vi);
    return E + self_energy(pot, u, N, species);
}

/* ------------------------------------------------------------ normal modes */
/* Orthonormal real DFT: columns are the ring polymer's normal modes. */
void orc_nm_matrix(int P, double *C)
{
    for (int s = 0; s < P; ++s)
        for (int k = 0; k < P; ++k) {
            double v;
            if (k == 0) v = 1.0 / sqrt((double)P);
            else if (2 * k < P) v = sqrt(2.0 / P) * cos(2.0 * PI_D * s * k / P);
            else if (2 * k == P) v = ((s & 1) ? -1.0 : 1.0) / sqrt((double)P);
            else v = sqrt(2.0 / P) * sin(2.0 * PI_D * s * k / P);
            C[s * P + k] = v;
        }
}

/* -------------------------------------------------------------- simulation */
struct orc_sim {
    orc_pot pot;
    orc_units u;
    int N, P, dims, D;
    double box[3];
    int32_t *species;
    double *homega;
    double T, gamma, dt;
    uint64_t seed;
    uint32_t stream;
    int noise_kind, two_nf;
    double *taps;
    double *r, *v, *f, *r0; /* [P][dims][N] */
    double *epot;           /* [P] physical potential energy of each bead */
    double *wpair;          /* [P] pair virial of each bead: sum over pairs of F(r) r */
    int64_t step;
    double *C, *wk;         /* NM matrix, free-ring frequencies */
    double *wring;          /* [two_nf][D], row m lives in slot m mod two_nf */
    /* neighbour list (pair potential): full list built from bead centroids */
    double *rref;           /* [3][N] */
    double nb_dev;          /* largest bead-to-centroid distance at the build */
    int *nb_start, *nb_j, nb_cap;
    double *nb_shift;       /* [3 * entries] */
    int nthreads;
    /* isotropic barostat (pair kind): 1 stochastic cell rescaling, 2 Langevin
     * piston; npt_pe is the piston momentum */
    int npt, nb_force;
    double npt_P0, npt_tau, npt_beta;
    double npt_W, npt_gp, npt_pe;
    /* scalings the last barostat update left for the next step: velocities
     * at its start (sv1) and after its closing kick (sv2), positions and box
     * before its forces (sr); between steps the box is the one the positions
     * were taken in */
    double npt_sr, npt_sv1, npt_sv2;
};

static int64_t pmod(int64_t a, int64_t m) { int64_t r = a % m; return r < 0 ? r + m : r; }

/*
 * Full list from the bead centroids.  A bead may sit up to dev from its
 * centroid, so the list radius is r_cut + skin + 2 dev: any pair that is not
 * listed then stays beyond r_cut while every bead remains within
 * skin/2 + dev of its reference (the rebuild test below).
 */
static void nlist_build(orc_sim *s)
{
    s->nb_force = 0;
    int N = s->N, P = s->P;
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < N; ++i) {
            double c = 0.0;
            for (int b = 0; b < P; ++b) c += s->r[(b * 3 + d) * N + i];
            s->rref[d * N + i] = c / P;
        }
    double dev2 = 0.0;
    for (int b = 0; b < P; ++b)
        for (int i = 0; i < N; ++i) {
            double x2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                double x = s->r[(b * 3 + d) * N + i] - s->rref[d * N + i];
                x2 += x * x;
            }
            if (x2 > dev2) dev2 = x2;
        }
    s->nb_dev = sqrt(dev2);
    double R = s->pot.r_cut + s->pot.skin + 2.0 * s->nb_dev;
    int m[3];
    for (int d = 0; d < 3; ++d) m[d] = (int)floor(R / s->box[d] + 0.5) + 1;
    int cnt = 0;
    for (int i = 0; i < N; ++i) {
        s->nb_start[i] = cnt;
        for (int j = 0; j < N; ++j) {
            double d0[3], n0[3];
            for (int d = 0; d < 3; ++d) {
                double x = s->rref[d * N + i] - s->rref[d * N + j];
                n0[d] = nearbyint(x / s->box[d]);
                d0[d] = x - s->box[d] * n0[d];
            }
            for (int nx = -m[0]; nx <= m[0]; ++nx)
                for (int ny = -m[1]; ny <= m[1]; ++ny)
                    for (int nz = -m[2]; nz <= m[2]; ++nz) {
                        double S[3] = {(n0[0] - nx) * s->box[0], (n0[1] - ny) * s->box[1],
                                       (n0[2] - nz) * s->box[2]};
                        double dx = d0[0] + nx * s->box[0], dy = d0[1] + ny * s->box[1],
                               dz = d0[2] + nz * s->box[2];
                        if (dx * dx + dy * dy + dz * dz >= R * R) continue;
                        if (j == i && S[0] == 0.0 && S[1] == 0.0 && S[2] == 0.0) continue;
                        if (cnt >= s->nb_cap) {
                            s->nb_cap *= 2;
                            s->nb_j = (int *)realloc(s->nb_j, sizeof(int) * s->nb_cap);
                            s->nb_shift = (double *)realloc(s->nb_shift, sizeof(double) * 3 * s->nb_cap);
                        }
                        s->nb_j[cnt] = j;
                        s->nb_shift[3 * cnt + 0] = S[0];
                        s->nb_shift[3 * cnt + 1] = S[1];
                        s->nb_shift[3 * cnt + 2] = S[2];
                        ++cnt;
                    }
        }
    }
    s->nb_start[N] = cnt;
}

static int nlist_stale(const orc_sim *s)
{
    int N = s->N;
    if (s->nb_force) return 1; /* the box changed */
    double lim = 0.5 * s->pot.skin + s->nb_dev;
    for (int b = 0; b < s->P; ++b)
        for (int i = 0; i < N; ++i) {
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                double x = s->r[(b * 3 + d) * N + i] - s->rref[d * N + i];
                d2 += x * x;
            }
            if (d2 > lim * lim) return 1;
        }
    return 0;
}

/* On-site potential of one dof and its force F = -dV/dx (the kinds above). */
static double onsite_eval(const orc_pot *p, int sp, double x, double *F)
{
    double V0 = p->os_V0[sp], d = p->os_d[sp];
    if (p->kind == ORC_POT_MORSE) {
        double e = exp(-x / d);
        *F = -2.0 * V0 * (1.0 - e) * e / d;
        return V0 * (1.0 - e) * (1.0 - e);
    }
    double y = x / d, w = y * y - 1.0;  /* double well */
    *F = -4.0 * V0 * w * y / d;
    return V0 * w * w;
}

/* f = -grad V(r^(s)) for every bead s (physical force, no 1/P); epot[s] = V. */
static void compute_forces(orc_sim *s)
{
    int N = s->N, P = s->P, dims = s->dims;
    if (s->pot.kind == ORC_POT_HARMONIC) {
        for (int b = 0; b < P; ++b) {
            double e = 0.0;
            for (int d = 0; d < dims; ++d)
                for (int i = 0; i < N; ++i) {
                    double m = s->pot.mass[s->species[i]] * s->u.mass_unit;
                    double k = m * s->homega[i] * s->homega[i];
                    double x = s->r[(b * dims + d) * N + i];
                    s->f[(b * dims + d) * N + i] = -k * x;
                    e += 0.5 * k * x * x;
                }
            s->epot[b] = e;
        }
        return;
    }
    if (s->pot.kind == ORC_POT_MORSE || s->pot.kind == ORC_POT_DOUBLE_WELL) {
        for (int b = 0; b < P; ++b) {
            double e = 0.0;
            for (int d = 0; d < dims; ++d)
                for (int i = 0; i < N; ++i) {
                    double F;
                    double x = s->r[(b * dims + d) * N + i];
                    e += onsite_eval(&s->pot, s->species[i], x, &F);
                    s->f[(b * dims + d) * N + i] = F;
                }
            s->epot[b] = e;
        }
        return;
    }
    if (nlist_stale(s)) nlist_build(s);
    double rc = s->pot.r_cut;
    double eself = self_energy(&s->pot, &s->u, N, s->species);
    double *ei = (double *)malloc(sizeof(double) * N);
    double *wi = (double *)malloc(sizeof(double) * N);
    for (int b = 0; b < P; ++b) {
        const double *x = s->r + (size_t)b * 3 * N;
        double *fo = s->f + (size_t)b * 3 * N;
#pragma omp parallel for schedule(dynamic, 16) num_threads(s->nthreads)
        for (int i = 0; i < N; ++i) {
            double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
            for (int q = s->nb_start[i]; q < s->nb_start[i + 1]; ++q) {
                int j = s->nb_j[q];
                double dx = x[i] - x[j] - s->nb_shift[3 * q + 0];
                double dy = x[N + i] - x[N + j] - s->nb_shift[3 * q + 1];
                double dz = x[2 * N + i] - x[2 * N + j] - s->nb_shift[3 * q + 2];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 >= rc * rc) continue;
                double r = sqrt(r2), F;
                double V = pair_eval(&s->pot, &s->u, s->species[i], s->species[j], r, &F);
                e += 0.5 * V;
                w += 0.5 * F * r; /* each pair is listed from both sides */
                fx += F * dx / r; fy += F * dy / r; fz += F * dz / r;
            }
            fo[i] = fx; fo[N + i] = fy; fo[2 * N + i] = fz;
            ei[i] = e;
            wi[i] = w;
        }
        double E = 0.0, Wp = 0.0;
        for (int i = 0; i < N; ++i) { E += ei[i]; Wp += wi[i]; }
        s->epot[b] = E + eself;
        s->wpair[b] = Wp;
    }
    free(ei);
    free(wi);
}

static void fill_noise_row(orc_sim *s, int64_t m)
{
    double *row = s->wring + (size_t)pmod(m, s->two_nf) * s->D;
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
    for (int d = 0; d < s->D; ++d) row[d] = orc_gauss(s->seed, m, (uint32_t)d, s->stream, 0);
}

orc_sim *orc_sim_new(const orc_pot *pot, const orc_units *u, int N, int P, int dims,
                     const double box[3], const int32_t *species,
                     const double *harm_omega, double T, double gamma, double dt,
                     uint64_t seed, uint32_t stream, int noise_kind, int two_nf,
                     const double *pos0, const double *vel0, int64_t step0,
                     int n_threads)
{
    if (N < 1 || P < 1 || P > 64 || (dims != 1 && dims != 3)) return NULL;
    if (pot->kind == ORC_POT_PAIR && dims != 3) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->pot = *pot; s->u = *u;
    s->N = N; s->P = P; s->dims = dims; s->D = dims * N * P;
    for (int d = 0; d < 3; ++d) s->box[d] = box ? box[d] : 0.0;
    s->species = (int32_t *)malloc(sizeof(int32_t) * N);
    memcpy(s->species, species, sizeof(int32_t) * N);
    s->homega = (double *)calloc(N, sizeof(double));
    if (harm_omega) memcpy(s->homega, harm_omega, sizeof(double) * N);
    s->T = T; s->gamma = gamma; s->dt = dt; s->seed = seed; s->stream = stream;
    s->noise_kind = noise_kind;
    s->two_nf = (noise_kind == 0) ? 2 : two_nf;
    s->nthreads = n_threads > 0 ? n_threads : 1;
    s->taps = (double *)malloc(sizeof(double) * s->two_nf);
    if (orc_taps(noise_kind, T, P, dt, s->two_nf, u, s->taps)) { orc_sim_free(s); return NULL; }
    size_t nst = (size_t)P * dims * N;
    s->r = (double *)malloc(sizeof(double) * nst);
    s->v = (double *)malloc(sizeof(double) * nst);
    s->f = (double *)calloc(nst, sizeof(double));
    s->r0 = (double *)malloc(sizeof(double) * nst);
    memcpy(s->r, pos0, sizeof(double) * nst);
    memcpy(s->r0, pos0, sizeof(double) * nst);
    if (vel0) memcpy(s->v, vel0, sizeof(double) * nst);
    else memset(s->v, 0, sizeof(double) * nst);
    s->epot = (double *)calloc(P, sizeof(double));
    s->wpair = (double *)calloc(P, sizeof(double));
    s->step = step0;
    s->C = (double *)malloc(sizeof(double) * P * P);
    orc_nm_matrix(P, s->C);
    s->wk = (double *)malloc(sizeof(double) * P);
    double wP = sqrt((double)P) * u->kB * T / u->hbar; /* omega_P = sqrt(P)/(beta hbar) */
    for (int k = 0; k < P; ++k) s->wk[k] = 2.0 * wP * sin(PI_D * k / P);
    s->wring = (double *)malloc(sizeof(double) * (size_t)s->two_nf * s->D);
    int Nf = s->two_nf / 2;
    for (int64_t m = step0 - Nf + 1; m <= step0 + Nf; ++m) fill_noise_row(s, m);
    if (pot->kind == ORC_POT_PAIR) {
        s->rref = (double *)malloc(sizeof(double) * 3 * N);
        s->nb_start = (int *)malloc(sizeof(int) * (N + 1));
        s->nb_cap = 64 * N;
        s->nb_j = (int *)malloc(sizeof(int) * s->nb_cap);
        s->nb_shift = (double *)malloc(sizeof(double) * 3 * s->nb_cap);
        nlist_build(s);
    }
    compute_forces(s);
    return s;
}

void orc_sim_free(orc_sim *s)
{
    if (!s) return;
    free(s->species); free(s->homega); free(s->taps);
    free(s->r); free(s->v); free(s->f); free(s->r0); free(s->epot); free(s->wpair);
    free(s->C); free(s->wk); free(s->wring);
    free(s->rref); free(s->nb_start); free(s->nb_j); free(s->nb_shift);
    free(s);
}

/* eq. (5) primitive estimator with instantaneous momenta, plus the centroid
 * virial estimator, kinetic temperature and mean square displacement from the
 * initial positions.  The centroid virial estimator replaces the kinetic
 * energy of the P - 1 internal ring modes by minus half the centroid virial,
 *   E_vir = K_c - (1/2P) sum_s (r_s - r_c) . F_s + (1/P) sum_s V(r_s),
 * with K_c = sum_i (1/2) m P |v_c,i|^2 the kinetic energy of the centroid
 * (normal mode k = 0) measured from the instantaneous velocities: k_B T / 2
 * per dof under white noise, kappa_P(omega / sqrt(P)) / 2 under the QTB-PIMD
 * noise of eq. (12), so that a harmonic oscillator gives theta exactly by
 * eq. (10).  For the pair potential the pressure by the primitive
 * (thermodynamic) estimator, the volume derivative of the ring-polymer
 * partition function with the instantaneous momenta standing in for
 * N P dims k_B T:  p = (2 K - 2 U_spring + (1/P) sum_s W_s) / (3 V), with
 * W_s = sum over pairs of F(r) r at bead s (P = 1: the virial pressure). */
void orc_sim_observe(orc_sim *s, double *o)
{
    int N = s->N, P = s->P, dims = s->dims;
    double mu = s->u.mass_unit;
    double wP = sqrt((double)P) * s->u.kB * s->T / s->u.hbar;
    double ke = 0.0, spring = 0.0, x2 = 0.0, vir = 0.0, kec = 0.0;
    for (int d = 0; d < dims; ++d)
        for (int i = 0; i < N; ++i) {
            double m = s->pot.mass[s->species[i]] * mu;
            double vc = 0.0;
            for (int b = 0; b < P; ++b) vc += s->v[((size_t)b * dims + d) * N + i];
            vc /= P;
            kec += 0.5 * m * P * vc * vc;
        }
    for (int b = 0; b < P; ++b)
        for (int d = 0; d < dims; ++d)
            for (int i = 0; i < N; ++i) {
                double m = s->pot.mass[s->species[i]] * mu;
                size_t id = ((size_t)b * dims + d) * N + i;
                ke += 0.5 * m * s->v[id] * s->v[id];
                if (P > 1) {
                    size_t nx = ((size_t)((b + 1) % P) * dims + d) * N + i;
                    double dr = s->r[id] - s->r[nx];
                    spring += 0.5 * m * wP * wP * dr * dr;
                }
                double dx0 = s->r[id] - s->r0[id];
                x2 += dx0 * dx0;
                double c = 0.0;
                for (int bb = 0; bb < P; ++bb) c += s->r[((size_t)bb * dims + d) * N + i];
                c /= P;
                vir += (s->r[id] - c) * s->f[id];
            }
    double U = 0.0;
    for (int b = 0; b < P; ++b) U += s->epot[b] / P;
    o[0] = ke;
    o[1] = U;
    o[2] = spring;
    o[3] = ke - spring + U;
    o[4] = kec - vir / (2.0 * P) + U;
    o[5] = 2.0 * ke / (dims * (double)N * P * s->u.kB);
    o[6] = x2 / ((double)dims * N * P);
    o[7] = (double)s->step;
    double W = 0.0;
    for (int b = 0; b < P; ++b) W += s->wpair[b];
    double V = s->box[0] * s->box[1] * s->box[2];
    o[8] = (s->pot.kind == ORC_POT_PAIR && V > 0.0)
               ? (2.0 * ke - 2.0 * spring + W / P) / (3.0 * V) : 0.0;
    o[9] = W;
}

double orc_sim_hamiltonian(orc_sim *s)
{
    double o[ORC_NOBS];
    orc_sim_observe(s, o);
    return o[0] + o[2] + o[1];
}

/*
 * Pressure of the closed step for the isotropic barostats: the volume
 * derivative of the ring polymer's configurational weight under uniform
 * scaling of every bead coordinate, with the instantaneous momenta for the
 * kinetic part (for P = 1 the virial pressure):
 *   p = (2K - 2 U_spring + (1/P) sum_s W_s) / (3V),
 * K the kinetic energy of all beads, U_spring the ring springs of eq. (3)
 * (homogeneous of degree 2 in the bead coordinates), W_s = sum over pairs of
 * F(r) r at bead s.  *kin receives K.
 */
static double npt_pressure(const orc_sim *s, double *kin)
{
    int N = s->N, P = s->P;
    double mu = s->u.mass_unit;
    double wP = sqrt((double)P) * s->u.kB * s->T / s->u.hbar;
    double ke = 0.0, spring = 0.0, W = 0.0;
    for (int b = 0; b < P; ++b)
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < N; ++i) {
                double m = s->pot.mass[s->species[i]] * mu;
                size_t id = ((size_t)b * 3 + d) * N + i;
                ke += 0.5 * m * s->v[id] * s->v[id];
                if (P > 1) {
                    size_t nx = ((size_t)((b + 1) % P) * 3 + d) * N + i;
                    double dr = s->r[id] - s->r[nx];
                    spring += 0.5 * m * wP * wP * dr * dr;
                }
            }
    for (int b = 0; b < P; ++b) W += s->wpair[b];
    double V = s->box[0] * s->box[1] * s->box[2];
    *kin = ke;
    return (2.0 * ke - 2.0 * spring + W / P) / (3.0 * V);
}

/*
 * One barostat update after the step of step index n (after its closing
 * kick), g the unit Gaussian at (step n, dof 0, tag 4).  In the next step
 * every velocity scales by s_v1 at its start and by s_v2 after its closing
 * kick, every bead coordinate by sqrt(s) before and after its A-O-A, and the
 * box by s with them (so its forces are those of the scaled system).
 *
 * Stochastic cell rescaling (after Bernetti and Bussi, J. Chem. Phys. 153,
 * 114107 (2020)), one Euler-Maruyama (Ito) step of eps = ln V:
 *   d eps = -(beta_T / tau_p) (P0 - p) dt + sqrt(2 k_B T beta_T dt / (V tau_p)) g,
 *   s = e^{d eps / 3},  s_v1 = 1 / s,  s_v2 = 1.
 * With the diffusion in eps proportional to 1 / V, the Ito drift needs no
 * separate k_B T / V term: the stationary law is V^N e^{-P0 V / k_B T} for an
 * ideal gas (pinned).
 *
 * Langevin piston (the isothermal-isobaric Langevin scheme of Quigley and
 * Probert, J. Chem. Phys. 120, 11432 (2004), isotropic): the strain
 * eps = ln(V) / 3 has a momentum p_e of mass W_p, driven by
 *   G = 3V (p - P0) + (3 / N_f) 2K,   N_f = 3 N P,
 * (the Martyna-Tobias-Klein form, whose invariant law for an ideal gas is
 * V^N e^{-P0 V / k_B T}) and thermostatted at T with friction gamma_p:
 *   p_e <- c_p (p_e + dt G / 2) + sqrt((1 - c_p^2) W_p k_B T) g + dt G / 2,
 *   c_p = e^{-gamma_p dt},  v_e = p_e / W_p,
 *   s = e^{dt v_e},  s_v1 = s_v2 = e^{-(1 + 3 / N_f) dt v_e / 2},
 * a symmetric splitting around the particle step (kicks of p_e between
 * steps, the strain velocity's drag on the momenta half before and half
 * after the step, the strain's drift with the positions).  The particle
 * dynamics within a step is that of eq. (4) / (8) with its own thermostat.
 * (The paper cites the Langevin barostat of refs 11-12 for its
 * constant-pressure runs without giving its equations; this is the reading.)
 */
static void barostat_step(orc_sim *s, int64_t n)
{
    int N = s->N, P = s->P;
    double kT = s->u.kB * s->T;
    double ke;
    double p = npt_pressure(s, &ke);
    double V = s->box[0] * s->box[1] * s->box[2];
    double g = orc_gauss(s->seed, n, 0, s->stream, 4);
    double sc, sv1, sv2;
    if (s->npt == 1) {
        double deps = -(s->npt_beta / s->npt_tau) * (s->npt_P0 - p) * s->dt +
                      sqrt(2.0 * kT * s->npt_beta * s->dt / (V * s->npt_tau)) * g;
        sc = exp(deps / 3.0);
        sv1 = 1.0 / sc;
        sv2 = 1.0;
    } else {
        double Nf = 3.0 * N * P;
        double G = 3.0 * V * (p - s->npt_P0) + (3.0 / Nf) * 2.0 * ke;
        double cp = exp(-s->npt_gp * s->dt);
        double pe = s->npt_pe + 0.5 * s->dt * G;
        pe = cp * pe + sqrt((1.0 - cp * cp) * s->npt_W * kT) * g;
        pe += 0.5 * s->dt * G;
        s->npt_pe = pe;
        double ve = pe / s->npt_W;
        sc = exp(s->dt * ve);
        sv1 = sv2 = exp(-(1.0 + 3.0 / Nf) * 0.5 * s->dt * ve);
    }
    s->npt_sr = sc;
    s->npt_sv1 = sv1;
    s->npt_sv2 = sv2;
}

/* Velocity scaling of the step (start: sv1; after the closing kick: sv2). */
static void barostat_scale_v(orc_sim *s, double f)
{
    size_t n = (size_t)3 * s->N * s->P;
    for (size_t q = 0; q < n; ++q) s->v[q] *= f;
}

/* After the step's update (which scaled the positions, half before and half
 * after its A-O-A): the box scales with them, and the list follows the new
 * box at the force pass. */
static void barostat_scale_r(orc_sim *s)
{
    for (int d = 0; d < 3; ++d) s->box[d] *= s->npt_sr;
    s->npt_sr = 1.0;
    s->nb_force = 1;
}

int orc_sim_set_barostat(orc_sim *s, double P0, double tau_p, double beta_T)
{
    if (s->pot.kind != ORC_POT_PAIR || s->dims != 3 || !(tau_p > 0.0) || !(beta_T > 0.0)) return 1;
    s->npt = 1;
    s->npt_P0 = P0;
    s->npt_tau = tau_p;
    s->npt_beta = beta_T;
    s->npt_sr = s->npt_sv1 = s->npt_sv2 = 1.0;
    return 0;
}

/* Piston mass W_p = (N_f + 3) k_B T tau_p^2 (tau_p the piston's time scale),
 * friction gamma_p; the piston starts at rest. */
int orc_sim_set_piston(orc_sim *s, double P0, double tau_p, double gamma_p)
{
    if (s->pot.kind != ORC_POT_PAIR || s->dims != 3 || !(tau_p > 0.0) || !(gamma_p >= 0.0) ||
        !(s->T > 0.0))
        return 1;
    s->npt = 2;
    s->npt_P0 = P0;
    s->npt_tau = tau_p;
    s->npt_gp = gamma_p;
    s->npt_W = (3.0 * s->N * s->P + 3.0) * s->u.kB * s->T * tau_p * tau_p;
    s->npt_pe = 0.0;
    s->npt_sr = s->npt_sv1 = s->npt_sv2 = 1.0;
    return 0;
}

double orc_sim_piston_momentum(const orc_sim *s) { return s->npt_pe; }

void orc_sim_barostat_state(orc_sim *s, double *get, const double *set)
{
    if (get) {
        get[0] = s->npt_pe; get[1] = s->npt_sr; get[2] = s->npt_sv1; get[3] = s->npt_sv2;
    }
    if (set) {
        s->npt_pe = set[0]; s->npt_sr = set[1]; s->npt_sv1 = set[2]; s->npt_sv2 = set[3];
    }
}

void orc_sim_box(const orc_sim *s, double *box)
{
    for (int d = 0; d < 3; ++d) box[d] = s->box[d];
}

/*
 * One step = B(dt/2) -> normal modes -> A(dt/2) -> O(dt) -> A(dt/2) ->
 * back to beads -> forces -> B(dt/2).  B uses the bead force -(1/P) grad V
 * of eq. (4) with bead mass m; A integrates the ring springs of eq. (3)-(4)
 * exactly in normal modes (frequencies 2 omega_P sin(k pi/P)); O is the
 * Langevin friction of eq. (8) with the coloured noise of eq. (7)/(12),
 * applied to the normal modes as Sec. 2.3 describes.
 */
int orc_sim_run(orc_sim *s, int64_t n_steps, int obs_every, double *obs_out)
{
    int N = s->N, P = s->P, dims = s->dims, D = s->D;
    double mu = s->u.mass_unit, dt = s->dt, h = 0.5 * dt;
    double c1 = exp(-s->gamma * dt);
    int Nf = s->two_nf / 2;
    int nobs = 0;
    for (int64_t it = 0; it < n_steps; ++it) {
        int64_t n = s->step;
        const double rh = s->npt ? sqrt(s->npt_sr) : 1.0;
        if (s->npt) barostat_scale_v(s, s->npt_sv1);
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
        for (int i = 0; i < N; ++i) {
            double qq[64], pp[64];
            double m = s->pot.mass[s->species[i]] * mu;
            double sig = sqrt((1.0 - c1 * c1) / m);
            for (int d = 0; d < dims; ++d) {
                /* B */
                for (int b = 0; b < P; ++b) {
                    size_t id = ((size_t)b * dims + d) * N + i;
                    s->v[id] += h * s->f[id] / (P * m);
                }
                /* to normal modes */
                for (int k = 0; k < P; ++k) {
                    double a = 0.0, c = 0.0;
                    for (int b = 0; b < P; ++b) {
                        size_t id = ((size_t)b * dims + d) * N + i;
                        a += s->C[b * P + k] * s->r[id];
                        c += s->C[b * P + k] * s->v[id];
                    }
                    qq[k] = a; pp[k] = c;
                }
                for (int k = 0; k < P; ++k) {
                    /* the barostat's strain: half of the position scaling */
                    if (s->npt) qq[k] *= rh;
                    /* A(dt/2) */
                    double w = s->wk[k];
                    if (k == 0) qq[k] += h * pp[k];
                    else {
                        double cw = cos(w * h), sw = sin(w * h);
                        double q1 = cw * qq[k] + sw / w * pp[k];
                        double p1 = -w * sw * qq[k] + cw * pp[k];
                        qq[k] = q1; pp[k] = p1;
                    }
                    /* O(dt) with zeta_{n, d'} */
                    int dof = ((dims * i + d) * P + k);
                    double z = 0.0;
                    for (int kk = -Nf; kk < Nf; ++kk)
                        z += s->taps[kk + Nf] * s->wring[(size_t)pmod(n - kk, s->two_nf) * D + dof];
                    pp[k] = c1 * pp[k] + sig * z;
                    /* A(dt/2) */
                    if (k == 0) qq[k] += h * pp[k];
                    else {
                        double cw = cos(w * h), sw = sin(w * h);
                        double q1 = cw * qq[k] + sw / w * pp[k];
                        double p1 = -w * sw * qq[k] + cw * pp[k];
                        qq[k] = q1; pp[k] = p1;
                    }
                    if (s->npt) qq[k] *= rh;  /* the other half */
                }
                /* back to beads */
                for (int b = 0; b < P; ++b) {
                    double a = 0.0, c = 0.0;
                    for (int k = 0; k < P; ++k) {
                        a += s->C[b * P + k] * qq[k];
                        c += s->C[b * P + k] * pp[k];
                    }
                    size_t id = ((size_t)b * dims + d) * N + i;
                    s->r[id] = a; s->v[id] = c;
                }
            }
        }
        if (s->npt) barostat_scale_r(s);
        compute_forces(s);
        for (int b = 0; b < P; ++b)
            for (int d = 0; d < dims; ++d)
                for (int i = 0; i < N; ++i) {
                    double m = s->pot.mass[s->species[i]] * mu;
                    size_t id = ((size_t)b * dims + d) * N + i;
                    s->v[id] += h * s->f[id] / (P * m);
                }
        if (s->npt) barostat_scale_v(s, s->npt_sv2);
        s->step = n + 1;
        /* slide the white-noise window: row n+1+Nf replaces row n+1-Nf */
        fill_noise_row(s, n + 1 + Nf);
        if (obs_every > 0 && (s->step % obs_every) == 0 && obs_out) {
            orc_sim_observe(s, obs_out + ORC_NOBS * nobs);
            ++nobs;
        }
        if (s->npt) barostat_step(s, n);
    }
    return nobs;
}

void orc_sim_get(const orc_sim *s, double *pos, double *vel, double *force, int64_t *step)
{
    size_t nst = (size_t)s->P * s->dims * s->N;
    if (pos) memcpy(pos, s->r, sizeof(double) * nst);
    if (vel) memcpy(vel, s->v, sizeof(double) * nst);
    if (force) memcpy(force, s->f, sizeof(double) * nst);
    if (step) *step = s->step;
}

const double *orc_sim_taps(const orc_sim *s, int *two_nf)
{
    if (two_nf) *two_nf = s->two_nf;
    return s->taps;
}
