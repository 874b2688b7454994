/*
 * qtb_oracle.h -- plain FP64 CPU oracle for the QTB / QTB-PIMD integrator step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no source with the GPU library.
 *
 * Paper: Dammak, Hayoun, Brieuc, Geneste, "Nuclear quantum effects in
 * molecular dynamics simulations" (arXiv:1905.02521).  Each function cites the
 * equation it follows.  Units are whatever the caller passes through
 * orc_units (the tests use eV, Angstrom, amu, fs, K, or reduced units).
 */
#ifndef QTB_ORACLE_H
#define QTB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double hbar;      /* energy * time */
    double kB;        /* energy / K */
    double coulomb_k; /* energy * length / e^2 */
    double mass_unit; /* energy per (mass * length^2 / time^2) */
} orc_units;

/* Eq. (1): mean energy of a quantum harmonic oscillator, even in omega. */
double orc_theta(double omega, double T, const orc_units *u);

/* Eq. (10)-(11): bead-modified spectrum kappa_P(omega, T), canonical
 * (completely monotone) solution written as a Laplace integral.  P = 1 gives
 * theta.  h_quad is the trapezoid step in log(tau); pass 0 for the default. */
double orc_kappa(double omega, double T, int P, const orc_units *u, double h_quad);

/* FIR taps from the noise spectrum S (eq. 7 for QTB, eq. 12 for QTB-PIMD,
 * k_B T for white noise).  kind: 0 classical, 1 QTB, 2 QTB-PIMD.
 * h_out[k + Nf], k = -Nf .. Nf-1, two_nf = 2 Nf taps.  Returns 0 on success. */
int orc_taps(int kind, double T, int P, double dt, int two_nf,
             const orc_units *u, double *h_out);

/* Philox4x32-10 counter-based generator (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Unit Gaussian for (step n, dof d, stream, tag): Philox block -> two 52-bit
 * uniforms -> Box-Muller cosine branch with project-defined ln / cos. */
double orc_gauss(uint64_t seed, int64_t n, uint32_t d, uint32_t stream, uint32_t tag);
void orc_gauss_fill(uint64_t seed, int64_t n0, int64_t n_rows, uint32_t d0, uint32_t n_dof,
                    uint32_t stream, uint32_t tag, double *out /* [n_rows][n_dof] */);
/* The pieces of the transform, exposed for the tests. */
double orc_log_spec(double u);
double orc_cos2pi_spec(uint64_t odd53);

/* Coloured noise value zeta_{n,d} = sum_k h_k w_{n-k,d} (direct sum). */
double orc_zeta(const double *h, int two_nf, uint64_t seed, uint32_t stream,
                int64_t n, uint32_t d);

/* ---------------------------------------------------------------- potential */
/* On-site kinds (independent oscillators, every dof alone), per species V0, d:
 *   MORSE        V(x) = V0 (1 - exp(-x/d))^2         (well at x = 0)
 *   DOUBLE_WELL  V(x) = V0 ((x/d)^2 - 1)^2           (wells at x = +-d)
 * The anharmonicity of eq. (13) is C = hbar^2 / (2 m V0 d^2). */
enum { ORC_POT_PAIR = 0, ORC_POT_HARMONIC = 1, ORC_POT_MORSE = 2, ORC_POT_DOUBLE_WELL = 3 };
#define ORC_MAX_SPECIES 4
typedef struct {
    int kind;
    int n_species;
    double mass[ORC_MAX_SPECIES];
    double charge[ORC_MAX_SPECIES];
    double buck_A[ORC_MAX_SPECIES * ORC_MAX_SPECIES];
    double buck_rho[ORC_MAX_SPECIES * ORC_MAX_SPECIES];
    double buck_C[ORC_MAX_SPECIES * ORC_MAX_SPECIES];
    double dsf_alpha, r_cut, skin;
    double os_V0[ORC_MAX_SPECIES];  /* on-site kinds: energy scale */
    double os_d[ORC_MAX_SPECIES];   /* on-site kinds: length scale */
} orc_pot;

/* Buckingham (shifted force) + damped shifted force Coulomb, summed over every
 * periodic image within r_cut (no minimum-image shortcut).  pos/f: [3][N].
 * Returns the energy including the DSF self term; f = -grad E.
 * virial (nullable) receives sum_pairs d (x) F  (9 entries). */
double orc_pair_bruteforce(const orc_pot *pot, const orc_units *u, int N,
                           const double box[3], const int32_t *species,
                           const double *pos, double *f, double *virial);

/* --------------------------------------------------------------- simulation */
typedef struct orc_sim orc_sim;

/* State layout [P][dims][N].  noise_kind: 0 white (classical Langevin / PIMD),
 * 1 QTB (theta), 2 QTB-PIMD (kappa_P).  For kind 0 the taps are sqrt(kB T)
 * delta_k0 and two_nf is ignored (set to 2). */
orc_sim *orc_sim_new(const orc_pot *pot, const orc_units *u, int N, int P, int dims,
                     const double box[3], const int32_t *species,
                     const double *harm_omega, double T, double gamma, double dt,
                     uint64_t seed, uint32_t stream, int noise_kind, int two_nf,
                     const double *pos0, const double *vel0, int64_t step0,
                     int n_threads);
/* Observables per sample: kinetic, potential, spring, e_primitive, e_virial,
 * t_kinetic, x2_mean, step, pressure (pair kind; 0 otherwise), pair virial
 * sum_s W_s. */
#define ORC_NOBS 10
/* Run n steps; every obs_every steps write ORC_NOBS observables to obs_out. */
int orc_sim_run(orc_sim *s, int64_t n_steps, int obs_every, double *obs_out);
void orc_sim_get(const orc_sim *s, double *pos, double *vel, double *force, int64_t *step);
const double *orc_sim_taps(const orc_sim *s, int *two_nf);
void orc_sim_free(orc_sim *s);
/* Observables of the current state (the same ORC_NOBS numbers). */
void orc_sim_observe(orc_sim *s, double *obs);
/* Isotropic stochastic cell rescaling after every step (pair kind, any P):
 * target pressure P0, relaxation time tau_p, compressibility beta_T (the
 * caller's units).  Returns nonzero if refused. */
int orc_sim_set_barostat(orc_sim *s, double P0, double tau_p, double beta_T);
/* Isotropic Langevin piston after every step (pair kind, any P): target
 * pressure P0, piston time scale tau_p (mass (3 N P + 3) k_B T tau_p^2),
 * piston friction gamma_p.  Returns nonzero if refused. */
int orc_sim_set_piston(orc_sim *s, double P0, double tau_p, double gamma_p);
double orc_sim_piston_momentum(const orc_sim *s);
/* {p_e, s, s_v1, s_v2}: piston momentum and the scalings pending for the
 * next step (1 when none; the box between steps is the one the positions
 * were taken in).  get and/or set may be NULL. */
void orc_sim_barostat_state(orc_sim *s, double *get, const double *set);
/* Current box lengths. */
void orc_sim_box(const orc_sim *s, double *box);
/* Hamiltonian of the ring polymer, sum p^2/2m + sum_s [V_s/P + springs]. */
double orc_sim_hamiltonian(orc_sim *s);

/* Normal-mode matrix C[s*P + k] (orthonormal real DFT). */
void orc_nm_matrix(int P, double *C);

#ifdef __cplusplus
}
#endif
#endif
