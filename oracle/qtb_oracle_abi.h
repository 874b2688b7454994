/*
 * The oracle behind the same call shape as the accelerated library's C ABI
 * (four calls of the method and state access), test infrastructure only, so
 * that one harness can drive either back end: the argument lists, struct
 * members and their order, status codes and the meaning of each value are
 * those of the library's interface, restated here; the differences are that
 * every array is a HOST array and that the state arrays of a replica
 * (pos / vel) are the caller's and are kept current after every
 * orc_qtb_step, as the library keeps the caller's device arrays.
 *
 * Scope: the pair potential and the independent harmonic oscillators (the
 * kinds the oracle integrates with its full step), FP64 throughout (prec and
 * fir are accepted and ignored), no workspace and no stream (pass NULL / 0).
 */
#ifndef QTB_ORACLE_ABI_H
#define QTB_ORACLE_ABI_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_qtb_ctx orc_qtb_ctx;

enum {
    ORC_QTB_OK = 0, ORC_QTB_E_INVALID = 1, ORC_QTB_E_NOMEM = 2, ORC_QTB_E_DEVICE = 3,
    ORC_QTB_E_STATE = 4, ORC_QTB_E_NONFINITE = 5, ORC_QTB_E_UNSUPPORTED = 6
};

#define ORC_QTB_MAX_SPECIES 4

typedef struct {
    int32_t kind;              /* 0 pair, 1 harmonic                            */
    int32_t n_species;         /* 1..ORC_QTB_MAX_SPECIES                        */
    const double *mass;        /* [n_species]                                   */
    const double *charge;      /* [n_species] (pair kind)                       */
    const double *buck_A;      /* [n_species^2]                                 */
    const double *buck_rho;    /* [n_species^2]                                 */
    const double *buck_C;      /* [n_species^2]                                 */
    double dsf_alpha;
    double r_cut;
    double skin;
    const double *onsite_V0;   /* unused here                                   */
    const double *onsite_d;    /* unused here                                   */
} orc_qtb_potential;

typedef struct {
    int32_t n_atoms;
    int32_t n_beads;
    int32_t n_dims;            /* 3 (pair) or 1 / 3 (harmonic)                  */
    int32_t noise;             /* 0 white, 1 QTB (eq. 1), 2 QTB-PIMD (eq. 10)   */
    double box[3];
    double T, gamma, dt;
    uint64_t seed;
    uint32_t stream;
    uint32_t reserved;
    const int32_t *species;    /* host [N]                                      */
    const double *harm_omega;  /* host [N] (harmonic kind)                      */
    double *pos;               /* HOST [P][n_dims][N], kept current             */
    double *vel;               /* HOST [P][n_dims][N], kept current             */
} orc_qtb_replica;

typedef struct {
    double hbar, kB, coulomb_k, mass_unit;
    int32_t prec, fir, fir_block_K, obs_every, max_two_nf, flags;
    double ml_r_cut;
} orc_qtb_options;

typedef struct {
    int64_t step;
    double kinetic, potential, spring, e_primitive, e_virial, t_kinetic, x2_mean;
    double virial_pair, pressure, volume;
    int32_t n_samples;
} orc_qtb_obs;

/* Bytes of device workspace the call shape asks for: 0 (the oracle keeps
 * its state on the host). */
size_t orc_qtb_workspace_bytes(const orc_qtb_potential *pot, const orc_qtb_replica *reps,
                               int32_t n_rep, const orc_qtb_options *opt);
/* Copy the descriptions (the replica structs' pointers stay the caller's).
 * ORC_QTB_E_INVALID for an unsupported kind, bad sizes, T <= 0, dt <= 0,
 * gamma < 0, or max_two_nf not a power of two. */
int orc_qtb_init(orc_qtb_ctx **out, const orc_qtb_potential *pot, const orc_qtb_replica *reps,
                 int32_t n_rep, const orc_qtb_options *opt, void *workspace, size_t ws_bytes,
                 void *stream);
/* Filter of replica (-1: all) for noise kind, two_nf taps (a power of two,
 * <= max_two_nf; ignored for white noise); taps_out (nullable host
 * [two_nf]) receives them.  The replica's integrator starts from its current
 * state and step. */
int orc_qtb_build_filter(orc_qtb_ctx *c, int32_t replica, int32_t kind, int32_t two_nf,
                         double *taps_out);
/* n_steps of every replica (ORC_QTB_E_STATE before its filter); samples
 * every obs_every steps of the replica's own step counter. */
int orc_qtb_step(orc_qtb_ctx *c, int64_t n_steps);
/* Means over the samples since the previous call (then reset). */
int orc_qtb_observables(orc_qtb_ctx *c, int32_t replica, orc_qtb_obs *out);
int orc_qtb_get_state(orc_qtb_ctx *c, int32_t replica, double *h_pos, double *h_vel,
                      int64_t *step);
/* Replace the state and step counter (nullable arrays keep theirs). */
int orc_qtb_set_state(orc_qtb_ctx *c, int32_t replica, const double *h_pos,
                      const double *h_vel, int64_t step);
const char *orc_qtb_last_error(const orc_qtb_ctx *c);
void orc_qtb_destroy(orc_qtb_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
