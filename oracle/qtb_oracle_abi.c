/*
 * The oracle behind the library's call shape (see qtb_oracle_abi.h): a
 * bookkeeping layer over orc_sim (qtb_oracle.c), test infrastructure only.
 * Each replica gets its own orc_sim when its filter is built (the noise kind
 * and the filter length are fixed at creation), started from the caller's
 * host state; after every orc_qtb_step the state is copied back into the
 * caller's arrays, and the samples are summed for orc_qtb_observables.
 */
#include "qtb_oracle_abi.h"
#include "qtb_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    orc_qtb_replica d;        /* the caller's description (its pointers) */
    int32_t *species;         /* own copy */
    double *omega;            /* own copy (harmonic kind) */
    orc_sim *sim;             /* NULL until the filter is built */
    int kind, two_nf;         /* the built filter */
    int64_t step;             /* step counter while no sim exists */
    double acc[ORC_NOBS + 1]; /* sums of the samples (+ volume) */
    int32_t n_samples;
} orc_qtb_rep;

struct orc_qtb_ctx {
    orc_pot pot;
    orc_units u;
    orc_qtb_options opt;
    int32_t n_rep;
    orc_qtb_rep *reps;
    char err[256];
};

static int fail(orc_qtb_ctx *c, int status, const char *msg)
{
    if (c) snprintf(c->err, sizeof c->err, "%s", msg);
    return status;
}

static int pow2(int32_t n) { return n >= 2 && (n & (n - 1)) == 0; }

static size_t nstate(const orc_qtb_replica *r)
{
    return (size_t)r->n_beads * r->n_dims * r->n_atoms;
}

size_t orc_qtb_workspace_bytes(const orc_qtb_potential *pot, const orc_qtb_replica *reps,
                               int32_t n_rep, const orc_qtb_options *opt)
{
    (void)pot; (void)reps; (void)n_rep; (void)opt;
    return 0;
}

int orc_qtb_init(orc_qtb_ctx **out, const orc_qtb_potential *pot, const orc_qtb_replica *reps,
                 int32_t n_rep, const orc_qtb_options *opt, void *workspace, size_t ws_bytes,
                 void *stream)
{
    (void)workspace; (void)ws_bytes; (void)stream;
    if (!out || !pot || !reps || !opt || n_rep < 1) return ORC_QTB_E_INVALID;
    *out = NULL;
    if (pot->kind != 0 && pot->kind != 1) return ORC_QTB_E_UNSUPPORTED;
    if (pot->n_species < 1 || pot->n_species > ORC_QTB_MAX_SPECIES || !pot->mass)
        return ORC_QTB_E_INVALID;
    if (!(opt->hbar > 0.0) || !(opt->kB > 0.0) || !(opt->mass_unit > 0.0) ||
        !pow2(opt->max_two_nf) || opt->obs_every < 0)
        return ORC_QTB_E_INVALID;
    for (int32_t r = 0; r < n_rep; ++r) {
        const orc_qtb_replica *d = &reps[r];
        if (d->n_atoms < 1 || d->n_beads < 1 || d->n_beads > 64 || !d->species || !d->pos ||
            !d->vel || !(d->T > 0.0) || !(d->dt > 0.0) || !(d->gamma >= 0.0) ||
            d->noise < 0 || d->noise > 2)
            return ORC_QTB_E_INVALID;
        if (pot->kind == 0 && d->n_dims != 3) return ORC_QTB_E_INVALID;
        if (pot->kind == 1 && ((d->n_dims != 1 && d->n_dims != 3) || !d->harm_omega))
            return ORC_QTB_E_INVALID;
        for (int32_t i = 0; i < d->n_atoms; ++i)
            if (d->species[i] < 0 || d->species[i] >= pot->n_species) return ORC_QTB_E_INVALID;
    }
    orc_qtb_ctx *c = (orc_qtb_ctx *)calloc(1, sizeof *c);
    if (!c) return ORC_QTB_E_NOMEM;
    c->opt = *opt;
    c->u.hbar = opt->hbar;
    c->u.kB = opt->kB;
    c->u.coulomb_k = opt->coulomb_k;
    c->u.mass_unit = opt->mass_unit;
    const int ns = pot->n_species;
    c->pot.kind = pot->kind == 0 ? ORC_POT_PAIR : ORC_POT_HARMONIC;
    c->pot.n_species = ns;
    for (int a = 0; a < ns; ++a) {
        c->pot.mass[a] = pot->mass[a];
        c->pot.charge[a] = pot->charge ? pot->charge[a] : 0.0;
    }
    for (int q = 0; q < ns * ns; ++q) {  /* [n_species][n_species], as the call shape */
        c->pot.buck_A[q] = pot->buck_A ? pot->buck_A[q] : 0.0;
        c->pot.buck_rho[q] = pot->buck_rho ? pot->buck_rho[q] : 1.0;
        c->pot.buck_C[q] = pot->buck_C ? pot->buck_C[q] : 0.0;
    }
    c->pot.dsf_alpha = pot->dsf_alpha;
    c->pot.r_cut = pot->r_cut;
    c->pot.skin = pot->skin;
    c->n_rep = n_rep;
    c->reps = (orc_qtb_rep *)calloc((size_t)n_rep, sizeof *c->reps);
    if (!c->reps) {
        free(c);
        return ORC_QTB_E_NOMEM;
    }
    for (int32_t r = 0; r < n_rep; ++r) {
        orc_qtb_rep *R = &c->reps[r];
        R->d = reps[r];
        R->species = (int32_t *)malloc(sizeof(int32_t) * (size_t)reps[r].n_atoms);
        if (R->species) memcpy(R->species, reps[r].species, sizeof(int32_t) * reps[r].n_atoms);
        if (reps[r].harm_omega) {
            R->omega = (double *)malloc(sizeof(double) * (size_t)reps[r].n_atoms);
            if (R->omega) memcpy(R->omega, reps[r].harm_omega, sizeof(double) * reps[r].n_atoms);
        }
        if (!R->species || (reps[r].harm_omega && !R->omega)) {
            orc_qtb_destroy(c);
            return ORC_QTB_E_NOMEM;
        }
    }
    *out = c;
    return ORC_QTB_OK;
}

/* (Re)create the replica's integrator from the caller's current state. */
static int make_sim(orc_qtb_ctx *c, int32_t r, int kind, int two_nf)
{
    orc_qtb_rep *R = &c->reps[r];
    const orc_qtb_replica *d = &R->d;
    int64_t step = R->step;
    if (R->sim) {
        orc_sim_get(R->sim, NULL, NULL, NULL, &step);
        orc_sim_free(R->sim);
        R->sim = NULL;
    }
    R->sim = orc_sim_new(&c->pot, &c->u, d->n_atoms, d->n_beads, d->n_dims, d->box, R->species,
                         R->omega, d->T, d->gamma, d->dt, d->seed, d->stream, kind,
                         kind ? two_nf : 2, d->pos, d->vel, step, 8);
    R->step = step;
    R->kind = kind;
    R->two_nf = two_nf;
    return R->sim ? ORC_QTB_OK : fail(c, ORC_QTB_E_NOMEM, "oracle simulation not created");
}

int orc_qtb_build_filter(orc_qtb_ctx *c, int32_t replica, int32_t kind, int32_t two_nf,
                         double *taps_out)
{
    if (!c) return ORC_QTB_E_INVALID;
    if (replica < -1 || replica >= c->n_rep) return fail(c, ORC_QTB_E_INVALID, "replica out of range");
    if (kind < 0 || kind > 2) return fail(c, ORC_QTB_E_INVALID, "noise kind");
    if (kind && (!pow2(two_nf) || two_nf > c->opt.max_two_nf))
        return fail(c, ORC_QTB_E_INVALID, "two_nf must be a power of two <= max_two_nf");
    for (int32_t r = (replica < 0 ? 0 : replica); r < (replica < 0 ? c->n_rep : replica + 1); ++r) {
        int s = make_sim(c, r, kind, two_nf);
        if (s) return s;
        if (taps_out && replica >= 0) {
            int n = 0;
            const double *h = orc_sim_taps(c->reps[r].sim, &n);
            memcpy(taps_out, h, sizeof(double) * (size_t)n);
        }
    }
    return ORC_QTB_OK;
}

int orc_qtb_step(orc_qtb_ctx *c, int64_t n_steps)
{
    if (!c || n_steps < 0) return fail(c, ORC_QTB_E_INVALID, "n_steps must be >= 0");
    for (int32_t r = 0; r < c->n_rep; ++r)
        if (!c->reps[r].sim) return fail(c, ORC_QTB_E_STATE, "build_filter not called");
    const int every = c->opt.obs_every;
    for (int32_t r = 0; r < c->n_rep; ++r) {
        orc_qtb_rep *R = &c->reps[r];
        const int64_t nmax = every > 0 ? n_steps / every + 1 : 0;
        double *obs = nmax ? (double *)malloc(sizeof(double) * ORC_NOBS * (size_t)nmax) : NULL;
        if (nmax && !obs) return fail(c, ORC_QTB_E_NOMEM, "observable buffer");
        const int n = orc_sim_run(R->sim, n_steps, every, obs);
        double box[3] = {0.0, 0.0, 0.0};
        if (c->pot.kind == ORC_POT_PAIR) orc_sim_box(R->sim, box);
        for (int k = 0; k < n; ++k) {
            for (int q = 0; q < ORC_NOBS; ++q) R->acc[q] += obs[(size_t)k * ORC_NOBS + q];
            R->acc[ORC_NOBS] += box[0] * box[1] * box[2];
        }
        R->n_samples += n;
        free(obs);
        orc_sim_get(R->sim, R->d.pos, R->d.vel, NULL, &R->step);
        const size_t m = nstate(&R->d);
        for (size_t q = 0; q < m; ++q)
            if (!isfinite(R->d.pos[q]) || !isfinite(R->d.vel[q]))
                return fail(c, ORC_QTB_E_NONFINITE, "non-finite position or velocity");
    }
    return ORC_QTB_OK;
}

int orc_qtb_observables(orc_qtb_ctx *c, int32_t replica, orc_qtb_obs *out)
{
    if (!c || !out) return fail(c, ORC_QTB_E_INVALID, "null argument");
    if (replica < 0 || replica >= c->n_rep) return fail(c, ORC_QTB_E_INVALID, "replica out of range");
    orc_qtb_rep *R = &c->reps[replica];
    memset(out, 0, sizeof *out);
    out->step = R->step;
    out->n_samples = R->n_samples;
    if (R->n_samples > 0) {
        /* oracle sample order: kinetic, potential, spring, e_primitive,
         * e_virial, t_kinetic, x2_mean, step, pressure, pair virial */
        const double inv = 1.0 / R->n_samples;
        out->kinetic = R->acc[0] * inv;
        out->potential = R->acc[1] * inv;
        out->spring = R->acc[2] * inv;
        out->e_primitive = R->acc[3] * inv;
        out->e_virial = R->acc[4] * inv;
        out->t_kinetic = R->acc[5] * inv;
        out->x2_mean = R->acc[6] * inv;
        out->pressure = R->acc[8] * inv;
        out->virial_pair = R->acc[9] * inv;
        out->volume = R->acc[ORC_NOBS] * inv;
    }
    memset(R->acc, 0, sizeof R->acc);
    R->n_samples = 0;
    return ORC_QTB_OK;
}

int orc_qtb_get_state(orc_qtb_ctx *c, int32_t replica, double *h_pos, double *h_vel,
                      int64_t *step)
{
    if (!c) return ORC_QTB_E_INVALID;
    if (replica < 0 || replica >= c->n_rep) return fail(c, ORC_QTB_E_INVALID, "replica out of range");
    orc_qtb_rep *R = &c->reps[replica];
    const size_t m = nstate(&R->d);
    if (h_pos) memcpy(h_pos, R->d.pos, sizeof(double) * m);
    if (h_vel) memcpy(h_vel, R->d.vel, sizeof(double) * m);
    if (step) *step = R->step;
    return ORC_QTB_OK;
}

int orc_qtb_set_state(orc_qtb_ctx *c, int32_t replica, const double *h_pos,
                      const double *h_vel, int64_t step)
{
    if (!c) return ORC_QTB_E_INVALID;
    if (replica < 0 || replica >= c->n_rep) return fail(c, ORC_QTB_E_INVALID, "replica out of range");
    orc_qtb_rep *R = &c->reps[replica];
    const size_t m = nstate(&R->d);
    if (h_pos) memmove(R->d.pos, h_pos, sizeof(double) * m);
    if (h_vel) memmove(R->d.vel, h_vel, sizeof(double) * m);
    R->step = step;
    if (R->sim) {  /* restart the integrator (its reference positions too) */
        orc_sim_free(R->sim);
        R->sim = NULL;
        return make_sim(c, replica, R->kind, R->two_nf);
    }
    return ORC_QTB_OK;
}

const char *orc_qtb_last_error(const orc_qtb_ctx *c) { return c ? c->err : "ctx is NULL"; }

void orc_qtb_destroy(orc_qtb_ctx *c)
{
    if (!c) return;
    for (int32_t r = 0; r < c->n_rep; ++r) {
        if (c->reps[r].sim) orc_sim_free(c->reps[r].sim);
        free(c->reps[r].species);
        free(c->reps[r].omega);
    }
    free(c->reps);
    free(c);
}
