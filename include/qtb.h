/*
 * qtb.h -- C ABI of libqtb.so, the MI355X (gfx950) integrator step for
 * quantum-thermal-bath (QTB) Langevin dynamics and its combination with
 * path-integral MD (QTB-PIMD), after Dammak, Hayoun, Brieuc and Geneste,
 * "Nuclear quantum effects in molecular dynamics simulations"
 * (arXiv:1905.02521).
 *
 * One step advances every replica of a context by dt:
 *   B(dt/2) -> normal modes -> A(dt/2) -> O(dt) -> A(dt/2) -> beads ->
 *   forces -> B(dt/2)
 * B applies the bead force -(1/P) grad V with bead mass m (eq. 4); A is the
 * exact propagation of the ring-polymer springs of eq. (3) in normal modes;
 * O is the Langevin friction of eq. (8) with a coloured random force of power
 * spectral density 2 m gamma theta(omega, T) (eq. 6-7, theta from eq. 1) for
 * QTB, or 2 m gamma kappa_P(omega, T) (eq. 10-12) for QTB-PIMD, acting on
 * the ring-polymer normal modes (Sec. 2.3).  White noise (k_B T) gives
 * classical Langevin dynamics (P = 1) or classical PIMD (P > 1).
 *
 * Conventions shared by every entry point:
 *  - Units are the caller's, fixed by qtb_options: the library takes hbar,
 *    k_B, the Coulomb constant and the mass unit as inputs (the tests use
 *    eV, Angstrom, amu, fs, K, or reduced units).
 *  - State arrays are FP64, layout [P][n_dims][N] (bead-major, then
 *    Cartesian component, then atom: structure of arrays), caller-owned
 *    device memory.  Positions are never wrapped into the box.
 *  - The library never allocates device memory: every device buffer comes
 *    from the caller (state arrays and one workspace sized by
 *    qtb_workspace_bytes).  The library frees only its host-side context.
 *  - Work is enqueued on the caller's HIP stream.  Only qtb_observables,
 *    qtb_get_state, qtb_set_state, qtb_evaluate and qtb_get_noise
 *    synchronise that stream.
 *  - Errors: every call returns a qtb_status; nothing aborts or throws
 *    across the ABI.  A failing call leaves a message for qtb_last_error.
 *  - A context is not re-entrant; separate contexts on separate streams are
 *    independent.
 */
#ifndef QTB_H
#define QTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtb_ctx qtb_ctx; /* opaque */

typedef enum {
    QTB_OK = 0,
    QTB_E_INVALID = 1,     /* bad argument or size */
    QTB_E_NOMEM = 2,       /* workspace too small, neighbour list overflow */
    QTB_E_DEVICE = 3,      /* HIP runtime error */
    QTB_E_STATE = 4,       /* call out of order (e.g. step before its filter) */
    QTB_E_NONFINITE = 5,   /* NaN / Inf found in the state */
    QTB_E_UNSUPPORTED = 6  /* valid request the library does not implement */
} qtb_status;

/* Noise kinds: the power spectral density of the random force, eq. (7)/(12). */
typedef enum {
    QTB_NOISE_CLASSICAL = 0, /* k_B T: white noise (Langevin / classical PIMD) */
    QTB_NOISE_QTB = 1,       /* theta(omega, T), eq. (1) and (7)              */
    QTB_NOISE_QTB_PIMD = 2   /* kappa_P(omega, T), eq. (10)-(12)              */
} qtb_noise;

/* Arithmetic of the force and noise kernels.  State, energies and the filter
 * design are FP64 in every mode. */
typedef enum { QTB_PREC_FP32 = 0, QTB_PREC_FP64 = 1 } qtb_prec;

/* Arithmetic of the coloured-noise contraction (FIR blocked over K steps). */
typedef enum {
    QTB_FIR_FP32 = 0,   /* FP32 matrix cores, FP32 accumulation                    */
    QTB_FIR_BF16X3 = 1, /* BF16 matrix cores, hi*hi + hi*lo + lo*hi split, FP32 acc */
    QTB_FIR_BF16 = 2,   /* BF16 matrix cores, single product, FP32 acc             */
    QTB_FIR_FP64 = 3    /* FP64 vector ALU                                          */
} qtb_fir;

typedef enum {
    QTB_POT_PAIR = 0,        /* Buckingham + damped shifted force Coulomb, 3D, periodic */
    QTB_POT_HARMONIC = 1,    /* independent oscillators V = 1/2 m omega_i^2 x^2 per dof  */
    QTB_POT_MORSE = 2,       /* independent dofs, V = V0 (1 - exp(-x/d))^2              */
    QTB_POT_DOUBLE_WELL = 3  /* independent dofs, V = V0 ((x/d)^2 - 1)^2               */
} qtb_pot_kind;

#define QTB_MAX_SPECIES 4

/*
 * Potential, shared by every replica of a context.  The paper gives no pair
 * potential; the pair kind is V = sum_pairs [Buckingham in shifted-force form
 * at r_cut: A exp(-r/rho) - C/r^6] + damped shifted force Coulomb (alpha,
 * r_cut) including its self term.  Pairs are summed over every periodic
 * image within r_cut (boxes smaller than 2 r_cut are handled).  The Morse and
 * double-well kinds are the one-dimensional anharmonic models of Sec. 3: every
 * dof is an independent oscillator with the anharmonicity
 * C = hbar^2 / (2 m V0 d^2) of eq. 13; like the harmonic kind they take no box.
 * Host pointers; copied at qtb_init.
 */
typedef struct {
    int32_t kind;              /* qtb_pot_kind                                  */
    int32_t n_species;         /* 1..QTB_MAX_SPECIES                            */
    const double *mass;        /* [n_species] mass                              */
    const double *charge;      /* [n_species] charge (pair kind)                */
    const double *buck_A;      /* [n_species^2] energy; 0 = no Buckingham term  */
    const double *buck_rho;    /* [n_species^2] length                          */
    const double *buck_C;      /* [n_species^2] energy * length^6               */
    double dsf_alpha;          /* damping parameter, 1/length                   */
    double r_cut;              /* cut-off, > 0                                  */
    double skin;               /* Verlet skin, >= 0                             */
    const double *onsite_V0;   /* [n_species] energy, > 0 (Morse, double well)  */
    const double *onsite_d;    /* [n_species] length, > 0 (Morse, double well)  */
} qtb_potential;

/*
 * One replica: N atoms x P beads (P = 1: QTB / Langevin; P > 1: the ring
 * polymer of eq. 3 with omega_P = sqrt(P) k_B T / hbar).  species and
 * harm_omega are host pointers copied at qtb_init; d_pos / d_vel are device
 * pointers that stay owned by the caller and must outlive the context.
 */
typedef struct {
    int32_t n_atoms;           /* N >= 1                                        */
    int32_t n_beads;           /* P >= 1                                        */
    int32_t n_dims;            /* 3 (pair kind) or 1 / 3 (harmonic kind)        */
    int32_t noise;             /* qtb_noise                                     */
    double box[3];             /* orthorhombic box lengths (pair kind)          */
    double T;                  /* temperature, > 0                              */
    double gamma;              /* friction, 1/time, >= 0                        */
    double dt;                 /* time step, > 0                                */
    uint64_t seed;             /* Philox key                                    */
    uint32_t stream;           /* Philox counter word: independent noise stream */
    uint32_t reserved;
    const int32_t *species;    /* host [N], values in [0, n_species)            */
    const double *harm_omega;  /* host [N] angular frequencies (harmonic kind)  */
    double *d_pos;             /* device [P][n_dims][N] FP64                    */
    double *d_vel;             /* device [P][n_dims][N] FP64                    */
} qtb_replica;

typedef struct {
    double hbar;               /* energy * time                                  */
    double kB;                 /* energy / temperature                           */
    double coulomb_k;          /* energy * length / charge^2                     */
    double mass_unit;          /* energy per (mass * length^2 / time^2)          */
    int32_t prec;              /* qtb_prec                                       */
    int32_t fir;               /* qtb_fir                                        */
    int32_t fir_block_K;       /* steps per noise block: multiple of 64, >= 64   */
    int32_t obs_every;         /* sample observables every n steps (0 = never)   */
    int32_t max_two_nf;        /* largest FIR length any replica will use, a     */
                               /* power of two in [2, 8192]                      */
    int32_t flags;             /* QTB_OPT_* bits                                 */
    double ml_r_cut;           /* > 0: reserve the surrogate's buffers for this  */
                               /* descriptor cut-off (<= r_cut); 0: none         */
} qtb_options;

/* qtb_options.flags: run every step eagerly instead of replaying whole noise
 * blocks as captured HIP graphs (graphs are used on a non-default stream when
 * obs_every is 0 or divides fir_block_K). */
#define QTB_OPT_NO_GRAPH 1
/* qtb_options.flags: keep the default force-kernel decomposition instead of
 * timing the candidates on the first qtb_step (the autotuner). */
#define QTB_OPT_NO_AUTOTUNE 2
/* qtb_options.flags: also reserve the surrogate's training buffers. */
#define QTB_OPT_ML_TRAIN 4
/* qtb_options.flags: one kernel per step (forces, list rebuild and update
 * fused; pair potential with P = 1, 2, 4 or 8 for every replica).  The
 * results equal the separate kernels' bit for bit, except for rounding in
 * steps that rebuild a list.  Off by default: on gfx950 the fused kernel's
 * update tail costs more than the two launches it saves. */
#define QTB_OPT_FUSE 8
/* qtb_options.flags: make the coloured noise with the paper's block generator
 * (eq. 9) instead of the streaming FIR: for each block of n = max_two_nf
 * steps (global steps B n .. B n + n - 1) and each dof, random Fourier
 * amplitudes (a_j + i b_j) sqrt(n S_j / 2) on the grid omega_j = 2 pi j / (n dt)
 * (a_j, b_j the library's Gaussians at the replica step of the block's first
 * step + j, tags 1 and 2), completed Hermitian (mode n - j the conjugate of
 * mode j; modes 0 and n/2 real, a_j sqrt(n S_j)), then an inverse DFT.  S is
 * the filter's spectrum (theta, kappa_P or k_B T) on the same grid.
 * Blocks are independent: the noise has the target spectrum inside a block
 * and no correlation across block boundaries.  n must be a power of two in
 * [fir_block_K, 4096]; qtb_build_filter's two_nf must equal n; the noise
 * precision follows prec; not with QTB_OPT_FUSE. */
#define QTB_OPT_NOISE_BLOCKS 16
/* Build every replica's neighbour lists in the separate list kernel (by
 * default only replicas above 16 384 atoms and contexts with surrogate
 * buffers do; smaller replicas rebuild inside the force kernel).  The lists,
 * forces and trajectories are the same. */
#define QTB_OPT_LIST_KERNEL 32

/* Means over the samples taken since the previous qtb_observables call of
 * this replica (eq. 5 primitive estimator with instantaneous momenta). */
typedef struct {
    int64_t step;              /* the replica's step counter at the call (as get_state) */
    double kinetic;            /* sum_s sum_i p^2 / 2m                            */
    double potential;          /* sum_s V(r^(s)) / P                              */
    double spring;             /* sum_s sum_i m omega_P^2 (r_s - r_s+1)^2 / 2     */
    double e_primitive;        /* kinetic - spring + potential (eq. 5)            */
    double e_virial;           /* centroid virial estimator: K_c - sum_s (r_s - r_c).F_s */
                               /* / 2P + potential, K_c = sum_i m P |v_c,i|^2 / 2 the    */
                               /* measured centroid (mode k = 0) kinetic energy          */
    double t_kinetic;          /* 2 kinetic / (dims N P k_B)                      */
    double x2_mean;            /* mean of (r - r(init))^2 over beads, dims, atoms */
    double virial_pair;        /* sum_s W_s, W_s = sum over pairs of F(r) r at bead s */
    double pressure;           /* (2 kinetic - 2 spring + virial_pair / P) / (3 V):   */
                               /* the volume derivative of the (ring-polymer)        */
                               /* partition function, instantaneous momenta (pair    */
                               /* potential only; 0 for other kinds and surrogates)  */
                               /* averaged over the samples, each at its own volume  */
    double volume;             /* mean box volume of the samples (pair potential)    */
    int32_t n_samples;
} qtb_obs;

/* Workspace bytes needed for these replicas and options (0 on bad input). */
size_t qtb_workspace_bytes(const qtb_potential *pot, const qtb_replica *reps, int32_t n_rep,
                           const qtb_options *opt);

/*
 * Create a context over n_rep replicas that step together (one launch per
 * kernel covers all of them).  d_workspace: device buffer of at least
 * qtb_workspace_bytes, 256-byte aligned, owned by the caller.  hip_stream:
 * a hipStream_t (NULL = default stream).  Builds neighbour lists and the
 * initial forces; replicas with noise != CLASSICAL need qtb_build_filter
 * before qtb_step.
 */
qtb_status qtb_init(qtb_ctx **out, const qtb_potential *pot, const qtb_replica *reps,
                    int32_t n_rep, const qtb_options *opt, void *d_workspace,
                    size_t ws_bytes, void *hip_stream);

/*
 * Design the FIR filter of a replica (replica = -1: all replicas) from the
 * spectrum of eq. (7) (kind QTB: theta) or eq. (12) (kind QTB_PIMD: kappa_P
 * solving eq. 10-11), sampled on omega_j = pi j / (Nf dt), j = 0..Nf: the
 * taps are the 2Nf-point inverse DFT of sqrt(S_j), so the realised noise
 * spectrum equals S on that grid.  FP64 on the host, then copied to the
 * device in the precision of the FIR mode.  two_nf: a power of two in
 * [2, max_two_nf], else QTB_E_INVALID.
 * taps_out (nullable, host, [two_nf]) receives h_k for k = -Nf..Nf-1.
 * kind must equal the replica's noise.
 */
qtb_status qtb_build_filter(qtb_ctx *ctx, int32_t replica, int32_t kind, int32_t two_nf,
                            double *taps_out);

/* The same FIR design without a context, on the host only (no device
 * call): the taps h_k, k = -Nf..Nf-1, of kind CLASSICAL (sqrt(k_B T) at
 * k = 0), QTB (theta of eq. 1) or QTB_PIMD (kappa_P of eq. 10-11 for n_beads
 * beads) at temperature T and step dt, in the caller's units (hbar, kB).
 * two_nf: a power of two in [2, 8192]; n_beads in [1, 64]; taps_out: host
 * [two_nf], caller-owned.  QTB_E_INVALID on a bad argument (nothing
 * written), QTB_E_NONFINITE if the design overflowed. */
qtb_status qtb_filter_taps(int32_t kind, double T, int32_t n_beads, double dt, int32_t two_nf,
                           double hbar, double kB, double *taps_out);

/* Enqueue n_steps integrator steps of every replica; returns without waiting. */
qtb_status qtb_step(qtb_ctx *ctx, int64_t n_steps);

/* Synchronise the stream and return the observables of one replica.
 * Returns QTB_E_NONFINITE if a NaN/Inf was found in any state since the last
 * check or a bead spread grew past the list search's limit of 8 periodic
 * images per direction (a diverged trajectory), QTB_E_NOMEM if a neighbour
 * list overflowed. */
qtb_status qtb_observables(qtb_ctx *ctx, int32_t replica, qtb_obs *out);

/* Copy a replica's state to / from host arrays [P][n_dims][N]; set_state
 * also sets the replica's step counter, rebuilds the neighbour lists and
 * recomputes the forces of every replica, and opens a new noise block at
 * that step.  Either pointer may be NULL (that half unchanged): a caller
 * that wrote new states into its device arrays in place (on the context's
 * stream, between calls) makes the context take them all with one set_state
 * with both pointers NULL.  Positions passed to set_state also become the
 * reference of the observables' x2_mean (as the positions given at
 * creation do); positions written in place leave that reference as it was.
 * A restored state continues bit for bit like a context created from it
 * (same seed, stream, filter and options) with white noise and with the
 * FP32 and FP64 noise contractions, whatever the context ran before.  With
 * QTB_FIR_BF16X3 the contraction sums the noise window in chunks aligned
 * to 8-row groups of the context's own step count: the two runs agree bit
 * for bit when their context step counts are equal modulo 8 (a restored
 * replica step minus the context's step count a multiple of 8), and
 * otherwise to FP32 rounding of the noise (measured 3e-7 A after 64 steps
 * of a 3x3x3 crystal). */
qtb_status qtb_get_state(qtb_ctx *ctx, int32_t replica, double *h_pos, double *h_vel,
                         int64_t *step);
qtb_status qtb_set_state(qtb_ctx *ctx, int32_t replica, const double *h_pos,
                         const double *h_vel, int64_t step);

/* Recompute forces of the current state of every replica (no kick) and
 * return replica's forces -grad V(r^(s)) per bead (host [P][n_dims][N]) and
 * per-bead potential energies V(r^(s)) (host [P]).  Either may be NULL. */
qtb_status qtb_evaluate(qtb_ctx *ctx, int32_t replica, double *h_force, double *h_epot);

/* The coloured noise zeta_{n,d} = sum_k h_k w_{n-k,d} of the last completed
 * noise block of a replica: host [K][n_dof] FP64 (n_dof = n_dims N P,
 * dof d = (n_dims * atom + dim) * P + mode), first step in *n0. */
qtb_status qtb_get_noise(qtb_ctx *ctx, int32_t replica, double *h_zeta, int64_t *n0);

/*
 * The library's white-noise generator, standalone: d_out[r * n_dof + j] =
 * w(n0 + r, d0 + j) for the given key and stream, FP64, device buffer of
 * n_rows * n_dof doubles.  w is a unit Gaussian from one Philox4x32-10 block
 * (Salmon et al., SC'11) at counter (n + 2^40 as two words, d, 16 stream +
 * tag), key (seed low, seed high): two 52-bit uniforms, then the cosine
 * branch of Box-Muller with the library's own ln and cos(2 pi u).  The paper
 * asks only for normally distributed numbers (eq. 9); the counter-based form
 * makes every value reproducible from its indices.
 */
qtb_status qtb_gaussian(uint64_t seed, uint32_t stream, uint32_t tag, int64_t n0,
                        int64_t n_rows, uint32_t d0, uint32_t n_dof, double *d_out,
                        void *hip_stream);

/*
 * Velocity density of states (Sec. 3: time-correlation functions are directly
 * accessible in QTB-MD, unlike in PIMD and QTB-PIMD, and the vibrational DOS
 * is the check to make when gamma is raised against zero-point-energy
 * leakage).  By the Wiener-Khinchin theorem the spectrum of the velocity
 * series is the Fourier transform of its autocorrelation; it is estimated by
 * segment periodograms,
 *   S_k = (1/n_seg) sum_segments sum_j w_j |sum_{t<seg} v_{t,j} e^{-2 pi i k t / seg}|^2 / seg,
 * k = 0 .. seg/2 (frequency 2 pi k / (seg * sampling interval)), FP64, with
 * w_j the mass of dof j (m * mass_unit, the energy units of qtb_obs): the
 * mean of S over all seg frequencies (k and seg - k both counted) is then
 * twice the mean kinetic energy of the sampled velocities.  seg: a power of
 * two, 16..4096.  The transform is a radix-2 FFT in LDS; partial sums are
 * added in a fixed order, so results repeat bit for bit.
 */

/* Device bytes of a spectrum workspace for n_dof dofs: recorder = 1 for
 * qtb_vdos_attach (two segments of trace, FP64), 0 for qtb_vdos_spectrum.
 * 0 on bad input. */
size_t qtb_vdos_workspace_bytes(int32_t n_dof, int32_t seg, int32_t recorder);

/* The spectrum of a device series (FP64): sample t of dof j at
 * d_v[t * sample_stride + j * dof_stride] (strides in elements, >= 1:
 * [n_samples][n_dof] row-major is (n_dof, 1), [n_dof][n_samples] is
 * (1, n_samples)), with device weights d_weight [n_dof], over its
 * n_samples / seg whole segments (a trailing partial segment is ignored;
 * with none, S = 0): d_spec (device, [seg/2 + 1]) receives S.  d_workspace:
 * device, 256-byte aligned, qtb_vdos_workspace_bytes(n_dof, seg, 0) bytes.
 * Enqueued on hip_stream; returns without waiting. */
qtb_status qtb_vdos_spectrum(const double *d_v, int64_t n_samples, int32_t n_dof,
                             int64_t sample_stride, int64_t dof_stride, const double *d_weight,
                             int32_t seg, double *d_spec, void *d_workspace, size_t ws_bytes,
                             void *hip_stream);

/* qtb_vdos_spectrum for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same arguments without the workspace.  The scratch is a static device
 * array of 16 MiB per GPU, held until the process ends; sizes whose
 * qtb_vdos_workspace_bytes(n_dof, seg, 0) exceeds it return QTB_E_INVALID
 * (nothing is enqueued).  No hipMalloc, hipFree or allocating call.  Every
 * call on a GPU uses that GPU's one scratch array: calls that overlap on one
 * GPU (on different streams, or from several threads) race; calls on one
 * stream are ordered by it.  hip_stream must belong to the current device.
 * The first call on a device looks up the array's device address. */
qtb_status qtb_vdos_spectrum_noalloc(const double *d_v, int64_t n_samples, int32_t n_dof,
                                     int64_t sample_stride, int64_t dof_stride,
                                     const double *d_weight, int32_t seg, double *d_spec,
                                     void *hip_stream);

/* Attach a velocity recorder to a replica with P = 1 (QTB_E_INVALID for
 * P > 1: ring-polymer bead velocities carry no physical time correlations).
 * From now on every observable sample (every obs_every steps; QTB_E_STATE
 * when obs_every is 0) also stores the replica's velocities [n_dims][N] in
 * the recorder's trace, and each completed segment of seg samples is
 * transformed on the context's stream during qtb_step.  Requires
 * seg * obs_every >= fir_block_K.  d_workspace: device, 256-byte aligned,
 * qtb_vdos_workspace_bytes(n_dims N, seg, 1) bytes, caller-owned, in use
 * until qtb_vdos_detach.  Attaching again replaces the recorder.
 * qtb_set_state of the replica restarts it (the series is cut there). */
qtb_status qtb_vdos_attach(qtb_ctx *ctx, int32_t replica, int32_t seg, void *d_workspace,
                           size_t ws_bytes);

/* Synchronise and return the replica's spectrum S (host [seg/2 + 1], zeros
 * before the first complete segment) averaged over the n_seg segments since
 * the recorder (re)started; restart != 0 then starts afresh (dropping a
 * partly filled segment).  Status errors as qtb_observables.  Either output
 * may be NULL. */
qtb_status qtb_vdos_read(qtb_ctx *ctx, int32_t replica, double *h_spec, int64_t *n_seg,
                         int32_t restart);

/* Stop recording (synchronises; the workspace is the caller's again). */
qtb_status qtb_vdos_detach(qtb_ctx *ctx, int32_t replica);

/*
 * Constant pressure.  Sec. 2.1 extends the equations of motion to the
 * isothermal-isobaric ensemble with a Langevin barostat (cited, not written
 * out), and Sec. 2.2 (Fig. 6) applies QTB-MD at constant pressure to the
 * lattice parameter of a crystal and its isotope shift.  Two isotropic
 * barostats, for classical replicas and ring polymers alike.  After every
 * step the pressure of the step just closed,
 *   p = (2 K - 2 U_spring + W / P) / (3 V),
 * is taken (the ring polymer's primitive pressure; K the kinetic energy of
 * all beads, U_spring the springs of eq. 3, W the pair virial sum of F(r) r
 * summed over the beads; for P = 1 the virial pressure), g is a unit
 * Gaussian of the replica's counter-based stream (step n, dof 0, tag 4), and
 * the update sets a scale factor s of the box lengths:
 *
 *   qtb_barostat: stochastic cell rescaling (Bernetti and Bussi, J. Chem.
 *   Phys. 153, 114107 (2020)), one Euler-Maruyama step of eps = ln V,
 *     d eps = -(beta_T / tau_p) (P0 - p) dt + sqrt(2 k_B T beta_T dt / (V tau_p)) g,
 *     s = e^{d eps / 3},  s_v1 = 1 / s,  s_v2 = 1;
 *   beta_T the isothermal compressibility (length^3 / energy).
 *
 *   qtb_barostat_piston: Langevin piston (Quigley and Probert, J. Chem.
 *   Phys. 120, 11432 (2004), in the Martyna-Tobias-Klein form): the strain
 *   ln(V) / 3 has momentum p_e and mass W_p = (3 N P + 3) k_B T tau_p^2
 *   (tau_p the piston's time scale), driven by G = 3V (p - P0) + (3/N_f) 2K,
 *   N_f = 3 N P, with friction gamma_p (1 / time):
 *     p_e <- c (p_e + dt G / 2) + sqrt((1 - c^2) W_p k_B T) g + dt G / 2,
 *     c = e^{-gamma_p dt},  s = e^{dt p_e / W_p},
 *     s_v1 = s_v2 = e^{-(1 + 3 / N_f) dt p_e / (2 W_p)}.
 *   The piston starts at rest; with gamma = gamma_p = 0 the dynamics keeps
 *   H + P0 V + p_e^2 / (2 W_p) up to the splitting error.
 *
 * The next step applies the scalings symmetrically: velocities times s_v1
 * before its first half-kick, every bead's normal-mode coordinates times
 * sqrt(s) before and after its A-O-A and the box times s with them (so its
 * forces see the scaled box and positions), velocities times s_v2 after its
 * closing half-kick.  Between steps the box is the one the positions were
 * taken in, and the factors wait as the barostat's state.  Both
 * sample V^N e^{-P0 V / k_B T} for an ideal gas.  The neighbour lists follow
 * the box by a scale factor and are rebuilt when the compression since
 * their build uses up half of the skin.  The list capacity is planned for
 * the initial density: compressing the box by more than about 20 % in
 * volume can overflow it (QTB_E_NOMEM at the next synchronising call).
 * Units: P0 in energy / length^3, tau_p in time.
 *
 * Enable with enable != 0, disable with 0 (either call disables whichever
 * barostat runs).  QTB_E_INVALID unless the potential is the pair potential,
 * the context has no surrogate buffers, the replica has three dimensions,
 * the one-kernel step (QTB_OPT_FUSE) is off, tau_p > 0, P0 finite, beta_T > 0
 * (cell rescaling) and gamma_p >= 0 (piston).  Synchronises.  While a
 * barostat runs every step's force pass also computes the observables.
 * Switching it off rebuilds the neighbour lists and recomputes the forces of
 * every replica at the current positions (as qtb_set_state does); the
 * scalings still pending from the last update are applied by the next step.
 * Force passes between steps (qtb_evaluate, qtb_set_state) see the box and
 * positions as they are, without the pending factors.
 *
 * qtb_get_box: synchronise and copy the replica's current box lengths
 * (host double[3]); status errors as qtb_observables.
 *
 * qtb_get_barostat_state / qtb_set_barostat_state: the part of a replica's
 * state that a checkpoint needs besides qtb_get_state and the box, host
 * double[4] = {p_e, s, s_v1, s_v2} (the piston momentum, 0 under cell
 * rescaling, and the scalings pending for the next step, 1 when none).
 * To resume exactly: create a context with the saved box, qtb_set_state,
 * enable the same barostat (which sets p_e = 0), then
 * qtb_set_barostat_state.  The setter returns QTB_E_INVALID for non-finite
 * values or non-positive scalings, and where no barostat can run (see
 * above).  Both synchronise.
 */
qtb_status qtb_barostat(qtb_ctx *ctx, int32_t replica, double P0, double tau_p, double beta_T,
                        int32_t enable);
qtb_status qtb_barostat_piston(qtb_ctx *ctx, int32_t replica, double P0, double tau_p,
                               double gamma_p, int32_t enable);
qtb_status qtb_get_box(qtb_ctx *ctx, int32_t replica, double *h_box);
qtb_status qtb_get_barostat_state(qtb_ctx *ctx, int32_t replica, double *h_state);
qtb_status qtb_set_barostat_state(qtb_ctx *ctx, int32_t replica, const double *h_state);

/*
 * Neighbour-list skin of one replica (replica = -1: every replica), pair
 * potential: 0 <= skin <= the potential's skin (which sizes the lists).  A
 * replica's list holds the pairs within r_cut + skin + the two atoms' bead
 * spreads and is rebuilt when an atom has moved more than skin / 2 from the
 * list's reference: a thin skin lists fewer pairs, a thick one rebuilds less
 * often (a cold replica moves little, a hot one much).  The forces are the
 * same (the order of the sums, and so the last bits, may differ).  The lists
 * are rebuilt and the forces recomputed at once; the state and step are
 * unchanged.  QTB_E_INVALID for a skin outside that range, other
 * potentials, or contexts with surrogate buffers.  Synchronises.
 */
qtb_status qtb_set_replica_skin(qtb_ctx *ctx, int32_t replica, double skin);

/*
 * Decomposition of the pair-force kernel (pair potential): waves_per_atom
 * wavefronts share one atom's neighbour list (1, 2 or 4), and each wavefront
 * holds G beads of it, G the widest power of two up to 8 that divides P, or
 * half of that (half_groups != 0; no effect where G = 1).  Every choice
 * computes the same forces; the order of the sums, and so the last bits,
 * depend on it.  The first qtb_step of a context times all choices on the
 * actual replicas and keeps the fastest (unless QTB_OPT_NO_AUTOTUNE),
 * separately for each force launch: a context whose replicas have different
 * bead-group widths G runs one launch per width, and each keeps its own
 * choice.  qtb_set_decomposition pins one choice for every launch instead
 * (for bit-reproducible runs across contexts) and skips that autotuning;
 * qtb_get_decomposition reports the choice of the launch with the most
 * workgroups.  QTB_E_INVALID for other values, a potential other than the
 * pair potential, with the surrogate attached anything but (1, 0), and half
 * groups with the one-kernel step.  Both synchronise.
 */
qtb_status qtb_set_decomposition(qtb_ctx *ctx, int32_t waves_per_atom, int32_t half_groups);
qtb_status qtb_get_decomposition(qtb_ctx *ctx, int32_t *waves_per_atom, int32_t *half_groups);
/*
 * The same for one force launch: group_width is the launch's whole bead-group
 * width G (1, 2, 4 or 8; the widest power of two up to 8 dividing the
 * replicas' P).  qtb_set_group_decomposition pins that launch's choice, keeps
 * the others' and skips the autotuning (with qtb_get_group_decomposition of
 * every width, an autotuned mix can be pinned again in another context).
 * QTB_E_INVALID where no launch has that width, for the values above, with
 * the surrogate attached or with the one-kernel step.  The setter
 * synchronises.
 */
qtb_status qtb_set_group_decomposition(qtb_ctx *ctx, int32_t group_width,
                                       int32_t waves_per_atom, int32_t half_groups);
qtb_status qtb_get_group_decomposition(qtb_ctx *ctx, int32_t group_width,
                                       int32_t *waves_per_atom, int32_t *half_groups);

/*
 * Diagnostics: while enabled, qtb_step records a HIP event pair around every
 * kernel phase on the context's stream (steps then run without graph
 * replay).  qtb_profile_read synchronises and returns, per phase, the total
 * GPU milliseconds and the number of launches since the last enable.
 * Phases: 0 white noise, 1 FIR, 2 update, 3 neighbour list, 4 forces,
 * 5 observable reduction.
 */
#define QTB_N_PHASES 6
qtb_status qtb_profile(qtb_ctx *ctx, int32_t enable);
qtb_status qtb_profile_read(qtb_ctx *ctx, double *ms, int64_t *launches);

/* ===================================================================
 * Learned force surrogate (not part of the paper's method: it replaces the
 * potential V of eq. 4 and eq. 8 by a sum of atomic energies, so the same
 * QTB / QTB-PIMD step runs on it).  Fixed architecture, two species:
 *   per centre atom i and neighbour species b, over every neighbour j (all
 *   periodic images) with r = |r_j - r_i| < r_c:
 *     f_c(r) = (cos(pi r / r_c) + 1) / 2
 *     phi_c(r) = exp(-(r - mu_c)^2 / (2 dr^2)) f_c(r), mu_c = r_min + c dr,
 *       dr = (r_c - r_min) / 31, c = 0..31
 *     psi_k(r) = exp(-(r - nu_k)^2 / (2 da^2)) f_c(r), nu_k = r_min + k da,
 *       da = (r_c - r_min) / 7, k = 0..7
 *     G[48 b + c]      = sum_j phi_c
 *     G[48 b + 32 + k] = |sum_j psi_k rhat_j|^2
 *     G[48 b + 40 + k] = ||sum_j psi_k (rhat_j rhat_j^T - I/3)||_F^2
 *   per centre species a: x = (G - mu_a) inv_sd_a, h1 = silu(W1 x + b1),
 *   h2 = silu(W2 h1 + b2), E_i = w3 . h2 + b3 + e0_a  (96 -> 64 -> 64 -> 1)
 *   V = sum_i E_i, F = -grad V.
 * Parameters (flat FP32, per species a in order): W1 [64][96], b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3 [1]: QTB_ML_PARAMS_PER_SPECIES values,
 * species 0 first.  The kernels use W1, W2, w3 rounded to BF16 (round to
 * nearest even) with FP32 arithmetic; biases stay FP32.  The normalisation
 * (FP64 host array, QTB_ML_NORM values): mu [2][96], inv_sd [2][96], e0 [2].
 * Training minimises, over the replicas of a context (frames, P = 1):
 *   L = w_E / B sum_f ((E_f - E_f^ref) / N_f)^2 + w_F / (3 sum_f N_f) sum |F - F^ref|^2
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master copy.
 * =================================================================== */
#define QTB_ML_FEATURES 96
#define QTB_ML_HIDDEN 64
#define QTB_ML_PARAMS_PER_SPECIES 10433
#define QTB_ML_PARAMS (2 * QTB_ML_PARAMS_PER_SPECIES)
#define QTB_ML_NORM (2 * 2 * QTB_ML_FEATURES + 2)

typedef struct qtb_ml qtb_ml; /* opaque */

/* Device bytes of a model (weights, Adam moments, gradient, normalisation). */
size_t qtb_ml_workspace_bytes(void);

/* Create a model in a caller-owned device buffer (256-byte aligned, at least
 * qtb_ml_workspace_bytes).  0 < r_min < r_c.  Weights start at zero, mu = 0,
 * inv_sd = 1, e0 = 0. */
qtb_status qtb_ml_create(qtb_ml **out, double r_cut, double r_min, void *d_workspace,
                         size_t ws_bytes, void *hip_stream);

/* Weights ~ N(0, 1/fan_in) from the library's Gaussian generator (tag 3,
 * step 0, dof = parameter index, stream 0), biases 0; resets Adam. */
qtb_status qtb_ml_init_params(qtb_ml *m, uint64_t seed);

/* Host copies in and out.  h_params: [QTB_ML_PARAMS] FP32 master values;
 * h_used (get only): the values the kernels use (W rounded to BF16);
 * h_norm: [QTB_ML_NORM] FP64.  Any pointer may be NULL. */
qtb_status qtb_ml_set_params(qtb_ml *m, const float *h_params, const double *h_norm);
qtb_status qtb_ml_get_params(qtb_ml *m, float *h_params, float *h_used, double *h_norm);

/* Step the context with the surrogate's forces (m = NULL: back to the pair
 * potential).  Every check_every steps (0 = never) the pair potential is
 * evaluated on the same positions and |F_ml - F_pair|^2 accumulated (the
 * pair potential checks the surrogate); read with qtb_ml_check.  Needs a
 * pair-potential context created with ml_r_cut >= the model's r_cut and
 * FP32 precision. */
qtb_status qtb_ml_attach(qtb_ctx *ctx, qtb_ml *m, int32_t check_every);

/* Surrogate forces (host [P][3][N]), per-bead energies (host [P]),
 * descriptors and dE/dG (host [P][N][96] FP32 each) of one replica at its
 * current positions.  Any output may be NULL.  Does not change the state. */
qtb_status qtb_ml_evaluate(qtb_ctx *ctx, qtb_ml *m, int32_t replica, double *h_force,
                           double *h_epot, float *h_desc, float *h_dEdG);

/* Set mu, inv_sd from the descriptors of every centre of every replica
 * (mean and 1 / max(standard deviation, 1e-3) per centre species and
 * feature) and e0 = mean over replicas of E_ref / N (both species).
 * d_eref: device [n_rep] FP64. */
qtb_status qtb_ml_fit_norm(qtb_ctx *ctx, qtb_ml *m, const double *d_eref);

/* One training step over every replica of ctx (each one frame, P = 1, at
 * its current positions): loss and gradient, then (update != 0) one Adam
 * step with learning rate lr.  d_eref: device [n_rep] FP64; d_fref: device
 * FP64, the replicas' [3][N] reference forces one after another.  loss_out
 * (nullable) receives L before the update; h_grad (nullable, host
 * [QTB_ML_PARAMS]) dL/dparams.  Needs QTB_OPT_ML_TRAIN. */
qtb_status qtb_ml_train_step(qtb_ctx *ctx, qtb_ml *m, const double *d_eref,
                             const double *d_fref, double w_E, double w_F, double lr,
                             int32_t update, double *loss_out, float *h_grad);

/* Checks since the last call: root mean square of F_ml - F_pair per
 * component, the same relative to the RMS of F_pair, and the number of
 * checks (host outputs; any may be NULL). */
qtb_status qtb_ml_check(qtb_ctx *ctx, int32_t replica, double *rmse, double *rel_rmse,
                        int64_t *n_checks);

const char *qtb_ml_last_error(const qtb_ml *m); /* never NULL */
void qtb_ml_destroy(qtb_ml *m);                  /* NULL is a no-op */

const char *qtb_last_error(const qtb_ctx *ctx); /* never NULL */
void qtb_destroy(qtb_ctx *ctx);                 /* NULL is a no-op */

/* Version string of the library build. */
const char *qtb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QTB_H */
