// qtb_internal.h -- structures shared by the host side of libqtb.so and its
// HIP kernels (gfx950).  Not part of the public ABI (include/qtb.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "qtb.h"

namespace qtb {

constexpr int kMaxSpecies = QTB_MAX_SPECIES;
constexpr int kPairs = kMaxSpecies * kMaxSpecies;
constexpr int kDofTile = 256;      // replica dof ranges are padded to this
constexpr int kWavesPerAtomDefault = 2;  // force kernel: wavefronts per atom (1, 2, 4)
// ke, U, spring, virial, x2, pair virial, centroid kinetic energy
constexpr int kNobs = 7;
// sample accumulators: the kNobs slots, then (pair potential) volume and the
// pressure of each sample
constexpr int kAcc = 9;
// atoms per chunk of the centroid kinetic-energy sums
constexpr int kCentroidChunk = 256;

// Pair potential in the form the force kernels evaluate:
//   F(r) = -dV/dr = Arho e^{-r irho} - C6 r^-7
//                   + kqq [erfc(a r)/r^2 + g e^{-a^2 r^2}/r] + F0
//   V(r) = A e^{-r irho} - C r^-6 + kqq erfc(a r)/r - F0 r + E0
// where the constants fold the shifted-force Buckingham and the damped
// shifted force Coulomb terms (both vanish with their slope at r_cut).
template <typename T>
struct PairParam {
    T Arho, irho, C6, kqq, F0, A, C, E0;
    T irho2;  // irho log2(e): e^{-r irho} = 2^{-r irho2}
};

// erfc(x) e^{x^2} on [0, alpha r_cut] as a polynomial of fixed degree in
// s = x (2/x_max) - 1, fitted on the host (Chebyshev interpolation, then
// monomial form).  ex_deg is 10 or kErfcxMaxDeg; 0 marks a range the fit
// cannot cover to 5e-7, where the FP32 kernel calls erfcf instead.
constexpr int kErfcxMaxDeg = 14;

// The Coulomb part of F(r) / kqq, erfc(a r) / r^2 + g e^{-a^2 r^2} / r, is
// phi(a r) / r^2 with phi(x) = erfc(x) + (2 x / sqrt(pi)) e^{-x^2}
// = 1 - (4 / sqrt(pi)) int_0^x t^2 e^{-t^2} dt = 1 + x^3 psi(x^2), psi entire;
// the FP32 force kernels take phi = 1 + (r r^2) ph(s), s = r^2 ph_s - 1,
// ph a polynomial of degree ex_deg fitted on the host (a^3 folded in).
template <typename T>
struct PairTable {
    PairParam<T> p[kPairs];
    T alpha, g, rc2;
    T a2l;     // alpha^2 log2(e): e^{-a^2 r^2} = 2^{-r^2 a2l}
    T s_mul;   // 2 alpha / x_max
    T ex[kErfcxMaxDeg + 1];
    T ph[kErfcxMaxDeg + 1];
    T ph_s;    // 2 / r_cut^2
    int32_t ex_deg;
    int32_t n_species;
};

// Per-replica description the kernels read (device copy in the workspace).
struct RepDev {
    double* pos;         // [P][dims][N]
    double* vel;         // [P][dims][N]
    void* force;         // T [P][dims][N]
    // Data that other atoms read are kept twice, by step parity (sync step
    // counter & 1), so one kernel can read a step's values while it writes
    // the next step's:
    void* ub[2];         // T4 [N][P]: position minus reference, species bits in .w
    double* cnb[2];      // [3][N] bead centroids
    double* devn[2];     // [N] largest bead-to-centroid distance
    double* rrefb[2];    // [3][N] reference positions (bead centroids at the last build)
    double* devbb[2];    // [N] bead spread at the last build
    double* r0;          // [P][dims][N] positions given at init / set_state
    double* eatom;       // [P][N] per-atom energies (evaluate mode)
    const int32_t* species;  // [N]
    const double* homega;    // [N]
    // T4 [N][maxnb]: reference displacement d_ij, j bits in .w; the core
    // entries (reference distance below r_cut) at slots 0 .. nb_core - 1 in
    // scan order, the shell entries at slots maxnb - 1, maxnb - 2, ... in
    // scan order, nb_count entries in all
    void* nb_entries;
    int32_t* nb_count;       // [N]
    int32_t* nb_core;        // [N]
    const double* nm;        // [P][P] orthonormal normal-mode matrix C[s][k]
    const double* ring;      // [3][P]: cos(w h), sin(w h)/w, -w sin(w h), h = dt/2
    int32_t* rflag;          // [3] neighbour-list rebuild flags, by step mod 3
    double* tbox;            // [ceil(N/kListTile)][8] per candidate tile: centroid
                             // bounds lo xyz, hi xyz, largest spread (list kernel)
    int64_t dof_off;         // first column in the global noise arrays
    int64_t step_off;        // replica step = global step + step_off
    int32_t N, P, dims, maxnb;
    int32_t two_nf, noise, obs_block0, obs_nblocks;
    double box[3];
    // half_skin: the displacement from the reference that triggers a list
    // rebuild (lowered under the barostat while the box is compressed)
    double c1, kT, omega_P, half_skin, r_cs;  // r_cs = r_cut + skin
    double r_cut;
    double kick[kMaxSpecies];   // dt / (2 P m mu)
    double sigma[kMaxSpecies];  // sqrt((1 - c1^2) / (m mu))
    double mmu[kMaxSpecies];    // m mu
    double osV0[kMaxSpecies];   // on-site kinds: energy scale V0
    double osd[kMaxSpecies];    // on-site kinds: length scale d
    uint64_t seed;
    uint32_t stream;
    int32_t pad;
    // descriptor-MLP surrogate (null unless the context reserved it)
    void* ml_nb;          // T4 [N][maxml]: like nb_entries, within r_ml + skin + margins
    int32_t* ml_nc;       // [N]
    int32_t* ml_rev;      // [N][maxml]: slot of the reverse entry in the neighbour's list
    float* ml_G;          // [P][N][96] descriptors
    float* ml_aux;        // [P][N][144] A1 [2][8][3], A2 [2][8][6]
    float* ml_g;          // [P][N][96] dE_i/dG_i
    float* ml_y;          // [P][N] atomic energies without e0
    float* ml_fpair;      // float4 [P][N][maxml]: dE_i/dd_ij per list entry (in range)
    int32_t* ml_in;       // [P][N][maxml]: list slots within r_ml this step
    int32_t* ml_nin;      // [P][N]
    float* ml_v;          // [P][N][96] training: J (u_j - u_i)
    float* ml_u;          // [P][3][N] training: dL/dF
    float* ml_adj;        // [P][N][kMlAdj] training: per-centre adjoint rows
    double* ml_ebar;      // [1] training: dL/dE of this replica
    int32_t maxml;
    int32_t ml_pad;
    double ml_rcs;        // r_ml + skin
    // velocity recorder (P = 1; null when off): every sample also stores the
    // velocities, row (vt_n mod vt_cap) of vt [vt_cap][dims][N]; the sample
    // reduction advances vt_n
    double* vt;
    int64_t* vt_n;
    int32_t vt_cap;
    // isotropic barostat after every step (pair potential, any P): 0 off,
    // 1 stochastic cell rescaling, 2 Langevin piston; box[] above is then
    // the current box, updated on the device
    int32_t npt;
    double npt_P0, npt_tau;            // target pressure, relaxation / piston time
    double npt_beta;                   // compressibility (cell rescaling)
    double npt_W, npt_gp, npt_pe;      // piston mass, friction, momentum
    // scalings the last barostat update left for the next step (1 when
    // none): velocities before its first kick (sv1) and after its closing
    // kick (sv2), normal-mode positions by sqrt(sr) before and after its
    // A-O-A; its force pass and sample use box and npt_S times sr, which the
    // barostat kernel commits at its end.  Every step applies them (a
    // multiplication by 1 is exact); between steps box, npt_S and the
    // positions agree.
    double npt_sr, npt_sv1, npt_sv2;
    double dt;
    // length scale of the box relative to the last list build (1 without a
    // barostat): list entries and reference centroids keep the geometry of
    // the build; a pair's displacement is npt_S * entry + u_i - u_j with
    // u = r - npt_S * reference
    double npt_S;
    double half_skin0;                 // half the skin
    int32_t list_built;                // the list kernel rebuilt inside this step (barostat)
};

// ------------------------------------------------ descriptor-MLP surrogate
constexpr int kMlSpecies = 2;
constexpr int kMlRad = 32;                       // radial channels per species
constexpr int kMlAng = 8;                        // angular channels (l = 1, 2 each)
constexpr int kMlFeatSp = kMlRad + 2 * kMlAng;   // 48
constexpr int kMlFeat = kMlSpecies * kMlFeatSp;  // 96
constexpr int kMlHidden = 64;
constexpr int kMlAux = kMlSpecies * kMlAng * 9;  // A1 (3) + A2 (6) per species, channel
// one species' trainable block: W1 [64][96], b1, W2 [64][64], b2, w3, b3
constexpr int kMlOffW1 = 0;
constexpr int kMlOffB1 = kMlOffW1 + kMlHidden * kMlFeat;
constexpr int kMlOffW2 = kMlOffB1 + kMlHidden;
constexpr int kMlOffB2 = kMlOffW2 + kMlHidden * kMlHidden;
constexpr int kMlOffW3 = kMlOffB2 + kMlHidden;
constexpr int kMlOffB3 = kMlOffW3 + kMlHidden;
constexpr int kMlParamsSp = kMlOffB3 + 1;        // 10433
constexpr int kMlParams = kMlSpecies * kMlParamsSp;
// adjoint row of one centre (training): xd[96] z1b[64] z1db[64] h1[64]
// h1d[64] z2b[64] z2db[64] t3[64] e[1] (pad to 576)
constexpr int kMlAdj = 576;
// workgroups of the weight-gradient sums (each keeps partials per species)
constexpr int kWgBlocks = 256;

// Model as the kernels see it (device pointers into the model workspace).
struct MlDev {
    const uint16_t* wq;     // [kMlParams] BF16 weights (biases too, only read as FP32)
    const float* master;    // [kMlParams] FP32 master copy (biases are read from here)
    const float* mu;        // [2][96]
    const float* inv_sd;    // [2][96]
    const double* e0;       // [2]
    float r_cut, r_min;
    float mu0, dr, eta_r;   // radial grid
    float nu0, da, eta_a;   // angular grid
};

// Workgroups are dealt to the 8 XCDs in turn (hardware block b runs on XCD
// b % 8), each with its own L2.  Kernels that gather from neighbouring atoms
// process table entry xcd_block() instead of blockIdx.x, so that each XCD
// works through one contiguous eighth of the table and its L2 holds the
// neighbours of its own region.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_block()
{
    const int b = blockIdx.x, n = gridDim.x;
    const int q = n >> 3, r = n & 7, x = b & 7, pos = b >> 3;
    return x < r ? x * (q + 1) + pos : r * (q + 1) + (x - r) * q + pos;
}

// Work tables: replica and first atom per block (uniform per block).
struct BlockEntry {
    int32_t rep;
    int32_t atom0;
    int32_t group;   // bead group (force kernel)
    int32_t pad;
};

// FIR tile descriptor: one per kDofTile columns.
struct FirTile {
    int32_t rep;
    int32_t two_nf;
    int32_t taps_off;   // offset (elements) of this replica's taps
    int32_t pad;
};

enum StatusBits : int32_t {
    kStatusNonfinite = 1,
    kStatusNbOverflow = 2,
    kStatusMlList = 8,
    kStatusRange = 16,  // pair range beyond kMaxImages periodic images (diverged state)
};
// Counts of atom i's list after the build (one lane calls it); an overflowing
// list is left empty (every entry read is then a written one) and reported.
__device__ __forceinline__ void list_finish(int32_t* nb_count, int32_t* nb_core, int i, int maxnb,
                                            int ncore, int nshell, int32_t* status)
{
    if (ncore + nshell > maxnb) {
        nb_count[i] = 0;
        nb_core[i] = 0;
        atomicOr(status, kStatusNbOverflow);
    } else {
        nb_count[i] = ncore + nshell;
        nb_core[i] = ncore;
    }
}

// Periodic images searched per direction when a list is built: enough for
// any box wider than r_cut / 8; a larger range (a diverging trajectory's
// bead spread) is clamped to it and reported through kStatusRange, so the
// search always ends.
constexpr int kMaxImages = 8;
// Candidate atoms per tile of the list kernel's scan (staged in LDS).
constexpr int kListTile = 256;
// Tiles whose out-of-range verdicts a list block precomputes in LDS (replicas
// of up to kListTile * kMaxListTiles atoms; larger ones test tile by tile).
constexpr int kMaxListTiles = 4096;
// Replicas above this many atoms build their lists in the list kernel, whose
// scan skips candidate tiles out of range by their bounding boxes; smaller
// ones rebuild inside the force kernel (one launch less per step).
constexpr int kInlineRebuildMaxAtoms = 16384;

// One step of a list build: each lane holds at most one accepted candidate
// (hit), stored with ballot compaction in lane order; core entries
// (reference distance below r_cut) go to slots ncore, ncore + 1, ...,
// shell entries to slots maxnb - 1 - nshell, maxnb - 2 - nshell, ....  A
// store that would cross into the other range is dropped: the total then
// exceeds maxnb and list_finish reports the overflow.
template <typename V>
__device__ __forceinline__ void list_push(V* __restrict__ ent, int maxnb, bool hit, bool core,
                                          const V& v, uint64_t below, int& ncore, int& nshell)
{
    const uint64_t mc = __ballot(hit && core), ms = __ballot(hit && !core);
    const int nc = __popcll(mc), ns = __popcll(ms);
    if (hit) {
        if (core) {
            const int slot = ncore + __popcll(mc & below);
            if (slot < maxnb - (nshell + ns)) ent[slot] = v;
        } else {
            const int slot = maxnb - 1 - (nshell + __popcll(ms & below));
            if (slot >= ncore + nc) ent[slot] = v;
        }
    }
    ncore += nc;
    nshell += ns;
}

// Image range ceil(R / L - 1/2) along one direction, clamped to
// [0, kMaxImages] (also for non-finite R); over is set when clamped.
__device__ __forceinline__ int image_range(double R, double inv_L, bool& over)
{
    const double m = ceil(R * inv_L - 0.5);
    if (!(m <= (double)kMaxImages)) {
        over = true;
        return kMaxImages;
    }
    return m > 0.0 ? (int)m : 0;
}
// status[kAnyRebuild + step mod 3]: some replica needs its neighbour list rebuilt
constexpr int kAnyRebuild = 4;

// Step bookkeeping shared by the kernels: the step n of the positions a
// kernel works on is *clk + off (clk: the device noise clock, the first step
// of the current noise block, so a captured block replays with the right
// steps) or off alone (clk null: launches outside a block).
struct StepRef {
    const int64_t* clk;
    int64_t off;
};
struct StepIdx {
    int p;  // parity n & 1: which copy of the double-kept data is current
    int f;  // n mod 3: which rebuild flag is current
};
__device__ __forceinline__ StepIdx step_index(const StepRef r)
{
    const int64_t n = (r.clk ? *r.clk : 0) + r.off;
    const int64_t m = n % 3;
    return StepIdx{(int)(n & 1), (int)(m < 0 ? m + 3 : m)};
}

// Kernel-side flags of the force kernels.
// kCompare: leave force and state untouched, accumulate |F - F_stored|^2 and
// |F|^2 into observable slots 0 and 1 (the surrogate's check).
// kPressure: only what a barostat needs of a step that does not sample:
// kinetic energy, springs and pair virial into slots 0, 2 and 5.
enum ForceFlags : int32_t { kKick = 1, kSample = 2, kEvaluate = 4, kCompare = 8, kPressure = 16 };

// Profiling: when set, the next launch time-stamps these events from its own
// dispatch packet (no marker packets around the kernel), then clears them.
struct LaunchStamp {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchStamp& launch_stamp();

template <typename F, typename... Args>
inline void launch(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st, Args... args)
{
    LaunchStamp& ls = launch_stamp();
    if (ls.start) {
        hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ls.start, ls.stop, 0, args...);
        ls = LaunchStamp{};
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    }
}

// ---------------------------------------------------------------- launchers
// noise.hip
// White-noise rows clock+off .. clock+off+rows-1 into the ring, in the
// layout of the FIR mode (FP64, FP32 rows, or BF16 hi/lo planes of 8-row
// groups; see fir.hip).
void launch_gen_white(hipStream_t st, const RepDev* reps, const FirTile* tiles, void* ring,
                      int fir_mode, const int64_t* clock, int64_t off, int rows, int R,
                      int64_t n_cols);
void launch_clock(hipStream_t st, int64_t* clock, int64_t v, bool add);
// Block noise (eq. 9, n = 2^L2 steps per block, n >= K): makes the noise
// blocks that the K-step noise block starting at *clock needs and has not got,
// in the [2 n][n_cols] buffer zeta (half B mod 2 holds block B); marker [2]
// names the block each half holds.  amp: per replica [amp_stride] amplitudes
// A_j, j = 0 .. n/2; tw: e^{-2 pi i k / n}, k < n/2 (double2).
void launch_eq9(hipStream_t st, bool fp64, const RepDev* reps, const FirTile* tiles,
                const double* amp, int amp_stride, const double* tw, int n, void* zeta,
                int64_t n_cols, const int64_t* clock, int64_t* marker, int K);
void launch_eq9_invalidate(hipStream_t st, int64_t* marker);
// Barostat update after the force pass of step n (sync gives n; partials
// hold that pass's block sums): box and list scale take the factor step n
// applied; for replicas with npt set, the scalings step n + 1 applies and a
// list rebuild flagged for it; for the others, the factors reset to 1.
void launch_barostat(hipStream_t st, RepDev* reps, int n_rep, const double* partials,
                     StepRef sync, int32_t* status);
int eq9_columns(int n);
void launch_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, uint32_t tag, int64_t n0,
                     int64_t n_rows, uint32_t d0, uint32_t n_dof, double* out);
// fir.hip
void launch_fir(hipStream_t st, int mode, int K, const FirTile* tiles, int n_tiles,
                const void* taps, const void* ring, void* zeta, int64_t n_cols, const int64_t* nb,
                int R, int max_two_nf);
int fir_pad();
size_t fir_lds_bytes(int mode, int max_two_nf);
// update.hip
// P: the largest bead count, threads: update_threads(largest dims P).
// zmod > 0 (block noise): zeta_row is the base of a [zmod][n_cols] ring and
// the step's row is (step mod zmod); zmod = 0: zeta_row is the step's row.
void launch_update(hipStream_t st, bool fp64, bool pair, int P, int threads,
                   const RepDev* reps, const BlockEntry* blocks, int n_blocks,
                   const void* zeta_row, int32_t* status, StepRef sync, int64_t zmod,
                   int64_t n_cols);
int update_threads(int max_dims_beads);
int update_block_atoms(int dims, int P, int threads);
// nlist.hip
void launch_nlist(hipStream_t st, bool fp64, const RepDev* reps, const BlockEntry* blocks,
                  int n_blocks, const BlockEntry* tiles, int n_tiles, int32_t* status,
                  bool centroids, StepRef sync, bool in_step = false);
void launch_mark_rebuild(hipStream_t st, const RepDev* reps, int n_rep, int32_t* status,
                         StepRef sync);
// forces.hip
// clear: reset this step's rebuild flags (the list is up to date).
void launch_forces_pair(hipStream_t st, bool fp64, int G, int W, const RepDev* reps,
                        const BlockEntry* blocks, int n_blocks, const void* table,
                        int32_t flags, double* partials, int clear, int n_rep,
                        int32_t* status, StepRef sync);
// One kernel per step (pair potential, P <= 8, bead group G = P): rebuild
// the lists if flagged, forces, closing half-kick, sampling, then the next
// step's opening half-kick, normal-mode A-O-A with zeta_row.
void launch_step_pair(hipStream_t st, bool fp64, int G, int W, const RepDev* reps,
                      const BlockEntry* blocks, int n_blocks, const void* table, int32_t flags,
                      double* partials, int n_rep, int32_t* status, StepRef sync,
                      const void* zeta_row);
void launch_forces_onsite(hipStream_t st, bool fp64, int kind, const RepDev* reps,
                          const BlockEntry* blocks, int n_blocks, int32_t flags,
                          double* partials);
// tick: a sample (advances the velocity recorders), not a surrogate check;
// pair: the pair potential (the volume and pressure slots are filled).
// cpart (may be null): [n_rep][cchunks] scratch; when given, the kinetic
// energy of the ring-polymer centroids is summed from the velocities first
// (chunks of kCentroidChunk atoms, max_atoms the largest replica) and added
// to slot 6; null: slot 6 of the partials already holds it.
void launch_obs_reduce(hipStream_t st, const RepDev* reps, int n_rep, const double* partials,
                       double* acc, int32_t* counts, bool tick, bool pair, double* cpart,
                       int cchunks);
void launch_fill(hipStream_t st, void* p, int64_t n_words, int32_t value);
// vdos.hip
constexpr int kVdosMinSeg = 16, kVdosMaxSeg = 4096;  // samples per segment, powers of two
struct VdosPlan {
    int seg, L2, cw, n_groups, grid, nk;  // cw complex columns per group, nk = seg/2 + 1
    int stage_rows;                       // rows of the first summing pass (0: one pass)
};
VdosPlan vdos_plan(int n_dof, int seg);
void launch_vdos_twiddle(hipStream_t st, double* tw, int seg);
// One segment: sample t of dof j at v[t ts + j js]; spec[k] = (accumulate ?
// spec[k] : 0) + scale * sum_j w_j |V_jk|^2, given sqrt_w[j] = sqrt(w_j).
// partials: plan.grid x plan.nk doubles, stage: plan.stage_rows x plan.nk.
void launch_vdos_segment(hipStream_t st, const VdosPlan& p, const double* v, int64_t ts,
                         int64_t js, int n_dof, const double* sqrt_w, const double* tw,
                         double* partials, double* stage, double* spec, double scale,
                         bool accumulate);
// sqrt_w of a replica's dofs ([dims][N]: the square roots of the masses)
void launch_vdos_weights(hipStream_t st, const RepDev* reps, int r, int n_dof, double* sqrt_w);
void launch_vdos_sqrt(hipStream_t st, const double* w, int n, double* sqrt_w);
// the error message of calls without a context (qtb_last_error(NULL))
void set_static_error(const std::string& m);
// ml.hip
void launch_ml_lists(hipStream_t st, bool fp64, const RepDev* reps, const BlockEntry* nl_blocks,
                     int n_nl, int32_t* status, StepRef sync);
void launch_ml_forward(hipStream_t st, bool fp64, const RepDev* reps, const MlDev& m,
                       const BlockEntry* cblocks, int n_cblocks, const BlockEntry* mblocks,
                       int n_mblocks, int n_rep, int32_t* status, StepRef sync);
// apb: atoms per block of the force table in use (4 / waves per atom)
void launch_ml_gather(hipStream_t st, bool fp64, int G, int apb, const RepDev* reps,
                      const MlDev& m, const BlockEntry* blocks, int n_blocks, int32_t flags,
                      double* partials);
void launch_ml_loss(hipStream_t st, const RepDev* reps, int n_rep, const double* eref,
                    const double* fref, const int64_t* fref_off, double w_E, double w_F,
                    double n_atoms_total, double* loss_parts);
void launch_ml_jvp(hipStream_t st, bool fp64, const RepDev* reps, const MlDev& m,
                   const BlockEntry* cblocks, int n_cblocks, StepRef sync);
void launch_ml_train_mlp(hipStream_t st, const RepDev* reps, const MlDev& m,
                         const BlockEntry* mblocks, int n_mblocks);
// part: kWgBlocks x kMlParams floats of scratch (partial sums)
void launch_ml_wgrad(hipStream_t st, const RepDev* reps, const MlDev& m,
                     const BlockEntry* mblocks, int n_mblocks, float* part, float* grad);
void launch_ml_adam(hipStream_t st, float* master, uint16_t* wq, float* mom1, float* mom2,
                    const float* grad, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2);
void launch_ml_round(hipStream_t st, const float* master, uint16_t* wq, int n);
void launch_ml_init(hipStream_t st, float* master, uint64_t seed);
void launch_ml_stats(hipStream_t st, const RepDev* reps, int n_rep, double* stats);

}  // namespace qtb
