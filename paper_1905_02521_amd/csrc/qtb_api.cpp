// qtb_api.cpp -- the C ABI of libqtb.so (include/qtb.h): argument checks,
// workspace layout, per-replica tables, and the step schedule.  All device
// memory comes from the caller's workspace; all work goes on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "qtb_internal.h"

namespace qtb {
double design_theta(double omega, double T, double hbar, double kB);
void design_taps(int kind, double T, int P, double dt, int two_nf, double hbar, double kB,
                 double* out);
void design_spectrum(int kind, double T, int P, double dt, int two_nf, double hbar, double kB,
                     double* S);
}  // namespace qtb

using namespace qtb;

namespace {

constexpr double kPi = 3.141592653589793238462643383;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Region {
    size_t off = 0, bytes = 0;
};

// Everything the workspace holds, in the order it is carved.
struct Layout {
    size_t total = 0;
    Region reps, status, rebuild, tiles, taps, ring, zeta, partials, acc, counts, pairtab, clock;
    Region cpart;  // [n_rep][cchunks] centroid kinetic energy per chunk of atoms
    Region eq9amp, eq9tw, eq9mark;  // block noise (eq. 9): amplitudes, twiddles, block markers
    Region blk_upd, blk_nl, blk_force, blk_tb;
    // surrogate (ml_r_cut > 0)
    Region blk_mlc, blk_mlm, ml_acc, ml_counts, ml_loss, ml_stats, ml_foff, ml_wpart;
    struct Per {
        Region force, r0, eatom, species, homega, nb, nbc, nbcore, nm, ring;
        Region u[2], rref[2], cnow[2], dev[2], devb[2];  // by step parity
        Region tbox;
        Region mlnb, mlnc, mlrev, mlG, mlaux, mlg, mly, mlfp, mlin, mlnin, mlv, mlu, mladj, mlebar;
    };
    std::vector<Per> per;
    // derived sizes
    int64_t n_cols = 0;
    int R = 0, K = 0, max_two_nf = 0, taps_stride = 0;
    int cchunks = 1;  // chunks of kCentroidChunk atoms in the largest replica
    bool eq9 = false;  // block noise: zeta is a [2 n][n_cols] ring, n = max_two_nf
    int64_t zeta_rows = 0;
    std::vector<int64_t> dof_off;
    std::vector<int> maxnb, maxml;
    bool ml = false, ml_train = false;
    std::vector<BlockEntry> mlc, mlm;     // surrogate: centre blocks, network tiles
    std::vector<int64_t> foff;            // offsets of the replicas' reference forces
    std::vector<BlockEntry> upd, nl, force;   // force: table of the chosen W
    std::vector<BlockEntry> tb;               // candidate tiles of the list kernel
    int upd_threads = 128;
    // force tables for every decomposition the autotuner tries: index
    // 2 wi + gi, W = 2^wi wavefronts per atom, gi = 0 the widest bead group
    // G that divides P (up to 8), gi = 1 half of it (G / 2 beads per
    // wavefront and twice the groups; the same as gi = 0 where G = 1)
    std::vector<BlockEntry> force_w[6];
    std::vector<std::pair<int, std::pair<int, int>>> force_groups_w[6];
    std::vector<int> obs_b0_w[6], obs_nb_w[6];
    size_t max_force_blocks = 1;
    std::vector<std::pair<int, std::pair<int, int>>> upd_groups;    // P -> [b0, b1)
    std::vector<std::pair<int, std::pair<int, int>>> force_groups;  // G -> [b0, b1)
    std::vector<int> force_group_W;   // waves per atom of each force group's launch
    std::vector<int> force_group_t;   // the decomposition table each group came from
    std::vector<int> obs_b0, obs_nb;
    std::vector<FirTile> tilev;
};

int bead_group(int P)
{
    int G = 1;
    while (G * 2 <= 8 && P % (G * 2) == 0) G *= 2;
    return G;
}

size_t add(size_t& cur, Region& r, size_t bytes)
{
    r.off = cur;
    r.bytes = bytes;
    cur += align_up(bytes);
    return r.off;
}

const char* check_inputs(const qtb_potential* pot, const qtb_replica* reps, int n_rep,
                         const qtb_options* opt)
{
    if (!pot || !reps || !opt) return "null argument";
    if (n_rep < 1) return "n_rep must be >= 1";
    if (pot->kind < QTB_POT_PAIR || pot->kind > QTB_POT_DOUBLE_WELL) return "unknown potential kind";
    if (pot->n_species < 1 || pot->n_species > QTB_MAX_SPECIES) return "n_species out of range";
    if (!pot->mass) return "mass table missing";
    for (int a = 0; a < pot->n_species; ++a)
        if (!(pot->mass[a] > 0.0)) return "masses must be > 0";
    if (pot->kind == QTB_POT_MORSE || pot->kind == QTB_POT_DOUBLE_WELL) {
        if (!pot->onsite_V0 || !pot->onsite_d) return "on-site potential tables missing";
        for (int a = 0; a < pot->n_species; ++a)
            if (!(pot->onsite_V0[a] > 0.0) || !(pot->onsite_d[a] > 0.0))
                return "onsite_V0 and onsite_d must be > 0";
    }
    if (pot->kind == QTB_POT_PAIR) {
        if (!pot->charge || !pot->buck_A || !pot->buck_rho || !pot->buck_C)
            return "pair potential tables missing";
        if (!(pot->r_cut > 0.0)) return "r_cut must be > 0";
        if (!(pot->skin >= 0.0)) return "skin must be >= 0";
        if (!(pot->dsf_alpha >= 0.0)) return "dsf_alpha must be >= 0";
        const int ns = pot->n_species;
        for (int ab = 0; ab < ns * ns; ++ab)
            if (pot->buck_A[ab] != 0.0 && !(pot->buck_rho[ab] > 0.0)) return "buck_rho must be > 0";
    }
    if (!(opt->hbar > 0.0) || !(opt->kB > 0.0) || !(opt->mass_unit > 0.0)) return "bad units";
    if (opt->prec != QTB_PREC_FP32 && opt->prec != QTB_PREC_FP64) return "bad precision";
    if (opt->fir < 0 || opt->fir > 3) return "bad FIR mode";
    if ((opt->prec == QTB_PREC_FP64) != (opt->fir == QTB_FIR_FP64))
        return "FP64 precision pairs with the FP64 FIR, FP32 with the FP32/BF16 FIRs";
    if (opt->fir_block_K != 64 && opt->fir_block_K != 128 && opt->fir_block_K != 256)
        return "fir_block_K must be 64, 128 or 256";
    if (opt->obs_every < 0) return "obs_every must be >= 0";
    if (!(opt->ml_r_cut >= 0.0)) return "ml_r_cut must be >= 0";
    if (opt->ml_r_cut > 0.0) {
        if (pot->kind != QTB_POT_PAIR) return "the surrogate needs the pair-potential kind";
        if (opt->ml_r_cut > pot->r_cut) return "ml_r_cut must not exceed r_cut";
        if (pot->n_species > 2) return "the surrogate has two species";
    }
    if (opt->max_two_nf < 2 || (opt->max_two_nf & (opt->max_two_nf - 1)) || opt->max_two_nf > 8192)
        return "max_two_nf must be a power of two in [2, 8192]";
    if (opt->fir != QTB_FIR_FP64 && opt->max_two_nf > 4096) return "BF16/FP32 FIR: max_two_nf <= 4096";
    if (opt->flags & QTB_OPT_NOISE_BLOCKS) {
        const int n = opt->max_two_nf;
        if ((n & (n - 1)) || n < opt->fir_block_K || n > 4096)
            return "block noise: max_two_nf must be a power of two in [fir_block_K, 4096]";
        if (opt->flags & QTB_OPT_FUSE) return "block noise does not combine with the one-kernel step";
    }
    for (int r = 0; r < n_rep; ++r) {
        const qtb_replica& R = reps[r];
        if (R.n_atoms < 1 || R.n_beads < 1 || R.n_beads > 64) return "replica sizes out of range";
        if (R.n_dims != 1 && R.n_dims != 3) return "n_dims must be 1 or 3";
        if (pot->kind == QTB_POT_PAIR && R.n_dims != 3) return "pair potential needs n_dims = 3";
        if (R.noise < 0 || R.noise > 2) return "bad noise kind";
        if (!(R.T > 0.0) || !(R.gamma >= 0.0) || !(R.dt > 0.0)) return "T, gamma, dt out of range";
        if (!R.species || !R.d_pos || !R.d_vel) return "replica pointers missing";
        if (pot->kind == QTB_POT_HARMONIC && !R.harm_omega) return "harmonic frequencies missing";
        for (int i = 0; i < R.n_atoms; ++i)
            if (R.species[i] < 0 || R.species[i] >= pot->n_species) return "species out of range";
        if (pot->kind == QTB_POT_PAIR) {
            for (int a = 0; a < 3; ++a)
                if (!(R.box[a] > 0.0)) return "box lengths must be > 0";
            if ((int64_t)R.n_atoms >= (1 << 30)) return "too many atoms";
        }
        if ((int64_t)R.n_dims * R.n_atoms * R.n_beads > (int64_t)1 << 31) return "too many dofs";
    }
    return nullptr;
}

int estimate_maxnb(const qtb_potential* pot, const qtb_replica& R)
{
    // bead spread widens the list radius (r_cut + skin + dev_i + dev_j)
    const double Rl = pot->r_cut + pot->skin + (R.n_beads > 1 ? 1.0 : 0.2);
    const double vol = R.box[0] * R.box[1] * R.box[2];
    const double n_est = 4.0 / 3.0 * kPi * Rl * Rl * Rl * R.n_atoms / vol;
    int m = (int)std::ceil(1.3 * n_est + 48.0);
    m = (m + 63) / 64 * 64;
    return std::max(m, 64);
}

int estimate_maxml(const qtb_potential* pot, const qtb_options* opt, const qtb_replica& R,
                   int maxnb)
{
    const double Rl = opt->ml_r_cut + pot->skin + (R.n_beads > 1 ? 1.0 : 0.2);
    const double vol = R.box[0] * R.box[1] * R.box[2];
    const double n_est = 4.0 / 3.0 * kPi * Rl * Rl * Rl * R.n_atoms / vol;
    int m = (int)std::ceil(1.3 * n_est + 48.0);
    m = (m + 63) / 64 * 64;
    return std::min(std::min(std::max(m, 64), maxnb), 512);
}

void plan(const qtb_potential* pot, const qtb_replica* reps, int n_rep, const qtb_options* opt,
          Layout& L)
{
    const bool pair = pot->kind == QTB_POT_PAIR;
    const size_t ts = opt->prec == QTB_PREC_FP64 ? 8 : 4;   // force / u element
    const size_t zs = opt->fir == QTB_FIR_FP64 ? 8 : 4;     // ring / zeta element
    L.K = opt->fir_block_K;
    L.max_two_nf = opt->max_two_nf;
    L.eq9 = (opt->flags & QTB_OPT_NOISE_BLOCKS) != 0;
    L.zeta_rows = L.eq9 ? 2 * (int64_t)opt->max_two_nf : L.K;
    L.R = (L.K + opt->max_two_nf + 15) / 16 * 16;  // ring rows (BF16 planes: groups of 8)
    L.taps_stride = opt->max_two_nf + 2 * fir_pad();
    L.per.assign(n_rep, {});
    L.dof_off.assign(n_rep, 0);
    L.maxnb.assign(n_rep, 0);
    L.maxml.assign(n_rep, 0);
    L.ml = pair && opt->ml_r_cut > 0.0;
    L.ml_train = L.ml && (opt->flags & QTB_OPT_ML_TRAIN);
    int64_t cols = 0;
    for (int r = 0; r < n_rep; ++r) {
        const qtb_replica& R = reps[r];
        L.dof_off[r] = cols;
        const int64_t D = (int64_t)R.n_dims * R.n_atoms * R.n_beads;
        cols += (D + kDofTile - 1) / kDofTile * kDofTile;
        if (pair) L.maxnb[r] = estimate_maxnb(pot, R);
        if (L.ml) L.maxml[r] = estimate_maxml(pot, opt, R, L.maxnb[r]);
    }
    L.mlc.clear();
    L.mlm.clear();
    L.foff.assign(n_rep, 0);
    if (L.ml) {
        int64_t fo = 0;
        for (int r = 0; r < n_rep; ++r) {
            const int N = reps[r].n_atoms, P = reps[r].n_beads;
            for (int s = 0; s < P; ++s)
                for (int a = 0; a < N; a += 4) L.mlc.push_back({r, a, s, 0});
            for (int c0 = 0; c0 < N * P; c0 += 64) L.mlm.push_back({r, c0, std::min(64, N * P - c0), 0});
            L.foff[r] = fo;
            fo += 3 * (int64_t)N * P;
        }
    }
    L.n_cols = cols;
    // block tables
    L.upd.clear(); L.nl.clear(); L.force.clear(); L.tb.clear();
    L.upd_groups.clear(); L.force_groups.clear();
    std::map<int, std::vector<int>> byP, byG;
    for (int r = 0; r < n_rep; ++r) {
        byP[reps[r].n_beads].push_back(r);
        byG[bead_group(reps[r].n_beads)].push_back(r);
    }
    {
        // one launch covers every replica
        int maxP = 1, maxDP = 1;
        for (int r = 0; r < n_rep; ++r) {
            maxP = std::max(maxP, reps[r].n_beads);
            maxDP = std::max(maxDP, reps[r].n_dims * reps[r].n_beads);
        }
        L.upd_threads = update_threads(maxDP);
        for (int r = 0; r < n_rep; ++r) {
            const int per = update_block_atoms(reps[r].n_dims, reps[r].n_beads, L.upd_threads);
            for (int a = 0; a < reps[r].n_atoms; a += per) L.upd.push_back({r, a, per, 0});
        }
        L.upd_groups.push_back({maxP, {0, (int)L.upd.size()}});
    }
    for (int r = 0; r < n_rep; ++r) {
        for (int a = 0; a < reps[r].n_atoms; a += 4) L.nl.push_back({r, a, 0, 0});
        for (int a = 0; a < reps[r].n_atoms; a += kListTile) L.tb.push_back({r, a, 0, 0});
    }
    // force tables for every decomposition (the autotuner picks one)
    for (int t = 0; t < 6; ++t) {
        const int wi = t / 2, gi = t % 2;
        const int W = 1 << wi, apb = 4 / W;
        auto& F = L.force_w[t];
        auto& FG = L.force_groups_w[t];
        F.clear();
        FG.clear();
        L.obs_b0_w[t].assign(n_rep, 0);
        L.obs_nb_w[t].assign(n_rep, 0);
        if (pair) {
            for (auto& kv : byG) {
                const int G = (gi && kv.first > 1) ? kv.first / 2 : kv.first;
                const int b0 = (int)F.size();
                for (int r : kv.second) {
                    L.obs_b0_w[t][r] = (int)F.size();
                    for (int g = 0; g < reps[r].n_beads / G; ++g)
                        for (int a = 0; a < reps[r].n_atoms; a += apb) F.push_back({r, a, g, 0});
                    L.obs_nb_w[t][r] = (int)F.size() - L.obs_b0_w[t][r];
                }
                FG.push_back({G, {b0, (int)F.size()}});
            }
        } else {
            for (int r = 0; r < n_rep; ++r) {
                L.obs_b0_w[t][r] = (int)F.size();
                for (int a = 0; a < reps[r].n_atoms; a += 256) F.push_back({r, a, 0, 0});
                L.obs_nb_w[t][r] = (int)F.size() - L.obs_b0_w[t][r];
            }
            FG.push_back({0, {0, (int)F.size()}});
        }
        L.max_force_blocks = std::max(L.max_force_blocks, F.size());
    }
    {   // a table that mixes decompositions per group takes each group's largest
        size_t mix = 0;
        for (size_t k = 0; k < L.force_groups_w[0].size(); ++k) {
            int most = 0;
            for (int t = 0; t < 6; ++t) {
                const auto& g = L.force_groups_w[t][k].second;
                most = std::max(most, g.second - g.first);
            }
            mix += (size_t)most;
        }
        L.max_force_blocks = std::max(L.max_force_blocks, mix);
    }
    const int wdef = 2 * (kWavesPerAtomDefault == 1 ? 0 : (kWavesPerAtomDefault == 2 ? 1 : 2));
    L.force = L.force_w[wdef];
    L.force_groups = L.force_groups_w[wdef];
    L.force_group_W.assign(L.force_groups.size(), kWavesPerAtomDefault);
    L.force_group_t.assign(L.force_groups.size(), wdef);
    L.obs_b0 = L.obs_b0_w[wdef];
    L.obs_nb = L.obs_nb_w[wdef];
    L.tilev.assign(cols / kDofTile, FirTile{0, 2, 0, 0});
    for (int r = 0; r < n_rep; ++r) {
        const int64_t D = (int64_t)reps[r].n_dims * reps[r].n_atoms * reps[r].n_beads;
        const int64_t nt = (D + kDofTile - 1) / kDofTile;
        for (int64_t t = 0; t < nt; ++t)
            L.tilev[L.dof_off[r] / kDofTile + t] = FirTile{r, 2, r * L.taps_stride, 0};
    }

    size_t cur = 0;
    add(cur, L.reps, sizeof(RepDev) * n_rep);
    add(cur, L.status, 64);
    add(cur, L.clock, 64);
    add(cur, L.rebuild, sizeof(int32_t) * 3 * n_rep);
    add(cur, L.tiles, sizeof(FirTile) * L.tilev.size());
    add(cur, L.taps, zs * (size_t)L.taps_stride * n_rep);
    add(cur, L.ring, L.eq9 ? 0 : zs * (size_t)L.R * cols);
    add(cur, L.zeta, zs * (size_t)L.zeta_rows * cols);
    if (L.eq9) {
        add(cur, L.eq9amp, sizeof(double) * (size_t)(opt->max_two_nf / 2 + 1) * n_rep);
        add(cur, L.eq9tw, 2 * sizeof(double) * (size_t)(opt->max_two_nf / 2));
        add(cur, L.eq9mark, 64);
    }
    add(cur, L.partials, sizeof(double) * kNobs * L.max_force_blocks);
    add(cur, L.acc, sizeof(double) * kAcc * n_rep);
    {
        int32_t nmax = 1;
        for (int r = 0; r < n_rep; ++r) nmax = std::max(nmax, reps[r].n_atoms);
        L.cchunks = (nmax + kCentroidChunk - 1) / kCentroidChunk;
    }
    add(cur, L.cpart, sizeof(double) * (size_t)L.cchunks * n_rep);
    add(cur, L.counts, sizeof(int32_t) * n_rep);
    add(cur, L.pairtab, sizeof(PairTable<double>));
    add(cur, L.blk_upd, sizeof(BlockEntry) * std::max<size_t>(1, L.upd.size()));
    add(cur, L.blk_nl, sizeof(BlockEntry) * std::max<size_t>(1, L.nl.size()));
    add(cur, L.blk_tb, sizeof(BlockEntry) * std::max<size_t>(1, L.tb.size()));
    add(cur, L.blk_force, sizeof(BlockEntry) * L.max_force_blocks);
    if (L.ml) {
        add(cur, L.blk_mlc, sizeof(BlockEntry) * L.mlc.size());
        add(cur, L.blk_mlm, sizeof(BlockEntry) * L.mlm.size());
        add(cur, L.ml_acc, sizeof(double) * kAcc * n_rep);
        add(cur, L.ml_counts, sizeof(int32_t) * n_rep);
        add(cur, L.ml_loss, sizeof(double) * n_rep);
        add(cur, L.ml_stats, sizeof(double) * (2 * kMlFeat * 2 + 2));
        add(cur, L.ml_foff, sizeof(int64_t) * n_rep);
        if (L.ml_train) add(cur, L.ml_wpart, sizeof(float) * (size_t)kWgBlocks * kMlParams);
    }
    for (int r = 0; r < n_rep; ++r) {
        const qtb_replica& R = reps[r];
        const size_t N = R.n_atoms, P = R.n_beads, dm = R.n_dims;
        auto& p = L.per[r];
        add(cur, p.force, ts * P * dm * N);
        add(cur, p.r0, 8 * P * dm * N);
        add(cur, p.eatom, 8 * P * N);
        add(cur, p.species, 4 * N);
        add(cur, p.nm, 8 * P * P);
        add(cur, p.ring, 8 * 3 * P);
        if (pair) {
            for (int q = 0; q < 2; ++q) {
                add(cur, p.u[q], 4 * ts * P * N);
                add(cur, p.rref[q], 8 * 3 * N);
                add(cur, p.cnow[q], 8 * 3 * N);
                add(cur, p.dev[q], 8 * N);
                add(cur, p.devb[q], 8 * N);
            }
            add(cur, p.tbox, 8 * 8 * ((N + kListTile - 1) / kListTile));
            add(cur, p.nb, 4 * ts * N * (size_t)L.maxnb[r]);
            add(cur, p.nbc, 4 * N);
            add(cur, p.nbcore, 4 * N);
            if (L.ml) {
                const size_t M = L.maxml[r];
                add(cur, p.mlnb, 4 * ts * N * M);
                add(cur, p.mlnc, 4 * N);
                add(cur, p.mlrev, 4 * N * M);
                add(cur, p.mlG, 4 * P * N * kMlFeat);
                add(cur, p.mlaux, 4 * P * N * kMlAux);
                add(cur, p.mlg, 4 * P * N * kMlFeat);
                add(cur, p.mly, 4 * P * N);
                add(cur, p.mlfp, 16 * P * N * M);
                add(cur, p.mlin, 4 * P * N * M);
                add(cur, p.mlnin, 4 * P * N);
                if (L.ml_train) {
                    add(cur, p.mlv, 4 * P * N * kMlFeat);
                    add(cur, p.mlu, 4 * P * 3 * N);
                    add(cur, p.mladj, 4 * P * N * kMlAdj);
                    add(cur, p.mlebar, 8);
                }
            }
        } else {
            add(cur, p.homega, 8 * N);
        }
    }
    L.total = cur;
}

std::string g_static_err;

}  // namespace

// ------------------------------------------------------------------ context
namespace {
// Byte offsets of a velocity-spectrum workspace (the recorder's, or the
// standalone transform's without trace, weights and counter).
struct VdosLayout {
    size_t trace = 0, spec = 0, part = 0, stage = 0, tw = 0, w = 0, cnt = 0, total = 0;
};

VdosLayout vdos_layout(int n_dof, int seg, bool recorder)
{
    const VdosPlan p = vdos_plan(n_dof, seg);
    VdosLayout l;
    size_t cur = 0;
    auto take = [&cur](size_t bytes) {
        const size_t o = cur;
        cur += (bytes + 255) & ~(size_t)255;
        return o;
    };
    l.part = take(8 * (size_t)p.grid * p.nk);
    l.stage = take(8 * (size_t)p.stage_rows * p.nk);
    l.tw = take(16 * (size_t)(seg / 2));
    l.w = take(8 * (size_t)n_dof);  // square roots of the weights
    if (recorder) {
        l.trace = take(8 * 2 * (size_t)seg * n_dof);
        l.spec = take(8 * (size_t)p.nk);
        l.cnt = take(8);
    }
    l.total = cur;
    return l;
}

// Velocity recorder of one replica, in the caller's device buffer.  The
// trace [2 seg][dof] holds two segments: a segment is transformed once
// complete, while the steps go on filling the other half.
struct VdosRec {
    bool on = false;
    char* ws = nullptr;
    VdosPlan plan{};
    VdosLayout lay{};
    int n_dof = 0;
    int64_t start = 0;  // global step of the (re)start: samples count from there
    int64_t n_seg = 0;  // segments transformed since
    template <typename X>
    X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
};
}  // namespace

struct qtb_ctx {
    qtb_options opt{};
    hipStream_t st = nullptr;
    // launches of different bead-group widths (disjoint replicas) run on
    // streams of their own, forked from and joined back into st
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;   // [0] the fork, [k] the join of side stream k - 1
    bool side_failed = false;
    bool fp64 = false, pair = false;
    int n_rep = 0;
    std::vector<qtb_replica> reps;
    std::vector<std::vector<int32_t>> species;
    std::vector<std::vector<double>> homega;
    int kind = QTB_POT_PAIR;
    std::vector<double> osV0, osd;  // on-site kinds, per species
    std::vector<double> mass, charge, bA, brho, bC;
    double alpha = 0, rc = 0, skin = 0;
    Layout L;
    char* ws = nullptr;
    std::vector<RepDev> rd;
    std::vector<int> two_nf;
    std::vector<bool> filter_ready;
    std::vector<std::vector<double>> taps;
    std::vector<double> eself;
    PairTable<float> tabf{};
    PairTable<double> tabd{};
    int64_t step = 0;          // global step counter
    int64_t block_start = -1;  // global step of the current noise block
    int block_row = 0;
    bool ring_valid = false;
    std::string err;
    int W = kWavesPerAtomDefault;  // force kernel wavefronts per atom
    bool half_groups = false;      // force kernel: half the widest bead group per wavefront
    bool tuned = false;
    // captured noise blocks of K steps, replayed while nothing changes; one
    // per sampling / checking pattern (block start modulo obs_every and
    // modulo the surrogate's check interval) and per row range of the block
    std::vector<std::pair<std::array<int64_t, 4>, hipGraphExec_t>> graphs;
    bool graph_failed = false;
    // surrogate
    qtb_ml* ml = nullptr;
    int32_t ml_check_every = 0;
    // one-kernel steps: a step's closing half-kick is pending (open) between
    // the step kernels of one qtb_step call; the call ends with a force pass
    bool open = false;
    bool npt_used = false;      // a barostat has run: the device table holds the boxes
    std::vector<VdosRec> vdos;  // per replica
    std::vector<double> eq9amp;  // block noise: amplitudes [n_rep][n/2 + 1] (host copy)
    // step of the kernels being recorded: host step (rec_row < 0), or the
    // device clock (first step of the noise block) + rec_row + rec_extra
    int rec_row = -1, rec_extra = 0;
    // profiling: event pairs per phase
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;  // (phase, index of start event)

    template <typename X>
    X* at(const Region& r) const { return reinterpret_cast<X*>(ws + r.off); }
};

// Surrogate model: weights, Adam moments and normalisation in the caller's
// device buffer.
struct qtb_ml {
    hipStream_t st = nullptr;
    char* ws = nullptr;
    Region master, wq, m1, m2, grad, mu, isd, e0;
    size_t total = 0;
    double r_cut = 0.0, r_min = 0.0;
    int64_t t = 0;  // Adam steps taken
    std::string err;
    std::vector<double> norm;  // host copy: mu [2][96], inv_sd [2][96], e0 [2]

    template <typename X>
    X* at(const Region& r) const { return reinterpret_cast<X*>(ws + r.off); }
    MlDev dev() const
    {
        MlDev d{};
        d.wq = at<uint16_t>(wq);
        d.master = at<float>(master);
        d.mu = at<float>(mu);
        d.inv_sd = at<float>(isd);
        d.e0 = at<double>(e0);
        d.r_cut = (float)r_cut;
        d.r_min = (float)r_min;
        const double dr = (r_cut - r_min) / (kMlRad - 1), da = (r_cut - r_min) / (kMlAng - 1);
        d.mu0 = (float)r_min;
        d.dr = (float)dr;
        d.eta_r = (float)(1.0 / (2.0 * dr * dr));
        d.nu0 = (float)r_min;
        d.da = (float)da;
        d.eta_a = (float)(1.0 / (2.0 * da * da));
        return d;
    }
};

namespace {
void ml_layout(qtb_ml& m)
{
    size_t cur = 0;
    add(cur, m.master, 4 * (size_t)kMlParams);
    add(cur, m.m1, 4 * (size_t)kMlParams);
    add(cur, m.m2, 4 * (size_t)kMlParams);
    add(cur, m.grad, 4 * (size_t)kMlParams);
    add(cur, m.wq, 2 * (size_t)kMlParams);
    add(cur, m.mu, 4 * 2 * (size_t)kMlFeat);
    add(cur, m.isd, 4 * 2 * (size_t)kMlFeat);
    add(cur, m.e0, 8 * 2);
    m.total = cur;
}
}  // namespace

namespace {
StepRef step_ref(const qtb_ctx* c)
{
    if (c->rec_row < 0) return StepRef{nullptr, c->step};
    return StepRef{c->at<int64_t>(c->L.clock), (int64_t)c->rec_row + c->rec_extra};
}
}  // namespace

namespace qtb {
LaunchStamp& launch_stamp()
{
    static thread_local LaunchStamp ls;
    return ls;
}
}  // namespace qtb

namespace {

hipEvent_t next_event(qtb_ctx* c)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Profiling marker of one phase: its first kernel launch stamps an event pair
// from its own dispatch (the phase's other launches, if any, are not timed).
// A phase with several launches (one per replica group) is timed with
// event markers around all of them instead.
struct Phase {
    qtb_ctx* c;
    size_t idx = 0;
    bool on = false, multi = false;
    Phase(qtb_ctx* cc, int ph, bool several = false) : c(cc), multi(several)
    {
        if (!c->prof) return;
        idx = c->ev_used;
        hipEvent_t a = next_event(c), b = next_event(c);
        if (!a || !b) return;
        if (multi) (void)hipEventRecord(a, c->st);
        else launch_stamp() = LaunchStamp{a, b};
        c->ev_marks.push_back({ph, idx});
        on = true;
    }
    ~Phase()
    {
        if (!on) return;
        if (multi) {
            (void)hipEventRecord(c->ev_pool[idx + 1], c->st);
        } else if (launch_stamp().start) {  // nothing was launched in this phase
            launch_stamp() = LaunchStamp{};
            c->ev_marks.pop_back();
        }
    }
};

qtb_status fail(qtb_ctx* c, qtb_status s, const std::string& m)
{
    if (c) c->err = m;
    else g_static_err = m;
    return s;
}

}  // namespace

void qtb::set_static_error(const std::string& m) { g_static_err = m; }

namespace {

qtb_status hip_check(qtb_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return QTB_OK;
    return fail(c, QTB_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define QTB_HIP(c, call)                                               \
    do {                                                               \
        qtb_status s_ = hip_check((c), (call), #call);                 \
        if (s_ != QTB_OK) return s_;                                   \
    } while (0)

void nm_matrix(int P, double* C)
{
    for (int s = 0; s < P; ++s)
        for (int k = 0; k < P; ++k) {
            double v;
            if (k == 0) v = 1.0 / std::sqrt((double)P);
            else if (2 * k < P) v = std::sqrt(2.0 / P) * std::cos(2.0 * kPi * s * k / P);
            else if (2 * k == P) v = ((s % 2) ? -1.0 : 1.0) / std::sqrt((double)P);
            else v = std::sqrt(2.0 / P) * std::sin(2.0 * kPi * s * k / P);
            C[s * P + k] = v;
        }
}

template <typename T>
void fill_pair_table(qtb_ctx* c, PairTable<T>& tab)
{
    const int ns = (int)c->mass.size();
    const double rc = c->rc, al = c->alpha, k = c->opt.coulomb_k;
    const double g = 2.0 * al / std::sqrt(kPi);
    const double erc = std::erfc(al * rc);
    const double Sc = erc / (rc * rc) + g * std::exp(-al * al * rc * rc) / rc;
    std::memset(&tab, 0, sizeof(tab));
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            const int ab = a * ns + b;
            const double A = c->bA[ab], rho = c->brho[ab], C = c->bC[ab];
            const double irho = A != 0.0 ? 1.0 / rho : 0.0;
            const double VB = A * std::exp(-rc * irho) - C / std::pow(rc, 6);
            const double dVB = -A * irho * std::exp(-rc * irho) + 6.0 * C / std::pow(rc, 7);
            const double kqq = k * c->charge[a] * c->charge[b];
            const double F0 = dVB - kqq * Sc;
            const double E0 = -VB + rc * dVB - kqq * erc / rc - kqq * Sc * rc;
            PairParam<T>& p = tab.p[a * kMaxSpecies + b];
            p.Arho = (T)(A * irho);
            p.irho = (T)irho;
            p.C6 = (T)(6.0 * C);
            p.kqq = (T)kqq;
            p.F0 = (T)F0;
            p.A = (T)A;
            p.C = (T)C;
            p.E0 = (T)E0;
            p.irho2 = (T)(irho * 1.4426950408889634);
        }
    tab.alpha = (T)al;
    tab.g = (T)g;
    tab.rc2 = (T)(rc * rc);
    tab.a2l = (T)(al * al * 1.4426950408889634);
    tab.n_species = ns;
    // erfcx on [0, x_max]: Chebyshev interpolation at 48 nodes, truncated where
    // the tail is below 2e-8 of the constant term, converted to monomials in s.
    const double xmax = std::max(al * rc, 1e-3);
    const int nn = 48;
    std::vector<double> cc(nn, 0.0);
    for (int j = 0; j < nn; ++j) {
        double acc = 0.0;
        for (int q = 0; q < nn; ++q) {
            const double th = kPi * (q + 0.5) / nn;
            const double x = 0.5 * (std::cos(th) + 1.0) * xmax;
            acc += std::erfc(x) * std::exp(x * x) * std::cos(j * th);
        }
        cc[j] = 2.0 * acc / nn;
    }
    cc[0] *= 0.5;
    // degree 10 when its Chebyshev tail is below 3e-7 of the constant term
    // (alpha r_cut up to about 2), else kErfcxMaxDeg, else no fit
    auto tail_after = [&](int d) {
        double t = 0.0;
        for (int j = d + 1; j < nn; ++j) t += std::fabs(cc[j]);
        return t;
    };
    int deg = 10;
    if (tail_after(10) >= 3e-7 * std::fabs(cc[0])) deg = kErfcxMaxDeg;
    bool fit_ok = tail_after(deg) < 5e-7 * std::fabs(cc[0]);
    // monomial coefficients of sum_j cc[j] T_j(s), j <= deg
    std::vector<double> mono(deg + 1, 0.0), tm1(deg + 1, 0.0), t0(deg + 1, 0.0), t1(deg + 1, 0.0);
    tm1[0] = 1.0;            // T_0
    mono[0] += cc[0];
    if (deg >= 1) {
        t0[1] = 1.0;         // T_1
        mono[1] += cc[1];
    }
    for (int j = 2; j <= deg; ++j) {
        std::fill(t1.begin(), t1.end(), 0.0);
        for (int q = 0; q < deg; ++q) t1[q + 1] += 2.0 * t0[q];
        for (int q = 0; q <= deg; ++q) t1[q] -= tm1[q];
        for (int q = 0; q <= deg; ++q) mono[q] += cc[j] * t1[q];
        tm1 = t0;
        t0 = t1;
    }
    for (int q = 0; q <= kErfcxMaxDeg; ++q) tab.ex[q] = (T)(q <= deg ? mono[q] : 0.0);
    tab.s_mul = (T)(2.0 * al / xmax);
    // Coulomb force shape phi(a r) = erfc(a r) + (2 a r / sqrt(pi)) e^{-a^2 r^2}
    // = 1 + (r r^2) a^3 psi(a^2 r^2) on r in [0, r_cut]: Chebyshev
    // interpolation of a^3 psi in s = r^2 (2 / r_cut^2) - 1, psi from its
    // Taylor series (alternating, all terms of one sign pair summed in FP64)
    // psi(y) = -(4 / sqrt(pi)) sum_n (-y)^n / (n! (2n + 3)).
    auto psi = [&](double y) {
        double t = 1.0, sum = 0.0;
        for (int n = 0; n < 200; ++n) {
            const double term = t / (2.0 * n + 3.0);
            sum += term;
            if (std::fabs(term) < 1e-18 * std::fabs(sum) && n > 2 * y + 5) break;
            t *= -y / (n + 1.0);
        }
        return -4.0 / std::sqrt(kPi) * sum;
    };
    std::vector<double> cp(nn, 0.0);
    for (int j = 0; j < nn; ++j) {
        double acc = 0.0;
        for (int q = 0; q < nn; ++q) {
            const double th = kPi * (q + 0.5) / nn;
            const double r2 = 0.5 * (std::cos(th) + 1.0) * rc * rc;
            acc += al * al * al * psi(al * al * r2) * std::cos(j * th);
        }
        cp[j] = 2.0 * acc / nn;
    }
    cp[0] *= 0.5;
    auto ptail = [&](int d) {
        double t = 0.0;
        for (int j = d + 1; j < nn; ++j) t += std::fabs(cp[j]);
        return t;
    };
    // relative to phi, whose smallest value on [0, r_cut] is phi(a r_cut):
    // the tail of r^3 ph must stay below 5e-8 of it (2e-7 for degree 14)
    const double phimin = std::erfc(xmax) + 2.0 * xmax / std::sqrt(kPi) * std::exp(-xmax * xmax);
    const double r3 = rc * rc * rc;
    const bool phi10 = ptail(10) * r3 < 5e-8 * phimin;
    const bool phi14 = ptail(kErfcxMaxDeg) * r3 < 2e-7 * phimin;
    if (!phi10 && deg == 10 && phi14) deg = kErfcxMaxDeg;  // both polynomials of one degree
    const bool phi_ok = deg == 10 ? phi10 : phi14;
    std::vector<double> pm(deg + 1, 0.0);
    {
        std::vector<double> a(deg + 1, 0.0), b(deg + 1, 0.0), c2(deg + 1, 0.0);
        a[0] = 1.0;
        pm[0] += cp[0];
        if (deg >= 1) {
            b[1] = 1.0;
            pm[1] += cp[1];
        }
        for (int j = 2; j <= deg; ++j) {
            std::fill(c2.begin(), c2.end(), 0.0);
            for (int q = 0; q < deg; ++q) c2[q + 1] += 2.0 * b[q];
            for (int q = 0; q <= deg; ++q) c2[q] -= a[q];
            for (int q = 0; q <= deg; ++q) pm[q] += cp[j] * c2[q];
            a = b;
            b = c2;
        }
    }
    for (int q = 0; q <= kErfcxMaxDeg; ++q) tab.ph[q] = (T)(q <= deg ? pm[q] : 0.0);
    tab.ph_s = (T)(2.0 / (rc * rc));
    tab.ex_deg = (fit_ok && phi_ok) ? deg : 0;
}

void fill_repdev(qtb_ctx* c, int r)
{
    const qtb_replica& R = c->reps[r];
    const Layout::Per& p = c->L.per[r];
    RepDev& d = c->rd[r];
    d.pos = R.d_pos;
    d.vel = R.d_vel;
    d.force = c->at<void>(p.force);
    for (int q = 0; q < 2; ++q) {
        d.ub[q] = c->pair ? c->at<void>(p.u[q]) : nullptr;
        d.rrefb[q] = c->pair ? c->at<double>(p.rref[q]) : nullptr;
        d.cnb[q] = c->pair ? c->at<double>(p.cnow[q]) : nullptr;
        d.devn[q] = c->pair ? c->at<double>(p.dev[q]) : nullptr;
        d.devbb[q] = c->pair ? c->at<double>(p.devb[q]) : nullptr;
    }
    d.r0 = c->at<double>(p.r0);
    d.eatom = c->at<double>(p.eatom);
    d.species = c->at<int32_t>(p.species);
    d.homega = c->pair ? nullptr : c->at<double>(p.homega);
    d.nb_entries = c->pair ? c->at<void>(p.nb) : nullptr;
    d.nb_count = c->pair ? c->at<int32_t>(p.nbc) : nullptr;
    d.nb_core = c->pair ? c->at<int32_t>(p.nbcore) : nullptr;
    d.tbox = c->pair ? c->at<double>(p.tbox) : nullptr;
    d.nm = c->at<double>(p.nm);
    d.ring = c->at<double>(p.ring);
    d.rflag = c->at<int32_t>(c->L.rebuild) + 3 * r;
    d.dof_off = c->L.dof_off[r];
    d.N = R.n_atoms;
    d.P = R.n_beads;
    d.dims = R.n_dims;
    d.maxnb = c->pair ? c->L.maxnb[r] : 0;
    d.two_nf = c->two_nf[r];
    d.noise = R.noise;
    d.obs_block0 = c->L.obs_b0[r];
    d.obs_nblocks = c->L.obs_nb[r];
    for (int a = 0; a < 3; ++a) d.box[a] = R.box[a];
    d.c1 = std::exp(-R.gamma * R.dt);
    d.kT = c->opt.kB * R.T;
    d.omega_P = std::sqrt((double)R.n_beads) * d.kT / c->opt.hbar;
    d.half_skin = 0.5 * c->skin;
    d.half_skin0 = d.half_skin;
    d.npt_S = 1.0;
    d.npt_sr = d.npt_sv1 = d.npt_sv2 = 1.0;
    d.r_cs = c->rc + c->skin;
    d.r_cut = c->rc;
    for (int a = 0; a < kMaxSpecies; ++a) {
        const double m = a < (int)c->mass.size() ? c->mass[a] * c->opt.mass_unit : 1.0;
        d.mmu[a] = m;
        d.kick[a] = R.dt / (2.0 * R.n_beads * m);
        d.sigma[a] = std::sqrt((1.0 - d.c1 * d.c1) / m);
        d.osV0[a] = a < (int)c->osV0.size() ? c->osV0[a] : 0.0;
        d.osd[a] = a < (int)c->osd.size() ? c->osd[a] : 1.0;
    }
    d.seed = R.seed;
    d.stream = R.stream;
    d.dt = R.dt;
    if (c->L.ml) {
        d.ml_nb = c->at<void>(p.mlnb);
        d.ml_nc = c->at<int32_t>(p.mlnc);
        d.ml_rev = c->at<int32_t>(p.mlrev);
        d.ml_G = c->at<float>(p.mlG);
        d.ml_aux = c->at<float>(p.mlaux);
        d.ml_g = c->at<float>(p.mlg);
        d.ml_y = c->at<float>(p.mly);
        d.ml_fpair = c->at<float>(p.mlfp);
        d.ml_in = c->at<int32_t>(p.mlin);
        d.ml_nin = c->at<int32_t>(p.mlnin);
        d.maxml = c->L.maxml[r];
        d.ml_rcs = c->opt.ml_r_cut + c->skin;
        if (c->L.ml_train) {
            d.ml_v = c->at<float>(p.mlv);
            d.ml_u = c->at<float>(p.mlu);
            d.ml_adj = c->at<float>(p.mladj);
            d.ml_ebar = c->at<double>(p.mlebar);
        }
    }
}

bool npt_any(const qtb_ctx* c)
{
    for (const auto& d : c->rd)
        if (d.npt) return true;
    return false;
}

// Once a barostat has run, the device copy of the replica table holds the
// current boxes, list scales and rebuild thresholds: bring them back to the
// host tables (synchronises).
qtb_status sync_boxes(qtb_ctx* c)
{
    if (!c->npt_used) return QTB_OK;
    std::vector<RepDev> dev(c->n_rep);
    QTB_HIP(c, hipMemcpyAsync(dev.data(), c->at<void>(c->L.reps), sizeof(RepDev) * c->n_rep,
                              hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    for (int r = 0; r < c->n_rep; ++r) {
        for (int a = 0; a < 3; ++a) {
            c->rd[r].box[a] = dev[r].box[a];
            c->reps[r].box[a] = dev[r].box[a];
        }
        c->rd[r].npt_S = dev[r].npt_S;
        c->rd[r].half_skin = dev[r].half_skin;
        c->rd[r].npt_pe = dev[r].npt_pe;
        c->rd[r].npt_sr = dev[r].npt_sr;
        c->rd[r].npt_sv1 = dev[r].npt_sv1;
        c->rd[r].npt_sv2 = dev[r].npt_sv2;
    }
    return QTB_OK;
}

// Host tables to the device as they are (the caller has synchronised them).
qtb_status upload_tables_raw(qtb_ctx* c)
{
    QTB_HIP(c, hipMemcpyAsync(c->at<void>(c->L.reps), c->rd.data(), sizeof(RepDev) * c->n_rep,
                              hipMemcpyHostToDevice, c->st));
    QTB_HIP(c, hipMemcpyAsync(c->at<void>(c->L.tiles), c->L.tilev.data(),
                              sizeof(FirTile) * c->L.tilev.size(), hipMemcpyHostToDevice, c->st));
    return QTB_OK;
}

qtb_status upload_tables(qtb_ctx* c)
{
    if (qtb_status s = sync_boxes(c)) return s;
    return upload_tables_raw(c);
}

// Block noise (eq. 9): amplitudes of replica r's Fourier modes on the grid
// omega_j = 2 pi j / (n dt), j = 0 .. n/2, n = max_two_nf: sqrt(n S_j / 2),
// and sqrt(n S_j) for the self-conjugate modes j = 0 and n/2.
qtb_status upload_eq9_amp(qtb_ctx* c, int r, int kind)
{
    const int n = c->L.max_two_nf, h = n / 2;
    const qtb_replica& R = c->reps[r];
    double* A = c->eq9amp.data() + (size_t)r * (h + 1);
    design_spectrum(kind, R.T, R.n_beads, R.dt, n, c->opt.hbar, c->opt.kB, A);
    for (int j = 0; j <= h; ++j) A[j] = std::sqrt((j == 0 || j == h ? 1.0 : 0.5) * n * A[j]);
    QTB_HIP(c, hipMemcpyAsync(c->at<double>(c->L.eq9amp) + (size_t)r * (h + 1), A,
                              8 * (size_t)(h + 1), hipMemcpyHostToDevice, c->st));
    return QTB_OK;
}

template <typename Z>
qtb_status upload_taps_T(qtb_ctx* c, int r)
{
    std::vector<Z> buf(c->L.taps_stride, Z(0));
    const int pad = fir_pad();
    for (int x = 0; x < c->two_nf[r]; ++x) buf[pad + x] = (Z)c->taps[r][x];
    QTB_HIP(c, hipMemcpyAsync(c->at<Z>(c->L.taps) + (size_t)r * c->L.taps_stride, buf.data(),
                              sizeof(Z) * buf.size(), hipMemcpyHostToDevice, c->st));
    return hipStreamSynchronize(c->st) == hipSuccess ? QTB_OK
                                                      : fail(c, QTB_E_DEVICE, "taps upload");
}

qtb_status upload_taps(qtb_ctx* c, int r)
{
    if (c->opt.fir == QTB_FIR_FP64) return upload_taps_T<double>(c, r);
    return upload_taps_T<float>(c, r);
}

// Pair-potential (or oscillator) forces of every replica.  kCompare leaves
// the rebuild flags alone (the surrogate's forward pass cleared them).
// Whether steps rebuild lists in the list kernel (else inside the force kernel).
bool list_kernel(const qtb_ctx* c)
{
    if (c->ml || c->L.ml || (c->opt.flags & QTB_OPT_LIST_KERNEL)) return true;
    for (const auto& R : c->reps)
        if (R.n_atoms > kInlineRebuildMaxAtoms) return true;
    return false;
}

// inline_rebuild: the force kernel rebuilds flagged lists itself (no list
// kernel launched before it).
// Streams for n independent launches: launch k on the returned stream k
// (stream 0 is st).  With more than one launch (and no phase profiling, whose
// event pairs bracket st only) the others get side streams that wait for an
// event recorded on st; join_branches makes st wait for them.  Any failure
// to create a stream or event leaves every launch on st.
std::vector<hipStream_t> fork_branches(qtb_ctx* c, size_t n)
{
    std::vector<hipStream_t> out(n, c->st);
    if (n <= 1 || c->prof || c->side_failed) return out;
    while (c->side.size() < n - 1) {
        hipStream_t x = nullptr;
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
            c->side_failed = true;
            (void)hipGetLastError();
            return out;
        }
        c->side.push_back(x);
    }
    while (c->side_ev.size() < n) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            c->side_failed = true;
            (void)hipGetLastError();
            return out;
        }
        c->side_ev.push_back(e);
    }
    if (hipEventRecord(c->side_ev[0], c->st) != hipSuccess) {
        c->side_failed = true;
        (void)hipGetLastError();
        return out;
    }
    for (size_t k = 1; k < n; ++k) {
        if (hipStreamWaitEvent(c->side[k - 1], c->side_ev[0], 0) != hipSuccess) {
            c->side_failed = true;  // this launch and later ones stay on st
            (void)hipGetLastError();
            break;
        }
        out[k] = c->side[k - 1];
    }
    return out;
}

void join_branches(qtb_ctx* c, const std::vector<hipStream_t>& br)
{
    for (size_t k = 1; k < br.size(); ++k) {
        if (br[k] == c->st) continue;
        if (hipEventRecord(c->side_ev[k], br[k]) != hipSuccess ||
            hipStreamWaitEvent(c->st, c->side_ev[k], 0) != hipSuccess) {
            // without the join st must not run ahead: wait for the branch
            c->side_failed = true;
            (void)hipGetLastError();
            (void)hipStreamSynchronize(br[k]);
        }
    }
}

// Force group k of the current table (only = k), or all of them (only < 0).
void launch_plain_forces(qtb_ctx* c, int32_t flags, bool inline_rebuild = false, int only = -1)
{
    const Layout& L = c->L;
    const RepDev* dreps = c->at<RepDev>(L.reps);
    const BlockEntry* fb = c->at<BlockEntry>(L.blk_force);
    double* part = c->at<double>(L.partials);
    const int clear = (flags & kCompare) ? 0 : (inline_rebuild ? 2 : 1);
    const auto br = fork_branches(c, only >= 0 ? 1 : L.force_groups.size());
    for (size_t k = 0; k < L.force_groups.size(); ++k) {
        if (only >= 0 && (size_t)only != k) continue;
        const hipStream_t st = only >= 0 ? c->st : br[k];
        const auto& g = L.force_groups[k];
        const int b0 = g.second.first, nb = g.second.second - g.second.first;
        if (nb <= 0) continue;
        if (c->pair) {
            const void* tab = c->fp64 ? (const void*)&c->tabd : (const void*)&c->tabf;
            launch_forces_pair(st, c->fp64, g.first, L.force_group_W[k], dreps, fb + b0, nb,
                               tab, flags, part + (size_t)b0 * kNobs, clear, c->n_rep,
                               c->at<int32_t>(L.status), step_ref(c));
        } else {
            launch_forces_onsite(st, c->fp64, c->kind, dreps, fb + b0, nb, flags,
                                 part + (size_t)b0 * kNobs);
        }
    }
    join_branches(c, br);
}

// Surrogate forces of every replica with model m: descriptors, network,
// per-pair derivatives, then the gather with the force kernels' epilogue.
void launch_ml_forces(qtb_ctx* c, const qtb_ml* m, int32_t flags)
{
    const Layout& L = c->L;
    const RepDev* dreps = c->at<RepDev>(L.reps);
    const MlDev md = m->dev();
    launch_ml_forward(c->st, c->fp64, dreps, md, c->at<BlockEntry>(L.blk_mlc), (int)L.mlc.size(),
                      c->at<BlockEntry>(L.blk_mlm), (int)L.mlm.size(), c->n_rep,
                      c->at<int32_t>(L.status), step_ref(c));
    const BlockEntry* fb = c->at<BlockEntry>(L.blk_force);
    double* part = c->at<double>(L.partials);
    for (auto& g : L.force_groups) {
        const int b0 = g.second.first, nb = g.second.second - g.second.first;
        if (nb > 0)
            launch_ml_gather(c->st, c->fp64, g.first, 4 / c->W, dreps, md, fb + b0, nb, flags,
                             part + (size_t)b0 * kNobs);
    }
}

// Forces of the context's current force provider.
void launch_forces(qtb_ctx* c, int32_t flags)
{
    if (c->ml) launch_ml_forces(c, c->ml, flags);
    else launch_plain_forces(c, flags);
}

// in_step: inside a step, after its update (positions carry a barostat's
// pending box factor; the builds are marked for the barostat).
void launch_rebuild(qtb_ctx* c, bool centroids = false, bool in_step = false)
{
    if (!c->pair) return;
    const Layout& L = c->L;
    launch_nlist(c->st, c->fp64, c->at<RepDev>(L.reps), c->at<BlockEntry>(L.blk_nl),
                 (int)L.nl.size(), c->at<BlockEntry>(L.blk_tb), (int)L.tb.size(),
                 c->at<int32_t>(L.status), centroids, step_ref(c), in_step);
    if (L.ml)  // the surrogate's shorter lists follow every rebuild
        launch_ml_lists(c->st, c->fp64, c->at<RepDev>(L.reps), c->at<BlockEntry>(L.blk_nl),
                        (int)L.nl.size(), c->at<int32_t>(L.status), step_ref(c));
}

qtb_status refresh_forces(qtb_ctx* c)
{
    if (c->npt_used) {  // every list is rebuilt from the current geometry
        if (qtb_status s = sync_boxes(c)) return s;
        for (auto& d : c->rd) {  // (a pending box factor still applies next step)
            d.npt_S = 1.0;
            d.half_skin = d.half_skin0 - std::max(0.0, 1.0 - d.npt_sr) * 0.5 * d.r_cs;
        }
        if (qtb_status s = upload_tables_raw(c)) return s;
    }
    if (c->pair) {
        launch_mark_rebuild(c->st, c->at<RepDev>(c->L.reps), c->n_rep, c->at<int32_t>(c->L.status),
                            step_ref(c));
        launch_rebuild(c, true);
    }
    launch_forces(c, 0);
    QTB_HIP(c, hipGetLastError());
    return QTB_OK;
}

qtb_status read_status(qtb_ctx* c)
{
    int32_t st[2] = {0, 0};
    QTB_HIP(c, hipMemcpyAsync(st, c->at<int32_t>(c->L.status), sizeof(st), hipMemcpyDeviceToHost,
                              c->st));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (st[0] & kStatusRange)  // first: a diverged state also overflows the lists
        return fail(c, QTB_E_NONFINITE,
                    "diverged state: pair range beyond the periodic-image limit of the list search");
    if (st[0] & kStatusNbOverflow)
        return fail(c, QTB_E_NOMEM, "neighbour list overflow: density above the planned maximum");
    if (st[0] & kStatusMlList)
        return fail(c, QTB_E_NOMEM, "surrogate neighbour list overflow or unmatched pair");
    if (st[0] & kStatusNonfinite) return fail(c, QTB_E_NONFINITE, "non-finite position or velocity");
    return QTB_OK;
}

// White-noise rows clock + off .. clock + off + rows - 1 into the ring.
void gen_rows(qtb_ctx* c, int64_t off, int64_t rows)
{
    const Layout& L = c->L;
    Phase ph(c, 0, rows > 1024);
    for (int64_t r0 = 0; r0 < rows; r0 += 1024) {
        const int rr = (int)std::min<int64_t>(1024, rows - r0);
        launch_gen_white(c->st, c->at<RepDev>(L.reps), c->at<FirTile>(L.tiles),
                         c->at<void>(L.ring), c->opt.fir,
                         c->at<int64_t>(L.clock), off + r0, rr, L.R, L.n_cols);
    }
}

// First block after init / set_state / build_filter: put the clock one block
// behind and fill the history rows of the window.
void prime_ring(qtb_ctx* c)
{
    const int K = c->L.K, maxNf = c->L.max_two_nf / 2;
    launch_clock(c->st, c->at<int64_t>(c->L.clock), c->step - K, false);
    if (!c->L.eq9) gen_rows(c, K - maxNf + 1, 2 * maxNf - 1);  // block noise keeps no history
    c->ring_valid = true;
}

// Kernels of one step; row = step index inside the noise block.
void record_step(qtb_ctx* c, int row, bool sample, bool check)
{
    c->rec_row = row;  // the update works on step row, the rest on row + 1
    c->rec_extra = 0;
    const Layout& L = c->L;
    const size_t zs = c->opt.fir == QTB_FIR_FP64 ? 8 : 4;
    // block noise: the update finds its row in the [2 n] ring from the step
    const char* zrow = c->at<char>(L.zeta) + (L.eq9 ? 0 : (size_t)row * L.n_cols * zs);
    const int64_t zmod = L.eq9 ? L.zeta_rows : 0;
    const RepDev* dreps = c->at<RepDev>(L.reps);
    const BlockEntry* ub = c->at<BlockEntry>(L.blk_upd);
    {
        Phase ph(c, 2);
        const auto br = fork_branches(c, L.upd_groups.size());
        for (size_t k = 0; k < L.upd_groups.size(); ++k) {
            const auto& g = L.upd_groups[k];
            const int b0 = g.second.first, nb = g.second.second - g.second.first;
            if (nb > 0)
                launch_update(br[k], c->fp64, c->pair, g.first, L.upd_threads, dreps, ub + b0, nb,
                              zrow, c->at<int32_t>(L.status), step_ref(c), zmod, L.n_cols);
        }
        join_branches(c, br);
    }
    c->rec_extra = 1;
    // the pair potential's force kernel rebuilds flagged lists itself, except
    // for large replicas (the list kernel prunes its scan by tile bounds) and
    // with surrogate buffers (the surrogate's lists follow the list kernel)
    const bool inline_rebuild = c->pair && !list_kernel(c);
    if (c->pair && !inline_rebuild) {
        Phase ph(c, 3, true);  // tile bounds and list kernels (+ surrogate lists)
        launch_rebuild(c, false, true);
    }
    // the barostat needs the kinetic energy, springs and pair virial of every
    // step (the sampling pass has them; otherwise the pressure-only pass)
    const bool npt = npt_any(c);
    const int32_t fflags = kKick | (sample ? kSample : npt ? kPressure : 0);
    {
        Phase ph(c, 4, L.force_groups.size() > 1 || c->ml);
        if (inline_rebuild) launch_plain_forces(c, fflags, true);
        else launch_forces(c, fflags);
    }
    if (sample) {
        Phase ph(c, 5);
        launch_obs_reduce(c->st, dreps, c->n_rep, c->at<double>(L.partials), c->at<double>(L.acc),
                          c->at<int32_t>(L.counts), true, c->pair && !c->ml,
                          c->at<double>(L.cpart), L.cchunks);
    }
    // after the sample: observables see the box the step ran in; once a
    // barostat has run, replicas whose barostat is off have their pending
    // scalings cleared here too
    if (c->npt_used) {
        Phase ph(c, 5);
        c->rec_extra = 0;  // step n itself
        launch_barostat(c->st, c->at<RepDev>(L.reps), c->n_rep, c->at<double>(L.partials),
                        step_ref(c), c->at<int32_t>(L.status));
    }
    if (check) {  // the pair potential judges the surrogate on the same positions
        launch_plain_forces(c, kCompare);
        launch_obs_reduce(c->st, dreps, c->n_rep, c->at<double>(L.partials),
                          c->at<double>(L.ml_acc), c->at<int32_t>(L.ml_counts), false, false,
                          nullptr, 0);
    }
    c->rec_row = -1;
    c->rec_extra = 0;
}

bool sample_at(const qtb_ctx* c, int64_t step)
{
    return c->opt.obs_every > 0 && ((step + 1) % c->opt.obs_every) == 0;
}

bool check_at(const qtb_ctx* c, int64_t step)
{
    return c->ml && c->ml_check_every > 0 && ((step + 1) % c->ml_check_every) == 0;
}

// One kernel per step: pair potential, one bead group with G = P for every
// replica (P = 1, 2, 4, 8), pair-potential forces.
bool fused_step(const qtb_ctx* c)
{
    // (contexts with surrogate buffers keep the separate list kernel, whose
    // rebuilds also refresh the surrogate's lists)
    if (!c->pair || list_kernel(c) || !(c->opt.flags & QTB_OPT_FUSE)) return false;
    if (c->L.force_groups.size() != 1) return false;
    const int G = c->L.force_groups[0].first;
    for (const auto& R : c->reps)
        if (R.n_beads != G) return false;
    return true;
}

// Step row of the noise block with one kernel: the forces at the current
// positions close the previous step (sampling it if asked), then this step's
// update.  The first step of a run has no pending close: the update alone.
void record_fused(qtb_ctx* c, int row, bool sample_prev)
{
    const Layout& L = c->L;
    c->rec_row = row;
    c->rec_extra = 0;
    const size_t zs = c->opt.fir == QTB_FIR_FP64 ? 8 : 4;
    const char* zrow = c->at<char>(L.zeta) + (size_t)row * L.n_cols * zs;
    const RepDev* dreps = c->at<RepDev>(L.reps);
    if (!c->open) {
        Phase ph(c, 2);
        const BlockEntry* ub = c->at<BlockEntry>(L.blk_upd);
        for (auto& g : L.upd_groups) {
            const int b0 = g.second.first, nb = g.second.second - g.second.first;
            if (nb > 0)
                launch_update(c->st, c->fp64, true, g.first, L.upd_threads, dreps, ub + b0, nb, zrow,
                              c->at<int32_t>(L.status), step_ref(c), 0, L.n_cols);
        }
        c->open = true;
        c->rec_row = -1;
        return;
    }
    {
        Phase ph(c, 4);
        const auto& g = L.force_groups[0];
        const void* tab = c->fp64 ? (const void*)&c->tabd : (const void*)&c->tabf;
        launch_step_pair(c->st, c->fp64, g.first, c->W, dreps,
                         c->at<BlockEntry>(L.blk_force) + g.second.first,
                         g.second.second - g.second.first, tab, sample_prev ? kSample : 0,
                         c->at<double>(L.partials), c->n_rep, c->at<int32_t>(L.status),
                         step_ref(c), zrow);
    }
    if (sample_prev) {  // the one-kernel step sums the centroid kinetic energy itself
        Phase ph(c, 5);
        launch_obs_reduce(c->st, dreps, c->n_rep, c->at<double>(L.partials), c->at<double>(L.acc),
                          c->at<int32_t>(L.counts), true, c->pair && !c->ml, nullptr, 0);
    }
    c->rec_row = -1;
}

// End of a run of one-kernel steps: list check, forces, closing half-kick.
void close_steps(qtb_ctx* c)
{
    if (!c->open) return;
    const Layout& L = c->L;
    const bool sample = sample_at(c, c->step - 1);
    {
        Phase ph(c, 3, true);
        launch_rebuild(c);
    }
    {
        Phase ph(c, 4);
        launch_forces(c, kKick | (sample ? kSample : 0));
    }
    if (sample) {
        Phase ph(c, 5);
        launch_obs_reduce(c->st, c->at<RepDev>(L.reps), c->n_rep, c->at<double>(L.partials),
                          c->at<double>(L.acc), c->at<int32_t>(L.counts), true, c->pair && !c->ml,
                          c->at<double>(L.cpart), L.cchunks);
    }
    c->open = false;
}

// Kernels that open a noise block: advance the clock by K, K new white-noise
// rows, the FIR contraction for steps clock .. clock + K - 1.
void record_block_start(qtb_ctx* c)
{
    const Layout& L = c->L;
    const int maxNf = L.max_two_nf / 2;
    launch_clock(c->st, c->at<int64_t>(L.clock), L.K, true);
    if (L.eq9) {  // block noise: the paper's generator, whole blocks of n steps when due
        Phase ph(c, 1, true);
        launch_eq9(c->st, c->opt.fir == QTB_FIR_FP64, c->at<RepDev>(L.reps), c->at<FirTile>(L.tiles),
                   c->at<double>(L.eq9amp), maxNf + 1, c->at<double>(L.eq9tw), L.max_two_nf,
                   c->at<void>(L.zeta), L.n_cols, c->at<int64_t>(L.clock),
                   c->at<int64_t>(L.eq9mark), L.K);
        return;
    }
    gen_rows(c, maxNf, L.K);
    Phase ph(c, 1);
    launch_fir(c->st, c->opt.fir, L.K, c->at<FirTile>(L.tiles), (int)L.tilev.size(),
               c->at<void>(L.taps), c->at<void>(L.ring), c->at<void>(L.zeta), L.n_cols,
               c->at<int64_t>(L.clock), L.R, L.max_two_nf);
}


void one_step(qtb_ctx* c)
{
    const Layout& L = c->L;
    if (!c->ring_valid) prime_ring(c);
    if (c->block_start < 0 || c->block_row >= L.K) {
        // the clock advances by K per block: re-seat it if this block does not
        // follow the previous one (first block, new filter, new state)
        if (c->block_start < 0 || c->block_start + L.K != c->step)
            launch_clock(c->st, c->at<int64_t>(L.clock), c->step - L.K, false);
        record_block_start(c);
        c->block_start = c->step;
        c->block_row = 0;
    }
    if (fused_step(c))
        record_fused(c, c->block_row, sample_at(c, c->step - 1));
    else
        record_step(c, c->block_row, sample_at(c, c->step), check_at(c, c->step));
    c->step += 1;
    c->block_row += 1;
}

void drop_graph(qtb_ctx* c)
{
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
}

constexpr size_t kMaxGraphs = 32;
// Shortest row range of a noise block worth a graph of its own (shorter runs
// of steps launch eagerly).
constexpr int kMinGraphRows = 8;

// Rows r0 .. r1 - 1 of a noise block as one graph launch: at a block
// boundary r0 = 0 and the graph opens the new block (clock, white noise,
// FIR); otherwise it continues the current block from its next row.  r1 - r0
// is at most left.  Valid while the kernel arguments stay the same: they
// only depend on the workspace layout, the potential table, the force
// provider, the sampling / checking pattern and the row range, which are the
// key of the cached graphs.  Returns the number of steps launched (0: not
// taken, run eagerly).
int64_t graph_rows(qtb_ctx* c, int64_t left)
{
    const Layout& L = c->L;
    if (c->graph_failed || c->prof || c->st == nullptr) return 0;
    if (c->opt.flags & QTB_OPT_NO_GRAPH) return 0;
    if (c->opt.obs_every > 0 && L.K % c->opt.obs_every != 0) return 0;
    if (!c->ring_valid) return 0;
    const bool boundary = c->block_start < 0 || c->block_row >= L.K;
    const int r0 = boundary ? 0 : c->block_row;
    const int r1 = (int)std::min<int64_t>(L.K, r0 + left);
    if (r1 - r0 < kMinGraphRows && !(r0 == 0 && r1 == L.K)) return 0;
    const int64_t obs_phase = c->opt.obs_every > 0 ? c->step % c->opt.obs_every : 0;
    const int64_t chk_phase = (c->ml && c->ml_check_every > 0) ? c->step % c->ml_check_every : 0;
    const bool fused = fused_step(c);
    // the sequence also depends on whether a step's close is pending
    const std::array<int64_t, 4> key{obs_phase, chk_phase * 4 + (fused ? 2 : 0) + (c->open ? 1 : 0),
                                     r0, r1};
    hipGraphExec_t exec = nullptr;
    for (auto& g : c->graphs)
        if (g.first == key) exec = g.second;
    if (!exec) {
        if (c->graphs.size() >= kMaxGraphs) return 0;  // too many patterns: run eagerly
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            c->graph_failed = true;
            (void)hipGetLastError();
            return 0;
        }
        if (r0 == 0) record_block_start(c);
        const bool open0 = c->open;
        for (int r = r0; r < r1; ++r) {
            const int64_t n = c->step + (r - r0);
            if (fused) record_fused(c, r, sample_at(c, n - 1));
            else record_step(c, r, sample_at(c, n), check_at(c, n));
        }
        c->open = open0;  // capture records, it does not run
        if (hipStreamEndCapture(c->st, &g) != hipSuccess || !g ||
            hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            c->graph_failed = true;
            (void)hipGetLastError();
            return 0;
        }
        (void)hipGraphDestroy(g);
        c->graphs.push_back({key, exec});
    }
    if (boundary && (c->block_start < 0 || c->block_start + L.K != c->step))
        launch_clock(c->st, c->at<int64_t>(L.clock), c->step - L.K, false);
    if (hipGraphLaunch(exec, c->st) != hipSuccess) {
        drop_graph(c);
        c->graph_failed = true;
        (void)hipGetLastError();
        return 0;
    }
    if (boundary) c->block_start = c->step;
    c->block_row = r1;
    c->step += r1 - r0;
    if (fused) c->open = true;
    return r1 - r0;
}

// Make the force table of W current (host image, device copy, replica
// observable ranges); drops the captured graph, whose launches embed it.
qtb_status select_force_table(qtb_ctx* c, int W, int half)
{
    Layout& L = c->L;
    const int t = 2 * (W == 1 ? 0 : (W == 2 ? 1 : 2)) + (half ? 1 : 0);
    L.force = L.force_w[t];
    L.force_groups = L.force_groups_w[t];
    L.force_group_W.assign(L.force_groups.size(), W);
    L.force_group_t.assign(L.force_groups.size(), t);
    L.obs_b0 = L.obs_b0_w[t];
    L.obs_nb = L.obs_nb_w[t];
    c->W = W;
    c->half_groups = half != 0;
    for (int r = 0; r < c->n_rep; ++r) {
        c->rd[r].obs_block0 = L.obs_b0[r];
        c->rd[r].obs_nblocks = L.obs_nb[r];
    }
    QTB_HIP(c, hipMemcpyAsync(c->at<void>(L.blk_force), L.force.data(),
                              sizeof(BlockEntry) * L.force.size(), hipMemcpyHostToDevice, c->st));
    qtb_status s = upload_tables(c);
    if (s) return s;
    drop_graph(c);
    return QTB_OK;
}

// A table whose force group k comes from decomposition table tsel[k] (index
// 2 wi + gi as above): each bead-group width keeps its own waves per atom
// and bead-group split.  c->W and c->half_groups report the choice of the
// launch with the most workgroups.
qtb_status select_force_mix(qtb_ctx* c, const std::vector<int>& tsel)
{
    Layout& L = c->L;
    std::vector<BlockEntry> F;
    std::vector<std::pair<int, std::pair<int, int>>> FG;
    std::vector<int> gw, gt;
    std::vector<int> ob0(c->n_rep, 0), onb(c->n_rep, 0);
    for (size_t k = 0; k < tsel.size(); ++k) {
        const int t = tsel[k];
        const auto& src = L.force_groups_w[t][k];
        const int s0 = src.second.first, s1 = src.second.second, b0 = (int)F.size();
        F.insert(F.end(), L.force_w[t].begin() + s0, L.force_w[t].begin() + s1);
        FG.push_back({src.first, {b0, (int)F.size()}});
        gw.push_back(1 << (t / 2));
        gt.push_back(t);
        for (int r = 0; r < c->n_rep; ++r) {
            const int o = L.obs_b0_w[t][r];
            if (L.obs_nb_w[t][r] > 0 && o >= s0 && o < s1) {
                ob0[r] = b0 + (o - s0);
                onb[r] = L.obs_nb_w[t][r];
            }
        }
    }
    if (F.size() > L.max_force_blocks) return fail(c, QTB_E_STATE, "force table size");
    L.force = F;
    L.force_groups = FG;
    L.force_group_W = gw;
    L.force_group_t = gt;
    L.obs_b0 = ob0;
    L.obs_nb = onb;
    size_t kmax = 0;  // the launch with the most workgroups
    for (size_t k = 1; k < FG.size(); ++k)
        if (FG[k].second.second - FG[k].second.first >
            FG[kmax].second.second - FG[kmax].second.first)
            kmax = k;
    c->W = gw.empty() ? 1 : gw[kmax];
    c->half_groups = !gt.empty() && (gt[kmax] % 2) == 1;
    for (int r = 0; r < c->n_rep; ++r) {
        c->rd[r].obs_block0 = L.obs_b0[r];
        c->rd[r].obs_nblocks = L.obs_nb[r];
    }
    QTB_HIP(c, hipMemcpyAsync(c->at<void>(L.blk_force), L.force.data(),
                              sizeof(BlockEntry) * L.force.size(), hipMemcpyHostToDevice, c->st));
    qtb_status s = upload_tables(c);
    if (s) return s;
    drop_graph(c);
    return QTB_OK;
}

// Autotuner: time the pair-force kernel of the actual workload for every
// decomposition, waves per atom W in {1, 2, 4} times beads per wavefront G
// (the widest group that divides P, or half of it), forces only with no kick
// (the state is unchanged), and keep the fastest: one warm-up launch, then
// the best of five, separately for each launch (one per bead-group width, all
// replicas of that width).  The one-kernel step keeps whole ring polymers per
// wavefront.
qtb_status autotune(qtb_ctx* c)
{
    c->tuned = true;
    if (!c->pair || c->ml || (c->opt.flags & QTB_OPT_NO_AUTOTUNE)) return QTB_OK;
    bool can_half = !(c->opt.flags & QTB_OPT_FUSE);
    bool any_half = false;
    for (const auto& R : c->reps) any_half = any_half || bead_group(R.n_beads) > 1;
    can_half = can_half && any_half;
    hipEvent_t a = nullptr, b = nullptr;
    QTB_HIP(c, hipEventCreate(&a));
    QTB_HIP(c, hipEventCreate(&b));
    // each force group (one launch per bead-group width) is timed on its own
    // and keeps its own fastest decomposition
    const size_t ng = c->L.force_groups.size();
    std::vector<float> best(ng, 1e30f);
    std::vector<int> bestT(ng, c->L.force_group_t.empty() ? 0 : c->L.force_group_t[0]);
    for (int half = 0; half <= (can_half ? 1 : 0); ++half)
        for (int W : {1, 2, 4}) {
            qtb_status s = select_force_table(c, W, half);
            if (s) return s;
            for (size_t k = 0; k < ng; ++k) {
                float tmin = 1e30f;
                launch_plain_forces(c, 0, false, (int)k);  // warm-up (caches, first-touch)
                for (int rep = 0; rep < 5; ++rep) {
                    QTB_HIP(c, hipEventRecord(a, c->st));
                    launch_plain_forces(c, 0, false, (int)k);
                    QTB_HIP(c, hipEventRecord(b, c->st));
                    QTB_HIP(c, hipEventSynchronize(b));
                    float t = 0.0f;
                    QTB_HIP(c, hipEventElapsedTime(&t, a, b));
                    tmin = std::min(tmin, t);
                }
                if (tmin < best[k]) {
                    best[k] = tmin;
                    bestT[k] = c->L.force_group_t[k];
                }
            }
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    qtb_status s = ng == 1 ? select_force_table(c, 1 << (bestT[0] / 2), bestT[0] % 2)
                           : select_force_mix(c, bestT);
    if (s) return s;
    QTB_HIP(c, hipStreamSynchronize(c->st));
    return QTB_OK;
}

}  // namespace

// ====================================================================== ABI
namespace {
int64_t floor_div(int64_t a, int64_t b)
{
    const int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Transform every recorder segment completed by the work enqueued so far.
// The samples of steps before the last one are complete; so is the last
// step's unless its closing force pass is still pending (one-kernel steps).
void vdos_flush(qtb_ctx* c)
{
    const int64_t end = c->step - (c->open ? 1 : 0);
    for (int r = 0; r < c->n_rep; ++r) {
        VdosRec& v = c->vdos[r];
        if (!v.on || end <= v.start) continue;
        const int64_t e = c->opt.obs_every;
        const int64_t done = floor_div(end, e) - floor_div(v.start, e);  // steps s with (s + 1) % e == 0
        const int seg = v.plan.seg;
        while (v.n_seg < done / seg) {
            const double* base = v.at<double>(v.lay.trace) + (size_t)(v.n_seg & 1) * seg * v.n_dof;
            launch_vdos_segment(c->st, v.plan, base, v.n_dof, 1, v.n_dof,
                                v.at<double>(v.lay.w), v.at<double>(v.lay.tw),
                                v.at<double>(v.lay.part), v.at<double>(v.lay.stage),
                                v.at<double>(v.lay.spec), 1.0 / seg, v.n_seg > 0);
            ++v.n_seg;
        }
    }
}

void vdos_restart(qtb_ctx* c, int r)
{
    VdosRec& v = c->vdos[r];
    launch_fill(c->st, v.at<void>(v.lay.cnt), 2, 0);
    launch_fill(c->st, v.at<void>(v.lay.spec), 2 * (int64_t)v.plan.nk, 0);
    v.start = c->step;
    v.n_seg = 0;
}
}  // namespace

extern "C" {

size_t qtb_workspace_bytes(const qtb_potential* pot, const qtb_replica* reps, int32_t n_rep,
                           const qtb_options* opt)
{
    if (check_inputs(pot, reps, n_rep, opt)) return 0;
    Layout L;
    plan(pot, reps, n_rep, opt, L);
    return L.total;
}

qtb_status qtb_init(qtb_ctx** out, const qtb_potential* pot, const qtb_replica* reps,
                    int32_t n_rep, const qtb_options* opt, void* d_workspace, size_t ws_bytes,
                    void* hip_stream)
{
    if (!out) return fail(nullptr, QTB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (const char* e = check_inputs(pot, reps, n_rep, opt)) return fail(nullptr, QTB_E_INVALID, e);
    if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0)
        return fail(nullptr, QTB_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    qtb_ctx* c = new qtb_ctx();
    c->opt = *opt;
    c->st = (hipStream_t)hip_stream;
    c->fp64 = opt->prec == QTB_PREC_FP64;
    c->pair = pot->kind == QTB_POT_PAIR;
    c->kind = pot->kind;
    if (!c->pair && pot->kind != QTB_POT_HARMONIC) {
        c->osV0.assign(pot->onsite_V0, pot->onsite_V0 + pot->n_species);
        c->osd.assign(pot->onsite_d, pot->onsite_d + pot->n_species);
    }
    c->n_rep = n_rep;
    c->reps.assign(reps, reps + n_rep);
    const int ns = pot->n_species;
    c->mass.assign(pot->mass, pot->mass + ns);
    if (c->pair) {
        c->charge.assign(pot->charge, pot->charge + ns);
        c->bA.assign(pot->buck_A, pot->buck_A + ns * ns);
        c->brho.assign(pot->buck_rho, pot->buck_rho + ns * ns);
        c->bC.assign(pot->buck_C, pot->buck_C + ns * ns);
        c->alpha = pot->dsf_alpha;
        c->rc = pot->r_cut;
        c->skin = pot->skin;
    }
    plan(pot, reps, n_rep, opt, c->L);
    if (ws_bytes < c->L.total) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "workspace too small: %zu < %zu bytes", ws_bytes,
                      c->L.total);
        delete c;
        return fail(nullptr, QTB_E_NOMEM, msg);
    }
    c->ws = (char*)d_workspace;
    c->two_nf.assign(n_rep, 2);
    c->filter_ready.assign(n_rep, false);
    c->taps.assign(n_rep, {});
    c->eself.assign(n_rep, 0.0);
    c->rd.assign(n_rep, RepDev{});
    c->vdos.assign(n_rep, VdosRec{});
    c->species.resize(n_rep);
    c->homega.resize(n_rep);
    if (c->pair) {
        fill_pair_table(c, c->tabf);
        fill_pair_table(c, c->tabd);
    }
    qtb_status s = QTB_OK;
    auto bail = [&](qtb_status st) {
        std::string m = c->err;
        delete c;
        fail(nullptr, st, m);
        return st;
    };
    // zero every region first (fill kernel; the caller may capture later work)
    launch_fill(c->st, c->ws, (int64_t)(c->L.total / 4), 0);
    for (int r = 0; r < n_rep; ++r) {
        const qtb_replica& R = reps[r];
        c->species[r].assign(R.species, R.species + R.n_atoms);
        if (c->kind == QTB_POT_HARMONIC) c->homega[r].assign(R.harm_omega, R.harm_omega + R.n_atoms);
        else if (!c->pair) c->homega[r].assign(R.n_atoms, 0.0);
        fill_repdev(c, r);
        const Layout::Per& p = c->L.per[r];
        const int P = R.n_beads;
        std::vector<double> C(P * P), ring(3 * P);
        nm_matrix(P, C.data());
        const double h = 0.5 * R.dt;
        const double wP = c->rd[r].omega_P;
        for (int k = 0; k < P; ++k) {
            const double w = 2.0 * wP * std::sin(kPi * k / P);
            if (k == 0) {
                ring[k] = 1.0; ring[P + k] = h; ring[2 * P + k] = 0.0;
            } else {
                ring[k] = std::cos(w * h);
                ring[P + k] = std::sin(w * h) / w;
                ring[2 * P + k] = -w * std::sin(w * h);
            }
        }
        if ((s = hip_check(c, hipMemcpyAsync(c->at<void>(p.nm), C.data(), 8 * C.size(),
                                             hipMemcpyHostToDevice, c->st), "nm")) ||
            (s = hip_check(c, hipMemcpyAsync(c->at<void>(p.ring), ring.data(), 8 * ring.size(),
                                             hipMemcpyHostToDevice, c->st), "ring")) ||
            (s = hip_check(c, hipMemcpyAsync(c->at<void>(p.species), c->species[r].data(),
                                             4 * R.n_atoms, hipMemcpyHostToDevice, c->st), "species")) ||
            (s = hip_check(c, hipMemcpyAsync(c->at<void>(p.r0), R.d_pos,
                                             8 * (size_t)P * R.n_dims * R.n_atoms,
                                             hipMemcpyDeviceToDevice, c->st), "r0")))
            return bail(s);
        if (!c->pair &&
            (s = hip_check(c, hipMemcpyAsync(c->at<void>(p.homega), c->homega[r].data(),
                                             8 * R.n_atoms, hipMemcpyHostToDevice, c->st), "homega")))
            return bail(s);
        // default filter: white noise, sqrt(kT) delta
        c->taps[r].assign(2, 0.0);
        c->taps[r][1] = std::sqrt(opt->kB * R.T);
        c->filter_ready[r] = (R.noise == QTB_NOISE_CLASSICAL);
        if (c->pair) {
            double q2 = 0.0;
            for (int i = 0; i < R.n_atoms; ++i) q2 += c->charge[R.species[i]] * c->charge[R.species[i]];
            c->eself[r] = -(std::erfc(c->alpha * c->rc) / (2.0 * c->rc) + c->alpha / std::sqrt(kPi)) *
                          opt->coulomb_k * q2;
        }
    }
    if (c->L.eq9) {  // block noise: white amplitudes until a filter is built
        c->eq9amp.assign((size_t)n_rep * (c->L.max_two_nf / 2 + 1), 0.0);
        for (int r = 0; r < n_rep; ++r)
            if ((s = upload_eq9_amp(c, r, QTB_NOISE_CLASSICAL))) return bail(s);
        launch_vdos_twiddle(c->st, c->at<double>(c->L.eq9tw), c->L.max_two_nf);
        launch_eq9_invalidate(c->st, c->at<int64_t>(c->L.eq9mark));
    }
    if ((s = upload_tables(c))) return bail(s);
    if ((s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.blk_upd), c->L.upd.data(),
                                         sizeof(BlockEntry) * c->L.upd.size(), hipMemcpyHostToDevice, c->st), "blk")) ||
        (s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.blk_nl), c->L.nl.data(),
                                         sizeof(BlockEntry) * c->L.nl.size(), hipMemcpyHostToDevice, c->st), "blk")) ||
        (s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.blk_tb), c->L.tb.data(),
                                         sizeof(BlockEntry) * c->L.tb.size(), hipMemcpyHostToDevice, c->st), "blk")) ||
        (s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.blk_force), c->L.force.data(),
                                         sizeof(BlockEntry) * c->L.force.size(), hipMemcpyHostToDevice, c->st), "blk")))
        return bail(s);
    if (c->L.ml &&
        ((s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.blk_mlc), c->L.mlc.data(),
                                          sizeof(BlockEntry) * c->L.mlc.size(), hipMemcpyHostToDevice, c->st), "blk")) ||
         (s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.blk_mlm), c->L.mlm.data(),
                                          sizeof(BlockEntry) * c->L.mlm.size(), hipMemcpyHostToDevice, c->st), "blk")) ||
         (s = hip_check(c, hipMemcpyAsync(c->at<void>(c->L.ml_foff), c->L.foff.data(),
                                          sizeof(int64_t) * n_rep, hipMemcpyHostToDevice, c->st), "foff"))))
        return bail(s);
    for (int r = 0; r < n_rep; ++r)
        if ((s = upload_taps(c, r))) return bail(s);
    if ((s = refresh_forces(c))) return bail(s);
    if ((s = read_status(c))) return bail(s);
    *out = c;
    return QTB_OK;
}

qtb_status qtb_build_filter(qtb_ctx* c, int32_t replica, int32_t kind, int32_t two_nf,
                            double* taps_out)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < -1 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (kind < 0 || kind > 2) return fail(c, QTB_E_INVALID, "bad noise kind");
    if (two_nf < 2 || (two_nf & (two_nf - 1)) || two_nf > c->opt.max_two_nf)
        return fail(c, QTB_E_INVALID, "two_nf must be a power of two in [2, max_two_nf]");
    if (c->L.eq9 && two_nf != c->opt.max_two_nf)
        return fail(c, QTB_E_INVALID, "block noise: two_nf must equal max_two_nf (the block length)");
    const int r0 = replica < 0 ? 0 : replica, r1 = replica < 0 ? c->n_rep : replica + 1;
    for (int r = r0; r < r1; ++r)
        if (c->reps[r].noise != kind)
            return fail(c, QTB_E_STATE, "filter kind differs from the replica's noise kind");
    for (int r = r0; r < r1; ++r) {
        const qtb_replica& R = c->reps[r];
        c->taps[r].assign(two_nf, 0.0);
        design_taps(kind, R.T, R.n_beads, R.dt, two_nf, c->opt.hbar, c->opt.kB, c->taps[r].data());
        c->two_nf[r] = two_nf;
        c->rd[r].two_nf = two_nf;
        for (auto& t : c->L.tilev)
            if (t.rep == r) t.two_nf = two_nf;
        qtb_status s = upload_taps(c, r);
        if (s) return s;
        if (c->L.eq9 && (s = upload_eq9_amp(c, r, kind))) return s;
        c->filter_ready[r] = true;
        if (taps_out && replica >= 0) std::memcpy(taps_out, c->taps[r].data(), 8 * (size_t)two_nf);
    }
    qtb_status s = upload_tables(c);
    if (s) return s;
    if (c->L.eq9) launch_eq9_invalidate(c->st, c->at<int64_t>(c->L.eq9mark));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    // the current noise block (if any) was filtered with the old taps: restart
    c->block_start = -1;
    return QTB_OK;
}

qtb_status qtb_step(qtb_ctx* c, int64_t n_steps)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (n_steps < 0) return fail(c, QTB_E_INVALID, "n_steps must be >= 0");
    for (int r = 0; r < c->n_rep; ++r)
        if (!c->filter_ready[r]) return fail(c, QTB_E_STATE, "qtb_build_filter not called");
    if (!c->tuned && n_steps > 0) {
        qtb_status s = autotune(c);
        if (s) return s;
    }
    int64_t left = n_steps;
    while (left > 0) {
        if (const int64_t done = graph_rows(c, left)) {
            left -= done;
            vdos_flush(c);
            continue;
        }
        one_step(c);
        left -= 1;
        vdos_flush(c);
    }
    close_steps(c);
    vdos_flush(c);
    QTB_HIP(c, hipGetLastError());
    return QTB_OK;
}

qtb_status qtb_observables(qtb_ctx* c, int32_t replica, qtb_obs* out)
{
    if (!c || !out) return fail(c, QTB_E_INVALID, "null argument");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    double acc[kAcc];
    int32_t cnt = 0;
    QTB_HIP(c, hipMemcpyAsync(acc, c->at<double>(c->L.acc) + (size_t)replica * kAcc,
                              sizeof(acc), hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipMemcpyAsync(&cnt, c->at<int32_t>(c->L.counts) + replica, 4,
                              hipMemcpyDeviceToHost, c->st));
    qtb_status s = read_status(c);
    launch_fill(c->st, c->at<double>(c->L.acc) + (size_t)replica * kAcc, 2 * kAcc, 0);
    launch_fill(c->st, c->at<int32_t>(c->L.counts) + replica, 1, 0);
    QTB_HIP(c, hipStreamSynchronize(c->st));
    const qtb_replica& R = c->reps[replica];
    std::memset(out, 0, sizeof(*out));
    out->step = c->step + c->rd[replica].step_off;  // the replica's own step counter
    out->n_samples = cnt;
    if (cnt > 0) {
        const double inv = 1.0 / cnt;
        const double ke = acc[0] * inv, U = acc[1] * inv + (c->ml ? 0.0 : c->eself[replica]),
                     spr = acc[2] * inv, vir = acc[3] * inv, x2 = acc[4] * inv,
                     kec = acc[6] * inv;
        const double dof = (double)R.n_dims * R.n_atoms;
        out->kinetic = ke;
        out->potential = U;
        out->spring = spr;
        out->e_primitive = ke - spr + U;
        // centroid virial estimator with the measured centroid kinetic energy
        out->e_virial = kec - vir / (2.0 * R.n_beads) + U;
        out->t_kinetic = 2.0 * ke / (dof * R.n_beads * c->opt.kB);
        out->x2_mean = x2 / (dof * R.n_beads);
        if (c->pair && !c->ml) {
            out->virial_pair = acc[5] * inv;
            out->volume = acc[kNobs] * inv;
            out->pressure = acc[kNobs + 1] * inv;
        }
    }
    return s;
}

qtb_status qtb_get_state(qtb_ctx* c, int32_t replica, double* h_pos, double* h_vel,
                         int64_t* step)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    const qtb_replica& R = c->reps[replica];
    const size_t n = (size_t)R.n_beads * R.n_dims * R.n_atoms * 8;
    if (h_pos) QTB_HIP(c, hipMemcpyAsync(h_pos, R.d_pos, n, hipMemcpyDeviceToHost, c->st));
    if (h_vel) QTB_HIP(c, hipMemcpyAsync(h_vel, R.d_vel, n, hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (step) *step = c->step + c->rd[replica].step_off;
    return QTB_OK;
}

qtb_status qtb_set_state(qtb_ctx* c, int32_t replica, const double* h_pos, const double* h_vel,
                         int64_t step)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    const qtb_replica& R = c->reps[replica];
    const size_t n = (size_t)R.n_beads * R.n_dims * R.n_atoms * 8;
    if (h_pos) {
        QTB_HIP(c, hipMemcpyAsync(R.d_pos, h_pos, n, hipMemcpyHostToDevice, c->st));
        QTB_HIP(c, hipMemcpyAsync(c->at<void>(c->L.per[replica].r0), h_pos, n,
                                  hipMemcpyHostToDevice, c->st));
    }
    if (h_vel) QTB_HIP(c, hipMemcpyAsync(R.d_vel, h_vel, n, hipMemcpyHostToDevice, c->st));
    const int64_t off = step - c->step;
    // the next step opens a new noise block at the restored step, as the
    // first step of a new context would: a state restored from a checkpoint
    // then continues bit for bit like a context created from it
    c->ring_valid = false;
    c->block_start = -1;
    if (c->L.eq9) launch_eq9_invalidate(c->st, c->at<int64_t>(c->L.eq9mark));
    if (off != c->rd[replica].step_off) {
        c->rd[replica].step_off = off;
        qtb_status s = upload_tables(c);
        if (s) return s;
    }
    launch_fill(c->st, c->at<int32_t>(c->L.status), 1, 0);
    if (c->vdos[replica].on) vdos_restart(c, replica);  // the series starts afresh
    qtb_status s = refresh_forces(c);
    if (s) return s;
    return read_status(c);
}

qtb_status qtb_evaluate(qtb_ctx* c, int32_t replica, double* h_force, double* h_epot)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (c->pair) launch_rebuild(c);  // no-op unless a rebuild is pending
    launch_forces(c, kEvaluate);
    QTB_HIP(c, hipGetLastError());
    const qtb_replica& R = c->reps[replica];
    const Layout::Per& p = c->L.per[replica];
    const size_t nf = (size_t)R.n_beads * R.n_dims * R.n_atoms;
    if (h_force) {
        if (c->fp64) {
            QTB_HIP(c, hipMemcpyAsync(h_force, c->at<void>(p.force), 8 * nf, hipMemcpyDeviceToHost, c->st));
            QTB_HIP(c, hipStreamSynchronize(c->st));
        } else {
            std::vector<float> tmp(nf);
            QTB_HIP(c, hipMemcpyAsync(tmp.data(), c->at<void>(p.force), 4 * nf, hipMemcpyDeviceToHost, c->st));
            QTB_HIP(c, hipStreamSynchronize(c->st));
            for (size_t q = 0; q < nf; ++q) h_force[q] = tmp[q];
        }
    }
    if (h_epot) {
        std::vector<double> ea((size_t)R.n_beads * R.n_atoms);
        QTB_HIP(c, hipMemcpyAsync(ea.data(), c->at<void>(p.eatom), 8 * ea.size(), hipMemcpyDeviceToHost, c->st));
        QTB_HIP(c, hipStreamSynchronize(c->st));
        for (int s = 0; s < R.n_beads; ++s) {
            double e = 0.0;
            for (int i = 0; i < R.n_atoms; ++i) e += ea[(size_t)s * R.n_atoms + i];
            h_epot[s] = e + (c->ml ? 0.0 : c->eself[replica]);
        }
    }
    return read_status(c);
}

qtb_status qtb_get_noise(qtb_ctx* c, int32_t replica, double* h_zeta, int64_t* n0)
{
    if (!c || !h_zeta) return fail(c, QTB_E_INVALID, "null argument");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (c->block_start < 0) return fail(c, QTB_E_STATE, "no noise block computed yet");
    const qtb_replica& R = c->reps[replica];
    const int64_t D = (int64_t)R.n_dims * R.n_atoms * R.n_beads;
    const size_t zs = c->opt.fir == QTB_FIR_FP64 ? 8 : 4;
    const int K = c->L.K;
    std::vector<char> buf((size_t)K * D * zs);
    if (c->L.eq9) {  // rows (block_start + r) mod 2n of the block-noise ring
        const int64_t Z = c->L.zeta_rows;
        for (int r = 0; r < K;) {
            int64_t m = (c->block_start + r) % Z;
            if (m < 0) m += Z;
            const int run = (int)std::min<int64_t>(K - r, Z - m);
            QTB_HIP(c, hipMemcpy2DAsync(buf.data() + (size_t)r * D * zs, D * zs,
                                        c->at<char>(c->L.zeta) + (m * c->L.n_cols + c->L.dof_off[replica]) * zs,
                                        c->L.n_cols * zs, D * zs, run, hipMemcpyDeviceToHost, c->st));
            r += run;
        }
    } else {
        QTB_HIP(c, hipMemcpy2DAsync(buf.data(), D * zs,
                                    c->at<char>(c->L.zeta) + c->L.dof_off[replica] * zs,
                                    c->L.n_cols * zs, D * zs, K, hipMemcpyDeviceToHost, c->st));
    }
    QTB_HIP(c, hipStreamSynchronize(c->st));
    for (size_t q = 0; q < (size_t)K * D; ++q)
        h_zeta[q] = zs == 8 ? ((double*)buf.data())[q] : (double)((float*)buf.data())[q];
    if (n0) *n0 = c->block_start + c->rd[replica].step_off;
    return QTB_OK;
}

qtb_status qtb_gaussian(uint64_t seed, uint32_t stream, uint32_t tag, int64_t n0, int64_t n_rows,
                        uint32_t d0, uint32_t n_dof, double* d_out, void* hip_stream)
{
    if (!d_out || n_rows < 0) return fail(nullptr, QTB_E_INVALID, "bad gaussian arguments");
    launch_gaussian((hipStream_t)hip_stream, seed, stream, tag, n0, n_rows, d0, n_dof, d_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, QTB_E_DEVICE, hipGetErrorString(e));
    return QTB_OK;
}

size_t qtb_vdos_workspace_bytes(int32_t n_dof, int32_t seg, int32_t recorder)
{
    if (n_dof < 1 || seg < kVdosMinSeg || seg > kVdosMaxSeg || (seg & (seg - 1))) return 0;
    return vdos_layout(n_dof, seg, recorder != 0).total;
}

qtb_status qtb_vdos_spectrum(const double* d_v, int64_t n_samples, int32_t n_dof,
                             int64_t sample_stride, int64_t dof_stride, const double* d_weight,
                             int32_t seg, double* d_spec, void* d_workspace, size_t ws_bytes,
                             void* hip_stream)
{
    if (!d_v || !d_weight || !d_spec || n_samples < 0 || sample_stride < 1 || dof_stride < 1)
        return fail(nullptr, QTB_E_INVALID, "bad spectrum arguments");
    const size_t need = qtb_vdos_workspace_bytes(n_dof, seg, 0);
    if (need == 0) return fail(nullptr, QTB_E_INVALID, "n_dof >= 1 and seg a power of two in [16, 4096]");
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < need)
        return fail(nullptr, QTB_E_NOMEM, "spectrum workspace missing, misaligned or too small");
    const hipStream_t st = (hipStream_t)hip_stream;
    const VdosPlan p = vdos_plan(n_dof, seg);
    const VdosLayout l = vdos_layout(n_dof, seg, false);
    char* ws = (char*)d_workspace;
    const int64_t n_seg = n_samples / seg;
    if (n_seg == 0) {
        launch_fill(st, d_spec, 2 * (int64_t)p.nk, 0);
    } else {
        launch_vdos_twiddle(st, (double*)(ws + l.tw), seg);
        launch_vdos_sqrt(st, d_weight, n_dof, (double*)(ws + l.w));
        for (int64_t q = 0; q < n_seg; ++q)
            launch_vdos_segment(st, p, d_v + q * seg * sample_stride, sample_stride, dof_stride,
                                n_dof, (const double*)(ws + l.w), (const double*)(ws + l.tw),
                                (double*)(ws + l.part), (double*)(ws + l.stage), d_spec,
                                1.0 / ((double)seg * (double)n_seg), q > 0);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, QTB_E_DEVICE, hipGetErrorString(e));
    return QTB_OK;
}

qtb_status qtb_vdos_attach(qtb_ctx* c, int32_t replica, int32_t seg, void* d_workspace,
                           size_t ws_bytes)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    const qtb_replica& R = c->reps[replica];
    if (R.n_beads != 1)
        return fail(c, QTB_E_INVALID,
                    "velocity recorder needs P = 1: bead velocities carry no time correlations");
    if (c->opt.obs_every <= 0)
        return fail(c, QTB_E_STATE, "velocity recorder samples every obs_every steps, which is 0");
    const int n_dof = R.n_dims * R.n_atoms;
    const size_t need = qtb_vdos_workspace_bytes(n_dof, seg, 1);
    if (need == 0) return fail(c, QTB_E_INVALID, "seg must be a power of two in [16, 4096]");
    if ((int64_t)seg * c->opt.obs_every < c->L.K)
        return fail(c, QTB_E_INVALID, "seg * obs_every must be at least fir_block_K");
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < need)
        return fail(c, QTB_E_NOMEM, "recorder workspace missing, misaligned or too small");
    if (c->vdos[replica].on) QTB_HIP(c, hipStreamSynchronize(c->st));  // the old buffer's work
    VdosRec& v = c->vdos[replica];
    v = VdosRec{};
    v.on = true;
    v.ws = (char*)d_workspace;
    v.plan = vdos_plan(n_dof, seg);
    v.lay = vdos_layout(n_dof, seg, true);
    v.n_dof = n_dof;
    RepDev& d = c->rd[replica];
    d.vt = v.at<double>(v.lay.trace);
    d.vt_n = v.at<int64_t>(v.lay.cnt);
    d.vt_cap = 2 * seg;
    qtb_status s = upload_tables(c);
    if (s) return s;
    launch_vdos_twiddle(c->st, v.at<double>(v.lay.tw), seg);
    launch_vdos_weights(c->st, c->at<RepDev>(c->L.reps), replica, n_dof, v.at<double>(v.lay.w));
    vdos_restart(c, replica);
    QTB_HIP(c, hipGetLastError());
    return QTB_OK;
}

qtb_status qtb_vdos_read(qtb_ctx* c, int32_t replica, double* h_spec, int64_t* n_seg,
                         int32_t restart)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    VdosRec& v = c->vdos[replica];
    if (!v.on) return fail(c, QTB_E_STATE, "no velocity recorder attached to this replica");
    std::vector<double> buf(v.plan.nk);
    QTB_HIP(c, hipMemcpyAsync(buf.data(), v.at<double>(v.lay.spec), 8 * buf.size(),
                              hipMemcpyDeviceToHost, c->st));
    const qtb_status s = read_status(c);  // synchronises
    const int64_t n = v.n_seg;
    if (h_spec)
        for (int k = 0; k < v.plan.nk; ++k) h_spec[k] = n > 0 ? buf[k] / (double)n : 0.0;
    if (n_seg) *n_seg = n;
    if (restart) vdos_restart(c, replica);
    return s;
}

qtb_status qtb_vdos_detach(qtb_ctx* c, int32_t replica)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (!c->vdos[replica].on) return QTB_OK;
    QTB_HIP(c, hipStreamSynchronize(c->st));
    c->vdos[replica] = VdosRec{};
    RepDev& d = c->rd[replica];
    d.vt = nullptr;
    d.vt_n = nullptr;
    d.vt_cap = 0;
    qtb_status s = upload_tables(c);
    if (s) return s;
    QTB_HIP(c, hipStreamSynchronize(c->st));  // the buffer is the caller's again
    return QTB_OK;
}

namespace {
// Enable (kind 1 cell rescaling, 2 Langevin piston; q the compressibility or
// the piston friction) or disable (kind 0) the barostat of a replica.
qtb_status set_barostat(qtb_ctx* c, int32_t replica, int kind, double P0, double tau_p, double q)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (kind) {
        if (!c->pair || c->ml || c->L.ml)
            return fail(c, QTB_E_INVALID, "barostat: pair potential without surrogate buffers only");
        if (c->reps[replica].n_dims != 3)
            return fail(c, QTB_E_INVALID, "barostat: three dimensions only");
        if (c->opt.flags & QTB_OPT_FUSE)
            return fail(c, QTB_E_INVALID, "barostat: not with the one-kernel step");
        if (!(tau_p > 0.0) || !std::isfinite(tau_p) || !std::isfinite(P0))
            return fail(c, QTB_E_INVALID, "barostat: tau_p must be positive and finite");
        if (kind == 1 && !(q > 0.0 && std::isfinite(q)))
            return fail(c, QTB_E_INVALID, "barostat: beta_T must be positive and finite");
        if (kind == 2 && !(q >= 0.0 && std::isfinite(q)))
            return fail(c, QTB_E_INVALID, "piston: gamma_p must be non-negative and finite");
    }
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (qtb_status s = sync_boxes(c)) return s;
    RepDev& d = c->rd[replica];
    if (kind) c->npt_used = true;
    const qtb_replica& R = c->reps[replica];
    d.npt = kind;
    d.npt_P0 = kind ? P0 : 0.0;
    d.npt_tau = kind ? tau_p : 0.0;
    d.npt_beta = kind == 1 ? q : 0.0;
    d.npt_gp = kind == 2 ? q : 0.0;
    // piston mass (3 N P + 3) k_B T tau_p^2; the piston starts at rest
    d.npt_W = kind == 2 ? (3.0 * R.n_atoms * R.n_beads + 3.0) * d.kT * tau_p * tau_p : 0.0;
    d.npt_pe = 0.0;
    drop_graph(c);  // the step sequence changes
    qtb_status s = upload_tables_raw(c);  // synchronised above
    if (s) return s;
    // switched off: nothing follows the lists' scale any more, so they are
    // rebuilt from the current geometry (forces recomputed there)
    if (!kind && d.npt_S != 1.0 && (s = refresh_forces(c))) return s;
    QTB_HIP(c, hipStreamSynchronize(c->st));
    return read_status(c);
}
}  // namespace

qtb_status qtb_barostat(qtb_ctx* c, int32_t replica, double P0, double tau_p, double beta_T,
                        int32_t enable)
{
    return set_barostat(c, replica, enable ? 1 : 0, P0, tau_p, beta_T);
}

qtb_status qtb_barostat_piston(qtb_ctx* c, int32_t replica, double P0, double tau_p,
                               double gamma_p, int32_t enable)
{
    return set_barostat(c, replica, enable ? 2 : 0, P0, tau_p, gamma_p);
}

qtb_status qtb_get_barostat_state(qtb_ctx* c, int32_t replica, double* h_state)
{
    if (!c || !h_state) return fail(c, QTB_E_INVALID, "null argument");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (qtb_status s = sync_boxes(c)) return s;
    const RepDev& d = c->rd[replica];
    h_state[0] = d.npt_pe;
    h_state[1] = d.npt_sr;
    h_state[2] = d.npt_sv1;
    h_state[3] = d.npt_sv2;
    return read_status(c);
}

qtb_status qtb_set_barostat_state(qtb_ctx* c, int32_t replica, const double* h_state)
{
    if (!c || !h_state) return fail(c, QTB_E_INVALID, "null argument");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (!c->pair || c->ml || c->L.ml || (c->opt.flags & QTB_OPT_FUSE))
        return fail(c, QTB_E_INVALID, "barostat state: only where a barostat can run");
    for (int q = 0; q < 4; ++q)
        if (!std::isfinite(h_state[q]) || (q > 0 && !(h_state[q] > 0.0)))
            return fail(c, QTB_E_INVALID, "barostat state: non-finite or non-positive scaling");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (qtb_status s = sync_boxes(c)) return s;
    c->npt_used = true;  // the barostat kernel clears the scalings after use
    RepDev& d = c->rd[replica];
    d.npt_pe = h_state[0];
    d.npt_sr = h_state[1];
    d.npt_sv1 = h_state[2];
    d.npt_sv2 = h_state[3];
    // the skin the next step leaves for its list scale npt_S s
    d.half_skin = d.half_skin0 - std::max(0.0, 1.0 - d.npt_S * d.npt_sr) * 0.5 * d.r_cs;
    drop_graph(c);
    if (qtb_status s = upload_tables_raw(c)) return s;  // synchronised above
    QTB_HIP(c, hipStreamSynchronize(c->st));
    return read_status(c);
}

qtb_status qtb_get_box(qtb_ctx* c, int32_t replica, double* h_box)
{
    if (!c || !h_box) return fail(c, QTB_E_INVALID, "null argument");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (qtb_status s = sync_boxes(c)) return s;
    for (int a = 0; a < 3; ++a) h_box[a] = c->reps[replica].box[a];
    return read_status(c);
}

qtb_status qtb_set_replica_skin(qtb_ctx* c, int32_t replica, double skin)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (!c->pair) return fail(c, QTB_E_INVALID, "replica skin: pair potential only");
    if (c->ml || c->L.ml)
        return fail(c, QTB_E_INVALID, "replica skin: the surrogate's lists keep the potential's skin");
    if (replica < -1 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    if (!(skin >= 0.0) || skin > c->skin)
        return fail(c, QTB_E_INVALID, "replica skin must lie in [0, the potential's skin]");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (qtb_status s = sync_boxes(c)) return s;
    for (int r = 0; r < c->n_rep; ++r) {
        if (replica >= 0 && r != replica) continue;
        RepDev& d = c->rd[r];
        d.r_cs = c->rc + skin;
        d.half_skin0 = 0.5 * skin;
        d.half_skin = d.half_skin0 - std::max(0.0, 1.0 - d.npt_S * d.npt_sr) * 0.5 * d.r_cs;
    }
    drop_graph(c);
    if (qtb_status s = upload_tables_raw(c)) return s;
    if (qtb_status s = refresh_forces(c)) return s;  // lists rebuilt with the new radius
    return read_status(c);
}

qtb_status qtb_set_decomposition(qtb_ctx* c, int32_t waves_per_atom, int32_t half_groups)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (!c->pair) return fail(c, QTB_E_INVALID, "decomposition: pair potential only");
    if (waves_per_atom != 1 && waves_per_atom != 2 && waves_per_atom != 4)
        return fail(c, QTB_E_INVALID, "waves_per_atom must be 1, 2 or 4");
    if (c->ml && (waves_per_atom != 1 || half_groups))
        return fail(c, QTB_E_INVALID, "with the surrogate attached: 1 wavefront, whole groups");
    if (half_groups && (c->opt.flags & QTB_OPT_FUSE))
        return fail(c, QTB_E_INVALID, "the one-kernel step keeps whole groups");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    if (qtb_status s = select_force_table(c, waves_per_atom, half_groups ? 1 : 0)) return s;
    c->tuned = true;  // pinned: no autotuning at the next step
    QTB_HIP(c, hipStreamSynchronize(c->st));
    return read_status(c);
}

qtb_status qtb_get_decomposition(qtb_ctx* c, int32_t* waves_per_atom, int32_t* half_groups)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (waves_per_atom) *waves_per_atom = c->W;
    if (half_groups) *half_groups = c->half_groups ? 1 : 0;
    return QTB_OK;
}

namespace {
// Index of the force launch of bead-group width G (its whole-group width),
// or -1.
int force_group_of(const qtb_ctx* c, int32_t G)
{
    const auto& FG = c->L.force_groups_w[0];
    for (size_t k = 0; k < FG.size(); ++k)
        if (FG[k].first == G) return (int)k;
    return -1;
}
}  // namespace

qtb_status qtb_set_group_decomposition(qtb_ctx* c, int32_t group_width, int32_t waves_per_atom,
                                       int32_t half_groups)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (!c->pair || c->ml) return fail(c, QTB_E_INVALID, "group decomposition: pair potential, no surrogate");
    if (c->opt.flags & QTB_OPT_FUSE)
        return fail(c, QTB_E_INVALID, "the one-kernel step takes one decomposition");
    if (waves_per_atom != 1 && waves_per_atom != 2 && waves_per_atom != 4)
        return fail(c, QTB_E_INVALID, "waves_per_atom must be 1, 2 or 4");
    const int k = force_group_of(c, group_width);
    if (k < 0) return fail(c, QTB_E_INVALID, "no force launch of that bead-group width");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    std::vector<int> tsel = c->L.force_group_t;
    tsel[k] = 2 * (waves_per_atom == 1 ? 0 : (waves_per_atom == 2 ? 1 : 2)) + (half_groups ? 1 : 0);
    if (qtb_status s = select_force_mix(c, tsel)) return s;
    c->tuned = true;  // pinned: no autotuning at the next step
    QTB_HIP(c, hipStreamSynchronize(c->st));
    return read_status(c);
}

qtb_status qtb_get_group_decomposition(qtb_ctx* c, int32_t group_width, int32_t* waves_per_atom,
                                       int32_t* half_groups)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (!c->pair) return fail(c, QTB_E_INVALID, "group decomposition: pair potential only");
    const int k = force_group_of(c, group_width);
    if (k < 0) return fail(c, QTB_E_INVALID, "no force launch of that bead-group width");
    const int t = c->L.force_group_t[k];
    if (waves_per_atom) *waves_per_atom = 1 << (t / 2);
    if (half_groups) *half_groups = t % 2;
    return QTB_OK;
}

qtb_status qtb_profile(qtb_ctx* c, int32_t enable)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    c->prof = enable != 0;
    c->ev_used = 0;
    c->ev_marks.clear();
    return QTB_OK;
}

qtb_status qtb_profile_read(qtb_ctx* c, double* ms, int64_t* launches)
{
    if (!c || !ms || !launches) return fail(c, QTB_E_INVALID, "null argument");
    QTB_HIP(c, hipStreamSynchronize(c->st));
    for (int q = 0; q < QTB_N_PHASES; ++q) {
        ms[q] = 0.0;
        launches[q] = 0;
    }
    for (auto& m : c->ev_marks) {
        float t = 0.0f;
        QTB_HIP(c, hipEventElapsedTime(&t, c->ev_pool[m.second], c->ev_pool[m.second + 1]));
        ms[m.first] += t;
        launches[m.first] += 1;
    }
    return QTB_OK;
}

// ============================================================ surrogate
static qtb_status ml_fail(qtb_ml* m, qtb_status st, const std::string& msg)
{
    if (m) m->err = msg;
    else g_static_err = msg;
    return st;
}

static qtb_status ml_upload_norm(qtb_ml* m)
{
    std::vector<float> mu(2 * kMlFeat), isd(2 * kMlFeat);
    for (int q = 0; q < 2 * kMlFeat; ++q) {
        mu[q] = (float)m->norm[q];
        isd[q] = (float)m->norm[2 * kMlFeat + q];
    }
    if (hipMemcpyAsync(m->at<void>(m->mu), mu.data(), 4 * mu.size(), hipMemcpyHostToDevice, m->st) ||
        hipMemcpyAsync(m->at<void>(m->isd), isd.data(), 4 * isd.size(), hipMemcpyHostToDevice, m->st) ||
        hipMemcpyAsync(m->at<void>(m->e0), m->norm.data() + 4 * kMlFeat, 16, hipMemcpyHostToDevice, m->st) ||
        hipStreamSynchronize(m->st))
        return ml_fail(m, QTB_E_DEVICE, "normalisation upload");
    return QTB_OK;
}

static void ml_reset_adam(qtb_ml* m)
{
    launch_fill(m->st, m->at<void>(m->m1), kMlParams, 0);
    launch_fill(m->st, m->at<void>(m->m2), kMlParams, 0);
    m->t = 0;
}

size_t qtb_ml_workspace_bytes(void)
{
    qtb_ml m;
    ml_layout(m);
    return m.total;
}

qtb_status qtb_ml_create(qtb_ml** out, double r_cut, double r_min, void* d_workspace,
                         size_t ws_bytes, void* hip_stream)
{
    if (!out) return ml_fail(nullptr, QTB_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!(r_min > 0.0) || !(r_cut > r_min)) return ml_fail(nullptr, QTB_E_INVALID, "need 0 < r_min < r_cut");
    if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0)
        return ml_fail(nullptr, QTB_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    qtb_ml* m = new qtb_ml();
    ml_layout(*m);
    if (ws_bytes < m->total) {
        delete m;
        return ml_fail(nullptr, QTB_E_NOMEM, "model workspace too small");
    }
    m->st = (hipStream_t)hip_stream;
    m->ws = (char*)d_workspace;
    m->r_cut = r_cut;
    m->r_min = r_min;
    m->norm.assign(4 * kMlFeat + 2, 0.0);
    for (int q = 0; q < 2 * kMlFeat; ++q) m->norm[2 * kMlFeat + q] = 1.0;
    launch_fill(m->st, m->ws, (int64_t)(m->total / 4), 0);
    qtb_status s = ml_upload_norm(m);
    if (s) {
        std::string e = m->err;
        delete m;
        return ml_fail(nullptr, s, e);
    }
    *out = m;
    return QTB_OK;
}

qtb_status qtb_ml_init_params(qtb_ml* m, uint64_t seed)
{
    if (!m) return ml_fail(nullptr, QTB_E_INVALID, "model is NULL");
    launch_ml_init(m->st, m->at<float>(m->master), seed);
    launch_ml_round(m->st, m->at<float>(m->master), m->at<uint16_t>(m->wq), kMlParams);
    ml_reset_adam(m);
    if (hipStreamSynchronize(m->st) != hipSuccess) return ml_fail(m, QTB_E_DEVICE, "init");
    return QTB_OK;
}

qtb_status qtb_ml_set_params(qtb_ml* m, const float* h_params, const double* h_norm)
{
    if (!m) return ml_fail(nullptr, QTB_E_INVALID, "model is NULL");
    if (h_params) {
        if (hipMemcpyAsync(m->at<void>(m->master), h_params, 4 * (size_t)kMlParams,
                           hipMemcpyHostToDevice, m->st) != hipSuccess)
            return ml_fail(m, QTB_E_DEVICE, "params upload");
        launch_ml_round(m->st, m->at<float>(m->master), m->at<uint16_t>(m->wq), kMlParams);
        ml_reset_adam(m);
    }
    if (h_norm) {
        for (int q = 0; q < 2 * kMlFeat; ++q)
            if (!(h_norm[2 * kMlFeat + q] > 0.0)) return ml_fail(m, QTB_E_INVALID, "inv_sd must be > 0");
        m->norm.assign(h_norm, h_norm + 4 * kMlFeat + 2);
        return ml_upload_norm(m);
    }
    if (hipStreamSynchronize(m->st) != hipSuccess) return ml_fail(m, QTB_E_DEVICE, "set_params");
    return QTB_OK;
}

qtb_status qtb_ml_get_params(qtb_ml* m, float* h_params, float* h_used, double* h_norm)
{
    if (!m) return ml_fail(nullptr, QTB_E_INVALID, "model is NULL");
    std::vector<float> master(kMlParams);
    std::vector<uint16_t> wq(kMlParams);
    if (hipMemcpyAsync(master.data(), m->at<void>(m->master), 4 * (size_t)kMlParams,
                       hipMemcpyDeviceToHost, m->st) ||
        hipMemcpyAsync(wq.data(), m->at<void>(m->wq), 2 * (size_t)kMlParams, hipMemcpyDeviceToHost,
                       m->st) ||
        hipStreamSynchronize(m->st))
        return ml_fail(m, QTB_E_DEVICE, "params download");
    if (h_params) std::memcpy(h_params, master.data(), 4 * (size_t)kMlParams);
    if (h_used) {
        for (int p = 0; p < kMlParams; ++p) {
            const int off = p % kMlParamsSp;
            const bool weight = off < kMlOffB1 || (off >= kMlOffW2 && off < kMlOffB2) ||
                                (off >= kMlOffW3 && off < kMlOffB3);
            if (weight) {
                const uint32_t u = (uint32_t)wq[p] << 16;
                std::memcpy(&h_used[p], &u, 4);
            } else {
                h_used[p] = master[p];
            }
        }
    }
    if (h_norm) std::memcpy(h_norm, m->norm.data(), 8 * m->norm.size());
    return QTB_OK;
}

static qtb_status ml_ready(qtb_ctx* c, qtb_ml* m)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (!m) return fail(c, QTB_E_INVALID, "model is NULL");
    if (!c->L.ml) return fail(c, QTB_E_STATE, "context created without ml_r_cut");
    if (c->fp64) return fail(c, QTB_E_UNSUPPORTED, "the surrogate runs in FP32 precision only");
    if (m->r_cut > c->opt.ml_r_cut + 1e-12)
        return fail(c, QTB_E_INVALID, "model r_cut exceeds the context's ml_r_cut");
    return QTB_OK;
}

qtb_status qtb_ml_attach(qtb_ctx* c, qtb_ml* m, int32_t check_every)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (check_every < 0) return fail(c, QTB_E_INVALID, "check_every must be >= 0");
    if (m) {
        qtb_status s = ml_ready(c, m);
        if (s) return s;
    }
    QTB_HIP(c, hipStreamSynchronize(c->st));
    c->ml = m;
    c->ml_check_every = m ? check_every : 0;
    drop_graph(c);
    qtb_status s = QTB_OK;
    if (m) {
        // one wavefront per atom in the gather: the W = 1 table
        if ((s = select_force_table(c, 1, 0))) return s;
        c->tuned = true;
        launch_fill(c->st, c->at<double>(c->L.ml_acc), 2 * kAcc * c->n_rep, 0);
        launch_fill(c->st, c->at<int32_t>(c->L.ml_counts), c->n_rep, 0);
    } else {
        c->tuned = false;
    }
    // forces of the new provider for the next half-kick
    if (m) launch_rebuild(c);
    launch_forces(c, 0);
    QTB_HIP(c, hipGetLastError());
    return read_status(c);
}

qtb_status qtb_ml_evaluate(qtb_ctx* c, qtb_ml* m, int32_t replica, double* h_force,
                           double* h_epot, float* h_desc, float* h_dEdG)
{
    qtb_status s = ml_ready(c, m);
    if (s) return s;
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    launch_rebuild(c);  // no-op unless a rebuild is pending
    launch_ml_forces(c, m, kEvaluate);
    QTB_HIP(c, hipGetLastError());
    const qtb_replica& R = c->reps[replica];
    const Layout::Per& p = c->L.per[replica];
    const size_t N = R.n_atoms, P = R.n_beads;
    if (h_force) {
        std::vector<float> tmp(P * 3 * N);
        QTB_HIP(c, hipMemcpyAsync(tmp.data(), c->at<void>(p.force), 4 * tmp.size(), hipMemcpyDeviceToHost, c->st));
        QTB_HIP(c, hipStreamSynchronize(c->st));
        for (size_t q = 0; q < tmp.size(); ++q) h_force[q] = tmp[q];
    }
    if (h_epot) {
        std::vector<double> ea(P * N);
        QTB_HIP(c, hipMemcpyAsync(ea.data(), c->at<void>(p.eatom), 8 * ea.size(), hipMemcpyDeviceToHost, c->st));
        QTB_HIP(c, hipStreamSynchronize(c->st));
        for (size_t b = 0; b < P; ++b) {
            double e = 0.0;
            for (size_t i = 0; i < N; ++i) e += ea[b * N + i];
            h_epot[b] = e;
        }
    }
    if (h_desc)
        QTB_HIP(c, hipMemcpyAsync(h_desc, c->at<void>(p.mlG), 4 * P * N * kMlFeat, hipMemcpyDeviceToHost, c->st));
    if (h_dEdG)
        QTB_HIP(c, hipMemcpyAsync(h_dEdG, c->at<void>(p.mlg), 4 * P * N * kMlFeat, hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    // the stepping provider's forces back in place for the next half-kick
    if (c->ml != m) launch_forces(c, 0);
    QTB_HIP(c, hipGetLastError());
    return read_status(c);
}

qtb_status qtb_ml_fit_norm(qtb_ctx* c, qtb_ml* m, const double* d_eref)
{
    qtb_status s = ml_ready(c, m);
    if (s) return s;
    if (!d_eref) return fail(c, QTB_E_INVALID, "d_eref is NULL");
    launch_rebuild(c);
    launch_ml_forces(c, m, kEvaluate);  // descriptors of every centre
    launch_ml_stats(c->st, c->at<RepDev>(c->L.reps), c->n_rep, c->at<double>(c->L.ml_stats));
    std::vector<double> st(2 * kMlFeat * 2 + 2), eref(c->n_rep);
    QTB_HIP(c, hipMemcpyAsync(st.data(), c->at<void>(c->L.ml_stats), 8 * st.size(), hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipMemcpyAsync(eref.data(), d_eref, 8 * (size_t)c->n_rep, hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    std::vector<double> norm(4 * kMlFeat + 2, 0.0);
    for (int a = 0; a < 2; ++a) {
        const double n = st[2 * kMlFeat * 2 + a];
        for (int f = 0; f < kMlFeat; ++f) {
            const double s1 = st[(a * kMlFeat + f) * 2], s2 = st[(a * kMlFeat + f) * 2 + 1];
            const double mu = n > 0 ? s1 / n : 0.0;
            const double var = n > 0 ? std::max(s2 / n - mu * mu, 0.0) : 1.0;
            norm[a * kMlFeat + f] = mu;
            norm[2 * kMlFeat + a * kMlFeat + f] = 1.0 / std::max(std::sqrt(var), 1e-3);
        }
    }
    double e0 = 0.0;
    for (int r = 0; r < c->n_rep; ++r) e0 += eref[r] / c->reps[r].n_atoms;
    e0 /= c->n_rep;
    norm[4 * kMlFeat] = norm[4 * kMlFeat + 1] = e0;
    m->norm = norm;
    s = ml_upload_norm(m);
    if (s) return fail(c, s, m->err);
    if (c->ml != m) launch_forces(c, 0);
    return read_status(c);
}

qtb_status qtb_ml_train_step(qtb_ctx* c, qtb_ml* m, const double* d_eref, const double* d_fref,
                             double w_E, double w_F, double lr, int32_t update, double* loss_out,
                             float* h_grad)
{
    qtb_status s = ml_ready(c, m);
    if (s) return s;
    if (!c->L.ml_train) return fail(c, QTB_E_STATE, "context created without QTB_OPT_ML_TRAIN");
    if (!d_eref || !d_fref) return fail(c, QTB_E_INVALID, "reference arrays missing");
    if (!(w_E >= 0.0) || !(w_F >= 0.0) || !(lr >= 0.0)) return fail(c, QTB_E_INVALID, "weights and lr must be >= 0");
    double n_tot = 0.0;
    for (int r = 0; r < c->n_rep; ++r) {
        if (c->reps[r].n_beads != 1) return fail(c, QTB_E_UNSUPPORTED, "training frames have one bead");
        n_tot += c->reps[r].n_atoms;
    }
    const Layout& L = c->L;
    const RepDev* dreps = c->at<RepDev>(L.reps);
    const MlDev md = m->dev();
    launch_rebuild(c);
    launch_ml_forces(c, m, kEvaluate);
    launch_ml_loss(c->st, dreps, c->n_rep, d_eref, d_fref, c->at<int64_t>(L.ml_foff), w_E, w_F,
                   n_tot, c->at<double>(L.ml_loss));
    launch_ml_jvp(c->st, c->fp64, dreps, md, c->at<BlockEntry>(L.blk_mlc), (int)L.mlc.size(),
                  step_ref(c));
    launch_ml_train_mlp(c->st, dreps, md, c->at<BlockEntry>(L.blk_mlm), (int)L.mlm.size());
    launch_ml_wgrad(c->st, dreps, md, c->at<BlockEntry>(L.blk_mlm), (int)L.mlm.size(),
                    c->at<float>(L.ml_wpart), m->at<float>(m->grad));
    if (update) {
        m->t += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = (float)(1.0 - std::pow(0.9, (double)m->t));
        const float c2 = (float)(1.0 - std::pow(0.999, (double)m->t));
        launch_ml_adam(c->st, m->at<float>(m->master), m->at<uint16_t>(m->wq), m->at<float>(m->m1),
                       m->at<float>(m->m2), m->at<float>(m->grad), kMlParams, (float)lr, b1, b2,
                       1e-8f, c1, c2);
    }
    QTB_HIP(c, hipGetLastError());
    if (loss_out) {
        std::vector<double> parts(c->n_rep);
        QTB_HIP(c, hipMemcpyAsync(parts.data(), c->at<void>(L.ml_loss), 8 * parts.size(), hipMemcpyDeviceToHost, c->st));
        QTB_HIP(c, hipStreamSynchronize(c->st));
        double t = 0.0;
        for (double x : parts) t += x;
        *loss_out = t;
    }
    if (h_grad) {
        QTB_HIP(c, hipMemcpyAsync(h_grad, m->at<void>(m->grad), 4 * (size_t)kMlParams, hipMemcpyDeviceToHost, c->st));
        QTB_HIP(c, hipStreamSynchronize(c->st));
    }
    if (c->ml != m) launch_forces(c, 0);
    return read_status(c);
}

qtb_status qtb_ml_check(qtb_ctx* c, int32_t replica, double* rmse, double* rel_rmse,
                        int64_t* n_checks)
{
    if (!c) return fail(nullptr, QTB_E_INVALID, "ctx is NULL");
    if (!c->L.ml) return fail(c, QTB_E_STATE, "context created without ml_r_cut");
    if (replica < 0 || replica >= c->n_rep) return fail(c, QTB_E_INVALID, "replica out of range");
    double acc[kNobs];
    int32_t cnt = 0;
    QTB_HIP(c, hipMemcpyAsync(acc, c->at<double>(c->L.ml_acc) + (size_t)replica * kAcc, sizeof(acc),
                              hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipMemcpyAsync(&cnt, c->at<int32_t>(c->L.ml_counts) + replica, 4, hipMemcpyDeviceToHost, c->st));
    QTB_HIP(c, hipStreamSynchronize(c->st));
    launch_fill(c->st, c->at<double>(c->L.ml_acc) + (size_t)replica * kAcc, 2 * kAcc, 0);
    launch_fill(c->st, c->at<int32_t>(c->L.ml_counts) + replica, 1, 0);
    QTB_HIP(c, hipStreamSynchronize(c->st));
    const qtb_replica& R = c->reps[replica];
    const double n = 3.0 * R.n_atoms * R.n_beads * std::max(cnt, 1);
    if (rmse) *rmse = cnt ? std::sqrt(acc[0] / n) : 0.0;
    if (rel_rmse) *rel_rmse = (cnt && acc[1] > 0) ? std::sqrt(acc[0] / acc[1]) : 0.0;
    if (n_checks) *n_checks = cnt;
    return QTB_OK;
}

const char* qtb_ml_last_error(const qtb_ml* m)
{
    if (m) return m->err.c_str();
    return g_static_err.c_str();
}

void qtb_ml_destroy(qtb_ml* m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->st);
    delete m;
}

const char* qtb_last_error(const qtb_ctx* c)
{
    if (c) return c->err.c_str();
    return g_static_err.c_str();
}

void qtb_destroy(qtb_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    drop_graph(c);
    for (hipStream_t x : c->side) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
    }
    for (hipEvent_t e : c->side_ev) (void)hipEventDestroy(e);
    delete c;
}

qtb_status qtb_filter_taps(int32_t kind, double T, int32_t n_beads, double dt, int32_t two_nf,
                           double hbar, double kB, double* taps_out)
{
    if (!taps_out) return QTB_E_INVALID;
    if (kind < QTB_NOISE_CLASSICAL || kind > QTB_NOISE_QTB_PIMD) return QTB_E_INVALID;
    if (!(T > 0.0) || !(dt > 0.0) || !(hbar > 0.0) || !(kB > 0.0)) return QTB_E_INVALID;
    if (n_beads < 1 || n_beads > 64) return QTB_E_INVALID;
    if (two_nf < 2 || two_nf > 8192 || (two_nf & (two_nf - 1))) return QTB_E_INVALID;
    design_taps(kind, T, n_beads, dt, two_nf, hbar, kB, taps_out);
    for (int32_t k = 0; k < two_nf; ++k)
        if (!std::isfinite(taps_out[k])) return QTB_E_NONFINITE;
    return QTB_OK;
}

const char* qtb_version(void) { return "qtb-mi355x 0.1 (gfx950)"; }

}  // extern "C"
