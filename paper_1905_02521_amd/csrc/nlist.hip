// nlist.hip -- Verlet neighbour lists shared by all beads of a replica.
//
// The list is built from the bead centroids r_ref with radius r_cut + skin
// and stores, per entry, the reference displacement d_ij = r_ref_i - r_ref_j
// - S (S the periodic image shift) plus j.  Every bead then measures a pair
// as d_ij + u_i - u_j with u = r - r_ref small, which keeps the FP32 force
// path accurate at any box size and lets positions stay unwrapped.  All
// periodic images within range are listed (boxes smaller than twice the
// cut-off, e.g. 3x3x3 rock-salt cells at r_cut = 9 A, need them).
//
// The kernel runs every step and returns at once unless the update kernel
// flagged that some bead left the ball of radius devb_i + skin/2 around its
// reference.  Pairs are listed within r_cut + skin + dev_i + dev_j (dev: the
// largest bead-to-centroid distance of the atom at the build), so no pair
// within r_cut can be missing before that happens.  The build is all-pairs,
// one wavefront per atom, deterministic order.
#include "qtb_internal.h"

namespace qtb {
namespace {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

__device__ __forceinline__ float bits_f(int32_t b, float) { return __int_as_float(b); }
__device__ __forceinline__ double bits_f(int32_t b, double) { return __longlong_as_double((long long)b); }

// Bead centroids of the current positions (the update kernel writes them
// every step; this pass is for init and set_state).
__global__ void __launch_bounds__(256) k_centroids(const RepDev* __restrict__ reps,
                                                   const BlockEntry* __restrict__ blocks,
                                                   const StepRef sync)
{
    const int p = step_index(sync).p;
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int N = R.N, P = R.P;
    const int ii = be.atom0 + threadIdx.x;
    if (threadIdx.x >= 4 || ii >= N) return;
    double c[3];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < P; ++b) s += R.pos[((size_t)b * 3 + a) * N + ii];
        c[a] = s / P;
        R.cnb[p][(size_t)a * N + ii] = c[a];
    }
    double d2max = 0.0;
    for (int b = 0; b < P; ++b) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double x = R.pos[((size_t)b * 3 + a) * N + ii] - c[a];
            d2 += x * x;
        }
        d2max = fmax(d2max, d2);
    }
    R.devn[p][ii] = sqrt(d2max);
}

// Squared lower bound of the periodic distance from (x, y, z) to the box
// b = (lo xyz, hi xyz): per axis, the distance of the point's nearest image
// to the interval (0 when the interval spans the period).
__device__ __forceinline__ double box_dist2(double x, double y, double z, const double* b,
                                            double Lx, double Ly, double Lz, double iLx,
                                            double iLy, double iLz)
{
    auto axis = [](double p, double lo, double hi, double L, double iL) {
        const double h = 0.5 * (hi - lo);
        if (h >= 0.5 * L) return 0.0;
        double d = p - 0.5 * (lo + hi);
        d -= L * rint(d * iL);
        return fmax(fabs(d) - h, 0.0);
    };
    const double dx = axis(x, b[0], b[3], Lx, iLx), dy = axis(y, b[1], b[4], Ly, iLy),
                 dz = axis(z, b[2], b[5], Lz, iLz);
    return dx * dx + dy * dy + dz * dz;
}

// Bounds of the centroids of each tile of kListTile atoms and the largest
// spread in it, for the list kernel's pruning; one block per tile.
__global__ void __launch_bounds__(256) k_tile_box(const RepDev* __restrict__ reps,
                                                 const BlockEntry* __restrict__ tiles,
                                                 int n_tiles, const int32_t* __restrict__ status,
                                                 const StepRef sync)
{
    __shared__ double red[7][4];
    const StepIdx si = step_index(sync);
    if (status[kAnyRebuild + si.f] == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = blockIdx.x; e < n_tiles; e += gridDim.x) {
        const BlockEntry be = tiles[e];
        const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
        if (R.rflag[si.f] == 0) continue;  // uniform over the block
        const int N = R.N;
        const int j = be.atom0 + threadIdx.x;
        double v[7];
        if (j < N) {
            for (int a = 0; a < 3; ++a) v[a] = v[3 + a] = R.cnb[si.p][(size_t)a * N + j];
            v[6] = R.devn[si.p][j];
        } else {
            const int j0 = be.atom0;  // a real atom of the tile: neutral for min/max
            for (int a = 0; a < 3; ++a) v[a] = v[3 + a] = R.cnb[si.p][(size_t)a * N + j0];
            v[6] = 0.0;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                v[a] = fmin(v[a], __shfl_xor(v[a], off));
                v[3 + a] = fmax(v[3 + a], __shfl_xor(v[3 + a], off));
            }
            v[6] = fmax(v[6], __shfl_xor(v[6], off));
        }
        __syncthreads();
        if (lane == 0)
            for (int a = 0; a < 7; ++a) red[a][wave] = v[a];
        __syncthreads();
        if (threadIdx.x < 7) {
            const int a = threadIdx.x;
            double r = red[a][0];
            for (int w = 1; w < 4; ++w) r = (a < 3) ? fmin(r, red[a][w]) : fmax(r, red[a][w]);
            R.tbox[(size_t)(be.atom0 / kListTile) * 8 + a] = r;
        }
    }
}

// One wavefront per atom i: new reference r_ref_i = current bead centroid,
// relative positions of its beads, and its list.  Lane l scans atoms
// j = j0 + l; matches are compacted with a ballot, so entries come out in a
// fixed order (j chunk, image, lane) whatever the timing, the core entries
// (reference distance below r_cut, in range at almost every step) apart from
// the shell (list_push), so that the force loop's wavefronts meet the
// out-of-range pairs together.
template <typename T>
__device__ __forceinline__ void nlist_entry(RepDev& R, const BlockEntry be, const int p,
                                            int32_t* __restrict__ status, double* tx, double* ty,
                                            double* tz, double* td, double* dmax_s,
                                            uint8_t* skip, double box_scale)
{
    using T4 = typename Vec4<T>::type;
    const int N = R.N, P = R.P;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = be.atom0 + wave;
    const bool active = i < N;    // uniform over the wavefront
    const double* __restrict__ cx = R.cnb[p];
    const double* __restrict__ cy = R.cnb[p] + N;
    const double* __restrict__ cz = R.cnb[p] + 2 * (size_t)N;
    const double* __restrict__ devp = R.devn[p];
    double xi = 0.0, yi = 0.0, zi = 0.0, devi = 0.0;
    if (active) {
        xi = cx[i];
        yi = cy[i];
        zi = cz[i];
        devi = devp[i];
        if (lane < 3) R.rrefb[p][(size_t)lane * N + i] = R.cnb[p][(size_t)lane * N + i];
        if (lane == 0) R.devbb[p][i] = devi;
        T4* __restrict__ u = (T4*)R.ub[p] + (size_t)i * P;
        const T spb = bits_f(R.species[i], T());
        for (int b = lane; b < P; b += 64) {
            T4 v;
            v.x = (T)(R.pos[((size_t)b * 3 + 0) * N + i] - xi);
            v.y = (T)(R.pos[((size_t)b * 3 + 1) * N + i] - yi);
            v.z = (T)(R.pos[((size_t)b * 3 + 2) * N + i] - zi);
            v.w = spb;
            u[b] = v;
        }
    }
    // inside a step the positions carry a barostat's pending box factor
    const double Lx = R.box[0] * box_scale, Ly = R.box[1] * box_scale, Lz = R.box[2] * box_scale;
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
    // image range from the largest pair radius any atom of the block can have
    double dmax = 0.0;
    for (int j = threadIdx.x; j < N; j += 256) dmax = fmax(dmax, devp[j]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
    if (lane == 0) dmax_s[wave] = dmax;
    __syncthreads();
    dmax = fmax(fmax(dmax_s[0], dmax_s[1]), fmax(dmax_s[2], dmax_s[3]));
    const double Rmax = R.r_cs + devi + dmax;
    bool over = false;
    const int mx = image_range(Rmax, iLx, over), my = image_range(Rmax, iLy, over),
              mz = image_range(Rmax, iLz, over);
    if (over && active && lane == 0) atomicOr(status, kStatusRange);
    T4* __restrict__ ent = (T4*)R.nb_entries + (size_t)i * R.maxnb;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const double rc2 = R.r_cut * R.r_cut;
    int ncore = 0, nshell = 0;
    // tiles of 256 candidate atoms staged in LDS, shared by the 4 wavefronts;
    // a tile whose centroid bounds (widened by the spreads) are out of range
    // of all four atoms of the block is skipped, which leaves the entries and
    // their order unchanged.  The block first tests every tile (one thread
    // per tile) and keeps the verdicts in LDS.
    const int n_t = (N + kListTile - 1) / kListTile;
    const bool pre = n_t <= kMaxListTiles;
    if (pre) {
        // centroids and spreads of the block's atoms (block-uniform loads)
        double ax[4], ay[4], az[4], ad[4];
        bool av[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int a = be.atom0 + w;
            av[w] = a < N;
            const int ac = av[w] ? a : be.atom0;
            ax[w] = cx[ac];
            ay[w] = cy[ac];
            az[w] = cz[ac];
            ad[w] = devp[ac];
        }
        for (int t = threadIdx.x; t < n_t; t += blockDim.x) {
            const double* b = R.tbox + (size_t)t * 8;
            bool far = true;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const double Rt = R.r_cs + ad[w] + b[6];
                far = far && (!av[w] ||
                              box_dist2(ax[w], ay[w], az[w], b, Lx, Ly, Lz, iLx, iLy, iLz) >= Rt * Rt);
            }
            skip[t] = far ? 1 : 0;
        }
        __syncthreads();
    }
    for (int t0 = 0; t0 < N; t0 += kListTile) {
        if (pre) {
            if (skip[t0 / kListTile]) continue;  // the same verdict in every thread
            __syncthreads();
        } else {
            bool far = true;
            if (active) {
                const double* b = R.tbox + (size_t)(t0 / kListTile) * 8;
                const double Rt = R.r_cs + devi + b[6];
                far = box_dist2(xi, yi, zi, b, Lx, Ly, Lz, iLx, iLy, iLz) >= Rt * Rt;
            }
            if (__syncthreads_and(far)) continue;
        }
        const int jl = t0 + threadIdx.x;
        if (jl < N) {
            tx[threadIdx.x] = cx[jl];
            ty[threadIdx.x] = cy[jl];
            tz[threadIdx.x] = cz[jl];
            td[threadIdx.x] = devp[jl];
        }
        __syncthreads();
        if (!active) continue;
        const int tn = min(256, N - t0);
        for (int c0 = 0; c0 < tn; c0 += 64) {
            const int jj = c0 + lane;
            const int j = t0 + jj;
            const bool valid = jj < tn;
            // pair radius r_cut + skin + dev_i + dev_j
            const double Rij = R.r_cs + devi + (valid ? td[jj] : 0.0);
            const double R2 = Rij * Rij;
            double dx = 0.0, dy = 0.0, dz = 0.0;
            if (valid) {
                dx = xi - tx[jj];
                dy = yi - ty[jj];
                dz = zi - tz[jj];
                dx -= Lx * rint(dx * iLx);
                dy -= Ly * rint(dy * iLy);
                dz -= Lz * rint(dz * iLz);
            }
            for (int nx = -mx; nx <= mx; ++nx)
                for (int ny = -my; ny <= my; ++ny)
                    for (int nz = -mz; nz <= mz; ++nz) {
                        const double ex = dx + nx * Lx, ey = dy + ny * Ly, ez = dz + nz * Lz;
                        const double r2 = ex * ex + ey * ey + ez * ez;
                        const bool self = (j == i) && nx == 0 && ny == 0 && nz == 0;
                        const bool hit = valid && r2 < R2 && !self;
                        T4 v;
                        v.x = (T)ex;
                        v.y = (T)ey;
                        v.z = (T)ez;
                        v.w = bits_f(j, T());
                        list_push(ent, R.maxnb, hit, r2 < rc2, v, below, ncore, nshell);
                    }
        }
    }
    if (active && lane == 0)
        list_finish(R.nb_count, R.nb_core, i, R.maxnb, ncore, nshell, status);
}

// Grid-stride over the block table with at most 2048 workgroups, so the
// launch of a step that needs no rebuild costs one flag load per group.
// in_step: the build runs inside a step, after its update: the box takes
// the pending factor npt_sr of the positions, the list scale of this step's
// force pass becomes 1 (npt_S = 1 / npt_sr), and each rebuilt replica is
// marked for the barostat (list_built), which then resets the scale to 1.
// Between steps box and positions agree, and a rebuilt replica's list scale
// is 1 at once (its rebuild threshold with it).
template <typename T>
__global__ void __launch_bounds__(256) k_nlist(RepDev* __restrict__ reps,
                                               const BlockEntry* __restrict__ blocks,
                                               int n_entries, int32_t* __restrict__ status,
                                               const StepRef sync, int in_step)
{
    __shared__ double tx[256], ty[256], tz[256], td[256];
    __shared__ uint8_t skip[kMaxListTiles];
    __shared__ double dmax_s[4];
    const StepIdx si = step_index(sync);
    if (status[kAnyRebuild + si.f] == 0) return;  // nothing to do: one load, then exit
    for (int e = blockIdx.x; e < n_entries; e += gridDim.x) {
        const BlockEntry be = blocks[e];
        RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
        if (R.rflag[si.f] == 0) continue;  // uniform over the block
        nlist_entry<T>(R, be, si.p, status, tx, ty, tz, td, dmax_s, skip,
                       in_step ? R.npt_sr : 1.0);
        if (threadIdx.x == 0) {
            if (in_step) {
                // the entries are in this step's geometry: the force pass's
                // list scale npt_S npt_sr is 1; the barostat then sets it to
                // exactly 1 for the next step
                R.npt_S = 1.0 / R.npt_sr;
                R.list_built = 1;
            } else {  // between steps box and positions agree: the lists' scale is 1
                R.npt_S = 1.0;
                R.half_skin = R.half_skin0 - fmax(0.0, 1.0 - R.npt_sr) * 0.5 * R.r_cs;
            }
        }
        __syncthreads();
    }
}

}  // namespace

namespace {
// Flag every replica's list for a rebuild at the current step.
__global__ void k_mark_rebuild(const RepDev* __restrict__ reps, int n_rep,
                               int32_t* __restrict__ status, const StepRef sync)
{
    const int f = step_index(sync).f;
    for (int r = threadIdx.x; r < n_rep; r += blockDim.x) reps[r].rflag[f] = 1;
    if (threadIdx.x == 0) status[kAnyRebuild + f] = 1;
}
}  // namespace

void launch_mark_rebuild(hipStream_t st, const RepDev* reps, int n_rep, int32_t* status,
                         StepRef sync)
{
    launch(k_mark_rebuild, dim3(1), dim3(256), 0, st, reps, n_rep, status, sync);
}

void launch_nlist(hipStream_t st, bool fp64, const RepDev* reps, const BlockEntry* blocks,
                  int n_blocks, const BlockEntry* tiles, int n_tiles, int32_t* status,
                  bool centroids, StepRef sync, bool in_step)
{
    if (centroids)
        launch(k_centroids, dim3(n_blocks), dim3(64), 0, st, reps, blocks, sync);
    launch(k_tile_box, dim3(n_tiles < 256 ? n_tiles : 256), dim3(256), 0, st, reps, tiles,
           n_tiles, status, sync);
    // a list build is rare but long for large replicas: enough groups to
    // fill the chip; a step without a rebuild costs one flag load per group
    const int grid = n_blocks < 2048 ? n_blocks : 2048;
    RepDev* const wreps = const_cast<RepDev*>(reps);  // the builds mark their replicas
    const int ins = in_step ? 1 : 0;
    if (fp64)
        launch(k_nlist<double>, dim3(grid), dim3(256), 0, st, wreps, blocks, n_blocks, status,
               sync, ins);
    else
        launch(k_nlist<float>, dim3(grid), dim3(256), 0, st, wreps, blocks, n_blocks, status,
               sync, ins);
}

}  // namespace qtb
