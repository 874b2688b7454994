// forces.hip -- forces of every bead, the closing B(dt/2) kick, and the
// energy estimators.
//
// Each bead of the ring polymer feels the physical potential V (eq. 3-4;
// the 1/P factor is applied with the kick).  The pair potential is a
// Buckingham term in shifted-force form plus damped shifted force Coulomb
// (constants folded into PairParam; see qtb_internal.h).
//
// Mapping on CDNA4: one 64-wide wavefront per atom i.  Lane l takes bead
// s = group*G + l % G and neighbour chunk l / G; the G beads of an atom share
// one neighbour list (built from bead centroids, entries hold the reference
// displacement, so a pair distance is d_ij + u_i - u_j with small u in the
// working precision).  Per-bead sums are reduced across chunks with
// wavefront shuffles (FP64 accumulators), so no atomics and no write
// conflicts; lanes of chunk 0 finish the atom: store the force, apply the
// kick, and on sampling steps form the eq. (5) terms.
#include "qtb_internal.h"

namespace qtb {
namespace {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

__device__ __forceinline__ int32_t as_bits(float x) { return __float_as_int(x); }
__device__ __forceinline__ int32_t as_bits(double x) { return (int32_t)__double_as_longlong(x); }

__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_erfc(float x) { return erfcf(x); }
__device__ __forceinline__ double t_erfc(double x) { return erfc(x); }
__device__ __forceinline__ float t_rsqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double t_rsqrt(double x) { return 1.0 / sqrt(x); }

// Sum a value over all 64 lanes (result in every lane).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off);
    return x;
}

template <typename T, int G>
__global__ void __launch_bounds__(256) k_force_pair(const RepDev* __restrict__ reps,
                                                    const BlockEntry* __restrict__ blocks,
                                                    const PairTable<T> tab, int32_t flags,
                                                    double* __restrict__ partials,
                                                    int32_t* __restrict__ rebuild_clear, int n_rep)
{
    using T4 = typename Vec4<T>::type;
    constexpr int NCH = 64 / G;
    __shared__ double red[4][kNobs];
    const BlockEntry be = blocks[blockIdx.x];
    const int rep = __builtin_amdgcn_readfirstlane(be.rep);
    const RepDev& R = reps[rep];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bl = lane % G, ch = lane / G;
    const int i = be.atom0 + wave;
    const int N = R.N, P = R.P;
    const bool active = i < N;
    const int s = be.group * G + bl;
    const bool want_e = (flags & (kSample | kEvaluate)) != 0;

    if (blockIdx.x == 0)
        for (int r = threadIdx.x; r < n_rep; r += blockDim.x) rebuild_clear[r] = 0;

    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    int spi = 0;
    if (active) {
        const T4* __restrict__ u = (const T4*)R.u + (size_t)s * N;
        const T4 ui = u[i];
        spi = as_bits(ui.w);
        const int row = __builtin_amdgcn_readfirstlane(spi) * kMaxSpecies;
        const T4* __restrict__ ent = (const T4*)R.nb_entries + (size_t)i * R.maxnb;
        const int cnt = R.nb_count[i];
        const T rc2 = tab.rc2, alpha = tab.alpha, g = tab.g;
        const int ns = tab.n_species;
        for (int q = ch; q < cnt; q += NCH) {
            const T4 E = ent[q];
            const int j = as_bits(E.w);
            const T4 uj = u[j];
            const T dx = (E.x + ui.x) - uj.x;
            const T dy = (E.y + ui.y) - uj.y;
            const T dz = (E.z + ui.z) - uj.z;
            const T r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                const int spj = as_bits(uj.w);
                PairParam<T> pp = tab.p[row];
#pragma unroll
                for (int b = 1; b < kMaxSpecies; ++b)
                    if (b < ns && spj == b) pp = tab.p[row + b];
                const T rinv = t_rsqrt(r2);
                const T r = r2 * rinv;
                const T e1 = t_exp(-r * pp.irho);
                const T x = alpha * r;
                const T e2 = t_exp(-x * x);
                const T ec = t_erfc(x);
                const T rinv2 = rinv * rinv;
                const T rinv6 = rinv2 * rinv2 * rinv2;
                const T F = pp.Arho * e1 - pp.C6 * rinv6 * rinv +
                            pp.kqq * (ec * rinv2 + g * e2 * rinv) + pp.F0;
                const T fr = F * rinv;
                fx += (double)(fr * dx);
                fy += (double)(fr * dy);
                fz += (double)(fr * dz);
                if (want_e)
                    e += (double)(pp.A * e1 - pp.C * rinv6 + pp.kqq * ec * rinv - pp.F0 * r + pp.E0);
            }
        }
    }
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        if (want_e) e += __shfl_xor(e, off);
    }
    // lanes 0..G-1 now hold the totals of bead s
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active && ch == 0 && s < P) {
        const double f[3] = {fx, fy, fz};
        T* __restrict__ force = (T*)R.force;
        const double kick = R.kick[spi];
        double vn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t idx = ((size_t)s * 3 + a) * N + i;
            force[idx] = (T)f[a];
            double v = R.vel[idx];
            if (flags & kKick) {
                v += kick * f[a];
                R.vel[idx] = v;
            }
            vn[a] = v;
        }
        if (flags & kEvaluate) R.eatom[(size_t)s * N + i] = 0.5 * e;
        if (flags & kSample) {
            const double m = R.mmu[spi];
            const int sn = (s + 1 == P) ? 0 : s + 1;
            double ke = 0.0, spr = 0.0, vir = 0.0, x2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t idx = ((size_t)s * 3 + a) * N + i;
                const double ra = R.pos[idx];
                double c = 0.0;
                for (int b = 0; b < P; ++b) c += R.pos[((size_t)b * 3 + a) * N + i];
                c /= P;
                const double dn = ra - R.pos[((size_t)sn * 3 + a) * N + i];
                const double d0 = ra - R.r0[idx];
                ke += vn[a] * vn[a];
                spr += dn * dn;
                vir += (ra - c) * f[a];
                x2 += d0 * d0;
            }
            ob[0] = 0.5 * m * ke;
            ob[1] = 0.5 * e / P;
            ob[2] = (P > 1) ? 0.5 * m * R.omega_P * R.omega_P * spr : 0.0;
            ob[3] = vir;
            ob[4] = x2;
        }
    }
    if (flags & kSample) {
#pragma unroll
        for (int q = 0; q < kNobs; ++q) {
            const double t = wave_sum(ob[q]);
            if (lane == 0) red[wave][q] = t;
        }
        __syncthreads();
        if (threadIdx.x < kNobs) {
            const double t = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                             red[3][threadIdx.x];
            partials[(size_t)blockIdx.x * kNobs + threadIdx.x] = t;
        }
    }
}

// Independent oscillators: V = sum_i 1/2 m omega_i^2 |x_i|^2 per bead.
template <typename T>
__global__ void __launch_bounds__(256) k_force_harmonic(const RepDev* __restrict__ reps,
                                                        const BlockEntry* __restrict__ blocks,
                                                        int32_t flags, double* __restrict__ partials)
{
    __shared__ double red[4][kNobs];
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int i = be.atom0 + threadIdx.x;
    const int N = R.N, P = R.P, dims = R.dims;
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < N) {
        const int sp = R.species[i];
        const double m = R.mmu[sp], w = R.homega[i], kick = R.kick[sp];
        const double k = m * w * w;
        double ke = 0.0, U = 0.0, spr = 0.0, vir = 0.0, x2 = 0.0;
        for (int a = 0; a < dims; ++a) {
            double c = 0.0;
            for (int s = 0; s < P; ++s) c += R.pos[((size_t)s * dims + a) * N + i];
            c /= P;
            for (int s = 0; s < P; ++s) {
                const size_t idx = ((size_t)s * dims + a) * N + i;
                const double x = R.pos[idx];
                const double f = -k * x;
                ((T*)R.force)[idx] = (T)f;
                double v = R.vel[idx];
                if (flags & kKick) {
                    v += kick * f;
                    R.vel[idx] = v;
                }
                if (flags & (kSample | kEvaluate)) {
                    const int sn = (s + 1 == P) ? 0 : s + 1;
                    const double dn = x - R.pos[((size_t)sn * dims + a) * N + i];
                    const double d0 = x - R.r0[idx];
                    ke += 0.5 * m * v * v;
                    U += 0.5 * k * x * x;
                    spr += dn * dn;
                    vir += (x - c) * f;
                    x2 += d0 * d0;
                    if (flags & kEvaluate) {
                        double* ea = R.eatom + (size_t)s * N + i;
                        *ea = (a == 0 ? 0.0 : *ea) + 0.5 * k * x * x;
                    }
                }
            }
        }
        ob[0] = ke;
        ob[1] = U / P;
        ob[2] = (P > 1) ? 0.5 * m * R.omega_P * R.omega_P * spr : 0.0;
        ob[3] = vir;
        ob[4] = x2;
    }
    if (flags & kSample) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < kNobs; ++q) {
            const double t = wave_sum(ob[q]);
            if (lane == 0) red[wave][q] = t;
        }
        __syncthreads();
        if (threadIdx.x < kNobs) {
            const double t = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                             red[3][threadIdx.x];
            partials[(size_t)blockIdx.x * kNobs + threadIdx.x] = t;
        }
    }
}

// Per replica, in block order (deterministic): acc += sum of block partials.
__global__ void k_obs_reduce(const RepDev* __restrict__ reps, int n_rep,
                             const double* __restrict__ partials, double* __restrict__ acc,
                             int32_t* __restrict__ counts)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    const RepDev& R = reps[r];
    double t[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = R.obs_block0; b < R.obs_block0 + R.obs_nblocks; ++b)
        for (int q = 0; q < kNobs; ++q) t[q] += partials[(size_t)b * kNobs + q];
    for (int q = 0; q < kNobs; ++q) acc[(size_t)r * kNobs + q] += t[q];
    counts[r] += 1;
}

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n;
         id += (int64_t)gridDim.x * blockDim.x)
        p[id] = v;
}

template <typename T>
void launch_pair_T(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int32_t* rebuild_clear, int n_rep)
{
    const dim3 g(n_blocks), b(256);
    switch (G) {
    case 1: hipLaunchKernelGGL((k_force_pair<T, 1>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep); break;
    case 2: hipLaunchKernelGGL((k_force_pair<T, 2>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep); break;
    case 4: hipLaunchKernelGGL((k_force_pair<T, 4>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep); break;
    case 8: hipLaunchKernelGGL((k_force_pair<T, 8>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep); break;
    default: break;
    }
}

}  // namespace

void launch_forces_pair(hipStream_t st, bool fp64, int G, const RepDev* reps,
                        const BlockEntry* blocks, int n_blocks, const void* table, int32_t flags,
                        double* partials, int32_t* rebuild_clear, int n_rep)
{
    if (fp64)
        launch_pair_T<double>(st, G, reps, blocks, n_blocks, *(const PairTable<double>*)table,
                              flags, partials, rebuild_clear, n_rep);
    else
        launch_pair_T<float>(st, G, reps, blocks, n_blocks, *(const PairTable<float>*)table,
                             flags, partials, rebuild_clear, n_rep);
}

void launch_forces_harmonic(hipStream_t st, bool fp64, const RepDev* reps,
                            const BlockEntry* blocks, int n_blocks, int32_t flags,
                            double* partials)
{
    if (fp64)
        hipLaunchKernelGGL(k_force_harmonic<double>, dim3(n_blocks), dim3(256), 0, st, reps,
                           blocks, flags, partials);
    else
        hipLaunchKernelGGL(k_force_harmonic<float>, dim3(n_blocks), dim3(256), 0, st, reps,
                           blocks, flags, partials);
}

void launch_obs_reduce(hipStream_t st, const RepDev* reps, int n_rep, const double* partials,
                       double* acc, int32_t* counts)
{
    hipLaunchKernelGGL(k_obs_reduce, dim3((n_rep + 63) / 64), dim3(64), 0, st, reps, n_rep,
                       partials, acc, counts);
}

void launch_fill(hipStream_t st, void* p, int64_t n_words, int32_t value)
{
    if (n_words <= 0) return;
    int64_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, (int32_t*)p, n_words,
                       value);
}

}  // namespace qtb
