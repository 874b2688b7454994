// forces.hip -- forces of every bead, the closing B(dt/2) kick, and the
// energy estimators.
//
// Each bead of the ring polymer feels the physical potential V (eq. 3-4;
// the 1/P factor is applied with the kick).  The pair potential is a
// Buckingham term in shifted-force form plus damped shifted force Coulomb
// (constants folded into PairParam; see qtb_internal.h).
//
// Mapping on CDNA4: W 64-wide wavefronts per atom i.  Lane l takes bead
// s = group*G + l % G and neighbour chunk l / G (+ 64/G per extra wavefront);
// the G beads of an atom share one neighbour list (built from bead
// centroids, entries hold the reference displacement, so a pair distance is
// d_ij + u_i - u_j with small u in the working precision).  Per-bead sums are
// reduced across chunks with wavefront shuffles and across the W wavefronts
// in LDS (FP64 accumulators): no atomics, no write conflicts.  The first
// lanes of the atom finish it: store the force, apply the kick, and on
// sampling steps form the eq. (5) terms.
#include "force_epilogue.h"
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

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
template <typename T> struct NV;
template <> struct NV<float> { using v4 = f4v; };
template <> struct NV<double> { using v4 = d4v; };
// Workspace pointers live in RepDev (generic address space); casting them to
// the global address space lets the compiler emit global (not flat) loads.
template <typename X>
using gptr = const __attribute__((address_space(1))) X*;

__device__ __forceinline__ int32_t vbits(f4v x) { return __float_as_int(x.w); }
__device__ __forceinline__ int32_t vbits(d4v x) { return (int32_t)__double_as_longlong(x.w); }

// NS: species count rounded up to 2 or 4 (parameters of the centre atom's
// row are kept in registers and picked per neighbour with selects).
// FAST (FP32 only): hardware rsq / exp2 and the fitted erfcx polynomial.
template <typename T, int G, int NS, bool FAST, int DEG>
__global__ void __launch_bounds__(256) k_force_pair(const RepDev* __restrict__ reps,
                                                    const BlockEntry* __restrict__ blocks,
                                                    const PairTable<T> tab, int32_t flags,
                                                    double* __restrict__ partials,
                                                    int32_t* __restrict__ rebuild_clear, int n_rep,
                                                    int32_t* __restrict__ rebuild_any, int W)
{
    using V4 = typename NV<T>::v4;
    constexpr int NCH = 64 / G;   // neighbour chunks per wavefront
    // W wavefronts per atom (1, 2 or 4), 4 / W atoms per block
    __shared__ double part[4][G][4];
    __shared__ double red[4][kNobs];
    const BlockEntry be = blocks[blockIdx.x];
    const int rep = __builtin_amdgcn_readfirstlane(be.rep);
    const RepDev& R = reps[rep];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = wave / W, wsub = wave % W;
    const int bl = lane % G, ch = lane / G + wsub * NCH;
    const int i = be.atom0 + slot;
    const int N = R.N, P = R.P;
    const bool active = i < N;
    const int s = be.group * G + bl;
    const bool want_e = (flags & (kSample | kEvaluate)) != 0;

    if (blockIdx.x == 0 && rebuild_clear) {
        for (int r = threadIdx.x; r < n_rep; r += blockDim.x) rebuild_clear[r] = 0;
        if (threadIdx.x == 0) rebuild_any[0] = 0;
    }

    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    int spi = 0;
    if (active) {
        // u is atom-major [N][P]: the G beads of a neighbour share cache lines
        gptr<V4> u = (gptr<V4>)R.u + s;
        const V4 ui = u[(size_t)i * P];
        spi = vbits(ui);
        const int row = __builtin_amdgcn_readfirstlane(spi) * kMaxSpecies;
        T pArho[NS], pirho[NS], pC6[NS], pkqq[NS], pF0[NS], pA[NS], pC[NS], pE0[NS];
#pragma unroll
        for (int b = 0; b < NS; ++b) {
            const PairParam<T>& q = tab.p[row + b];
            pArho[b] = q.Arho;
            pirho[b] = FAST ? q.irho2 : q.irho;
            pC6[b] = q.C6;
            pkqq[b] = q.kqq;
            pF0[b] = q.F0;
            pA[b] = q.A;
            pC[b] = q.C;
            pE0[b] = q.E0;
        }
        // keep the neighbour-species parameters in VGPRs for the whole loop
        // (selects on gfx950 take at most one SGPR operand)
#pragma unroll
        for (int b = 0; b < NS; ++b) {
            asm volatile("" : "+v"(pArho[b]), "+v"(pirho[b]), "+v"(pC6[b]), "+v"(pkqq[b]),
                         "+v"(pF0[b]));
        }
        T ex[DEG + 1];
#pragma unroll
        for (int k = 0; k <= DEG; ++k) ex[k] = tab.ex[k];
        const T rc2 = tab.rc2, a2l = tab.a2l, s_mul = tab.s_mul, alpha = tab.alpha, g = tab.g;
        gptr<V4> ent = (gptr<V4>)R.nb_entries + (size_t)i * R.maxnb;
        const int cnt = R.nb_count[i];
        const int ST = NCH * W;
        // three-stage pipeline: entry q+2*ST and the neighbour of entry q+ST
        // are loading while the pair of entry q is evaluated
        int q = ch;
        V4 E0 = ent[q < cnt ? q : 0];
        V4 E1 = ent[q + ST < cnt ? q + ST : 0];
        V4 U0 = u[(size_t)vbits(E0) * P];
        while (q < cnt) {
            const int q2 = q + 2 * ST;
            const V4 E2 = ent[q2 < cnt ? q2 : 0];
            const V4 U1 = u[(size_t)vbits(E1) * P];
            const T dx = (E0.x + ui.x) - U0.x;
            const T dy = (E0.y + ui.y) - U0.y;
            const T dz = (E0.z + ui.z) - U0.z;
            const T r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                const int spj = vbits(U0);
                T Arho = pArho[0], irho = pirho[0], C6 = pC6[0], kqq = pkqq[0], F0 = pF0[0];
#pragma unroll
                for (int b = 1; b < NS; ++b) {
                    const bool m = spj == b;
                    Arho = m ? pArho[b] : Arho;
                    irho = m ? pirho[b] : irho;
                    C6 = m ? pC6[b] : C6;
                    kqq = m ? pkqq[b] : kqq;
                    F0 = m ? pF0[b] : F0;
                }
                T rinv, r, e1, e2, ec;
                if constexpr (FAST) {
                    rinv = __builtin_amdgcn_rsqf(r2);
                    r = r2 * rinv;
                    e1 = __builtin_amdgcn_exp2f(-r * irho);
                    e2 = __builtin_amdgcn_exp2f(-r2 * a2l);
                    const T sx = fmaf(r, s_mul, -1.0f);
                    T pe = ex[DEG];
#pragma unroll
                    for (int k = DEG - 1; k >= 0; --k) pe = fmaf(pe, sx, ex[k]);
                    ec = e2 * pe;
                } else {
                    rinv = t_rsqrt(r2);
                    r = r2 * rinv;
                    e1 = t_exp(-r * irho);
                    const T x = alpha * r;
                    e2 = t_exp(-x * x);
                    ec = t_erfc(x);
                }
                const T rinv2 = rinv * rinv;
                const T rinv6 = rinv2 * rinv2 * rinv2;
                const T F = Arho * e1 - C6 * rinv6 * rinv + kqq * (ec * rinv2 + g * e2 * rinv) + F0;
                const T fr = F * rinv;
                fx += (double)(fr * dx);
                fy += (double)(fr * dy);
                fz += (double)(fr * dz);
                if (want_e) {
                    T A = pA[0], C = pC[0], E0c = pE0[0];
#pragma unroll
                    for (int b = 1; b < NS; ++b) {
                        const bool m = spj == b;
                        A = m ? pA[b] : A;
                        C = m ? pC[b] : C;
                        E0c = m ? pE0[b] : E0c;
                    }
                    e += (double)(A * e1 - C * rinv6 + kqq * ec * rinv - F0 * r + E0c);
                }
            }
            E0 = E1;
            E1 = E2;
            U0 = U1;
            q += ST;
        }
    }
    // lanes with the same bead: reduce across chunks (shuffles), then across
    // the W wavefronts of the atom (LDS)
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
        if (want_e) e += __shfl_xor(e, off);
    }
    if (W > 1) {
        if (lane < G) {
            part[wave][lane][0] = fx;
            part[wave][lane][1] = fy;
            part[wave][lane][2] = fz;
            part[wave][lane][3] = e;
        }
        __syncthreads();
        if (wsub == 0 && lane < G) {
            for (int w = 1; w < W; ++w) {
                fx += part[wave + w][lane][0];
                fy += part[wave + w][lane][1];
                fz += part[wave + w][lane][2];
                e += part[wave + w][lane][3];
            }
        }
    }
    double ob[kNobs] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active && wsub == 0 && lane < G && s < P) {
        const double f[3] = {fx, fy, fz};
        force_epilogue<T>(R, i, s, spi, f, 0.5 * e, flags, ob);
    }
    if (flags & (kSample | kCompare)) {
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

template <typename T, int NS, bool FAST, int DEG>
void launch_pair_G(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int32_t* rebuild_clear, int n_rep, int32_t* rebuild_any, int W)
{
    const dim3 g(n_blocks), b(256);
    switch (G) {
    case 1: launch((k_force_pair<T, 1, NS, FAST, DEG>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep, rebuild_any, W); break;
    case 2: launch((k_force_pair<T, 2, NS, FAST, DEG>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep, rebuild_any, W); break;
    case 4: launch((k_force_pair<T, 4, NS, FAST, DEG>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep, rebuild_any, W); break;
    case 8: launch((k_force_pair<T, 8, NS, FAST, DEG>), g, b, 0, st, reps, blocks, tab, flags, partials, rebuild_clear, n_rep, rebuild_any, W); break;
    default: break;
    }
}

template <typename T, bool FAST, int DEG>
void launch_pair_T(hipStream_t st, int G, const RepDev* reps, const BlockEntry* blocks,
                   int n_blocks, const PairTable<T>& tab, int32_t flags, double* partials,
                   int32_t* rebuild_clear, int n_rep, int32_t* rebuild_any, int W)
{
    if (tab.n_species <= 2)
        launch_pair_G<T, 2, FAST, DEG>(st, G, reps, blocks, n_blocks, tab, flags, partials, rebuild_clear, n_rep, rebuild_any, W);
    else
        launch_pair_G<T, 4, FAST, DEG>(st, G, reps, blocks, n_blocks, tab, flags, partials, rebuild_clear, n_rep, rebuild_any, W);
}

}  // namespace

void launch_forces_pair(hipStream_t st, bool fp64, int G, int W, const RepDev* reps,
                        const BlockEntry* blocks, int n_blocks, const void* table, int32_t flags,
                        double* partials, int32_t* rebuild_clear, int n_rep,
                        int32_t* rebuild_any)
{
    if (fp64) {
        launch_pair_T<double, false, 1>(st, G, reps, blocks, n_blocks,
                                     *(const PairTable<double>*)table, flags, partials,
                                     rebuild_clear, n_rep, rebuild_any, W);
    } else {
        const PairTable<float>& t = *(const PairTable<float>*)table;
        if (t.ex_deg == 10)
            launch_pair_T<float, true, 10>(st, G, reps, blocks, n_blocks, t, flags, partials,
                                           rebuild_clear, n_rep, rebuild_any, W);
        else if (t.ex_deg == kErfcxMaxDeg)
            launch_pair_T<float, true, kErfcxMaxDeg>(st, G, reps, blocks, n_blocks, t, flags,
                                                     partials, rebuild_clear, n_rep, rebuild_any, W);
        else
            launch_pair_T<float, false, 1>(st, G, reps, blocks, n_blocks, t, flags, partials,
                                           rebuild_clear, n_rep, rebuild_any, W);
    }
}

void launch_forces_harmonic(hipStream_t st, bool fp64, const RepDev* reps,
                            const BlockEntry* blocks, int n_blocks, int32_t flags,
                            double* partials)
{
    if (fp64)
        launch(k_force_harmonic<double>, dim3(n_blocks), dim3(256), 0, st, reps,
                           blocks, flags, partials);
    else
        launch(k_force_harmonic<float>, dim3(n_blocks), dim3(256), 0, st, reps,
                           blocks, flags, partials);
}

void launch_obs_reduce(hipStream_t st, const RepDev* reps, int n_rep, const double* partials,
                       double* acc, int32_t* counts)
{
    launch(k_obs_reduce, dim3((n_rep + 63) / 64), dim3(64), 0, st, reps, n_rep,
                       partials, acc, counts);
}

void launch_fill(hipStream_t st, void* p, int64_t n_words, int32_t value)
{
    if (n_words <= 0) return;
    int64_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    launch(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, (int32_t*)p, n_words,
                       value);
}

}  // namespace qtb
