// update.hip -- the velocity/position part of one step, fused:
//   B(dt/2) with the forces of the previous evaluation, transform to ring
//   normal modes, A(dt/2), O(dt), A(dt/2), transform back.
//
// B: v += dt f / (2 P m): the bead force -(1/P) grad V of eq. (4) with bead
//    mass m.  A: exact propagation of the free ring polymer of eq. (3)-(4);
//    in the orthonormal normal modes the springs decouple into oscillators
//    of frequency 2 omega_P sin(k pi / P) (k = 0 drifts).  O: the Langevin
//    friction and random force of eq. (8), v_k <- c1 v_k + sqrt((1-c1^2)/m)
//    zeta, c1 = exp(-gamma dt), applied to the normal modes with the
//    coloured noise whose spectrum is theta (eq. 7) or kappa_P (eq. 12), as
//    Sec. 2.3 prescribes for QTB-PIMD.
// Under a barostat the velocities take the pending scaling s_v1 before B
// and the normal-mode positions sqrt(s) before and after A-O-A (both 1
// otherwise).
//
// Bead-parallel: one thread per (atom, component, bead); the P x P
// transforms exchange values through LDS.
// The pair potential also needs the positions relative to the neighbour
// list reference (FP32 in FP32 mode): they are written here, and the
// largest component decides whether the list must be rebuilt.
#include "qtb_internal.h"
#include "ring_step.h"

namespace qtb {
namespace {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

template <typename T>
__device__ __forceinline__ T bits_as(int32_t b);
template <>
__device__ __forceinline__ float bits_as<float>(int32_t b) { return __int_as_float(b); }
template <>
__device__ __forceinline__ double bits_as<double>(int32_t b) { return __longlong_as_double((long long)b); }

// Loads through the global address space: the state pointers are generic,
// and generic loads make every wait drain all outstanding memory operations.
template <typename X>
__device__ __forceinline__ X gld(const X* p, size_t k)
{
    return ((const __attribute__((address_space(1))) X*)p)[k];
}

// A wavefront-uniform double (a replica's constant): kept in scalar
// registers, so a select between such values does not become a load
// indexed by a per-lane value.
__device__ __forceinline__ double uni(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One thread per (atom, Cartesian component, bead).  Consecutive lanes are
// consecutive atoms, so every state load and store of a wavefront is a
// contiguous run of the [P][dims][N] arrays; the P x P normal-mode
// transforms read the partner beads of the same (atom, component) from LDS.
// A block holds A = BlockEntry::group atoms (A dims P <= kUpdThreads).
// 384 threads (P up to 64 beads in 3D).  Smaller workgroups, several per
// compute unit, measured slower on gfx950 for the 4096-atom x 8-bead case.
constexpr int kUpdThreads = 384;

template <typename T, bool PAIR>
__global__ void __launch_bounds__(kUpdThreads) k_update(const RepDev* __restrict__ reps,
                                                        const BlockEntry* __restrict__ blocks,
                                                        const T* __restrict__ zeta_row,
                                                        int32_t* __restrict__ status,
                                                        const StepRef sync, int64_t zmod,
                                                        int64_t n_cols)
{
    using T4 = typename Vec4<T>::type;
    __shared__ double xr[kUpdThreads], xv[kUpdThreads];
    extern __shared__ double Cs[];  // [P][P], dynamic
    __shared__ double cen[kUpdThreads / 3][3];
    __shared__ int flags;
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const StepIdx si = step_index(sync);
    const int pin = si.p, pout = si.p ^ 1;        // this step's data, the next step's
    const int fnext = si.f == 2 ? 0 : si.f + 1;   // (step + 1) mod 3
    const int N = R.N, P = R.P, dims = R.dims;
    const int A = be.group;
    const int t = threadIdx.x;
    const int il = t % A, rest = t / A;
    const int s = rest % P, a = rest / P;        // bead (then mode), component
    const int i = be.atom0 + il;
    const bool active = (a < dims) && (i < N);
    const size_t idx = ((size_t)s * dims + a) * N + i;
    // Every global load of the thread is issued here, before the first LDS or
    // global store: the state pointers are generic, so the compiler keeps
    // loads behind any store that might alias them, and each store between
    // loads would add a round of memory latency.
    const int PP = P * P;
    const double nm0 = t < PP ? gld(R.nm, t) : 0.0;
    const double c1 = R.c1, sv1 = R.npt_sv1, sr = R.npt_sr;
    const double lsc = R.npt_S * R.npt_sr;  // the lists' scale for this step's force pass
    const double half_skin = R.half_skin;
    double r = 0.0, v = 0.0, f = 0.0, z = 0.0, ref3[3] = {0.0, 0.0, 0.0}, devb = 0.0;
    double kick = 0.0, sig = 0.0, cw = 0.0, sw = 0.0, ws = 0.0;
    int sp = 0;
    if (active) {
        sp = gld(R.species, i);
        r = gld(R.pos, idx);
        v = gld(R.vel, idx);
        f = (double)gld((const T*)R.force, idx);
        const T* zr = zeta_row;
        if (zmod > 0) {  // block noise: the row of this step in the [zmod] ring
            int64_t m = ((sync.clk ? *sync.clk : 0) + sync.off) % zmod;
            if (m < 0) m += zmod;
            zr += m * n_cols;
        }
        z = (double)gld(zr, (size_t)(R.dof_off + ((int64_t)dims * i + a) * P + s));
        if (PAIR && a == 0) {
            for (int a2 = 0; a2 < 3; ++a2) ref3[a2] = gld(R.rrefb[pin], (size_t)a2 * N + i);
            devb = gld(R.devbb[pin], i);
        }
        // this thread holds mode k = s after the transform
        cw = gld(R.ring, s);
        sw = gld(R.ring, P + s);
        ws = gld(R.ring, 2 * P + s);
        kick = uni(R.kick[0]);
        sig = uni(R.sigma[0]);
#pragma unroll
        for (int q = 1; q < kMaxSpecies; ++q) {
            kick = (sp == q) ? uni(R.kick[q]) : kick;
            sig = (sp == q) ? uni(R.sigma[q]) : sig;
        }
    }
    if (PAIR && active && a == 0 && s == 0) {  // the references carry over to the next step
        for (int a2 = 0; a2 < 3; ++a2) R.rrefb[pout][(size_t)a2 * N + i] = ref3[a2];
        R.devbb[pout][i] = devb;
    }
    if (t < PP) Cs[t] = nm0;
    for (int x = t + (int)blockDim.x; x < PP; x += blockDim.x) Cs[x] = gld(R.nm, x);
    if (t == 0) flags = 0;
    if (active) v = half_kick(v * sv1, kick, f);  // barostat's pending velocity scaling
    xr[t] = r;
    xv[t] = v;
    __syncthreads();
    // partner of bead b of this (atom, component) sits at (a P + b) A + il
    const int base = a * P * A + il;
    double q = 0.0, pm = 0.0;
    if (active) {
        for (int b = 0; b < P; ++b) {
            const double c = Cs[b * P + s];
            q = nm_acc(q, c, xr[base + b * A]);
            pm = nm_acc(pm, c, xv[base + b * A]);
        }
        // this thread now holds mode k = s (its noise value z); the
        // barostat's pending length scaling, half before and half after
        const double rh = sqrt(sr);
        q *= rh;
        mode_aoa(q, pm, cw, sw, ws, c1, sig, z);
        q *= rh;
    }
    __syncthreads();
    xr[t] = q;
    xv[t] = pm;
    __syncthreads();
    if (active) {
        double rn = 0.0, vn = 0.0;
        for (int k = 0; k < P; ++k) {
            const double c = Cs[s * P + k];
            rn = nm_acc(rn, c, xr[base + k * A]);
            vn = nm_acc(vn, c, xv[base + k * A]);
        }
        r = rn;
        v = vn;
        R.pos[idx] = r;
        R.vel[idx] = v;
        if (!(__builtin_isfinite(r) && __builtin_isfinite(v))) atomicOr(&flags, kStatusNonfinite);
    }
    if (PAIR) {
        // centroid per (atom, component); relative positions, bead spread and
        // the rebuild test per (atom, bead)
        __syncthreads();
        xr[t] = r;
        __syncthreads();
        if (active && s == 0) {
            double c = 0.0;
            for (int b = 0; b < P; ++b) c += xr[base + b * A];
            c /= P;
            R.cnb[pout][(size_t)a * N + i] = c;
            cen[il][a] = c;
        }
        __syncthreads();
        // lsc: the lists' scale for this step's force pass, with the box
        // factor this update applies (committed at the end of the step)
        if (active && a == 0) {
            double u3[3], u2 = 0.0, d2 = 0.0;
            for (int a2 = 0; a2 < 3; ++a2) {
                const double x = xr[(a2 * P + s) * A + il];
                u3[a2] = __builtin_fma(-lsc, ref3[a2], x);  // lsc = 1: x - ref
                const double dc = x - cen[il][a2];
                u2 = nm_acc(u2, u3[a2], u3[a2]);
                d2 = nm_acc(d2, dc, dc);
            }
            T4 val;
            val.x = (T)u3[0];
            val.y = (T)u3[1];
            val.z = (T)u3[2];
            val.w = bits_as<T>(sp);
            ((T4*)R.ub[pout])[(size_t)i * P + s] = val;
            xv[t] = d2;
            // a compressed box (npt_S < 1) shrinks the bead spreads with it
            const double lim = __builtin_fma(devb, fmin(1.0, lsc), half_skin);
            if (!(u2 <= lim * lim) || !(lim > 0.0)) atomicOr(&flags, 8);
        }
        __syncthreads();
        if (t < A && be.atom0 + t < N) {
            double d2 = 0.0;
            for (int b = 0; b < P; ++b) d2 = fmax(d2, xv[b * A + t]);
            R.devn[pout][be.atom0 + t] = sqrt(d2);
        }
    }
    __syncthreads();
    if (t == 0 && flags) {
        if (flags & 8) {
            atomicOr(R.rflag + fnext, 1);
            atomicOr(status + kAnyRebuild + fnext, 1);
        }
        if (flags & kStatusNonfinite) atomicOr(status, kStatusNonfinite);
    }
}

}  // namespace

// Block tables hold A atoms per entry (in .group), A dims P <= kUpdThreads.
int update_threads(int) { return kUpdThreads; }

int update_block_atoms(int dims, int P, int threads)
{
    int A = threads / (dims * P);
    return A < 1 ? 1 : A;
}

void launch_update(hipStream_t st, bool fp64, bool pair, int P, int threads,
                   const RepDev* reps, const BlockEntry* blocks, int n_blocks,
                   const void* zeta_row, int32_t* status, StepRef sync, int64_t zmod,
                   int64_t n_cols)
{
    const dim3 g(n_blocks), b(threads);
    const uint32_t lds = 8u * (uint32_t)P * (uint32_t)P;  // the largest P of the launch
    if (fp64) {
        if (pair) launch((k_update<double, true>), g, b, lds, st, reps, blocks, (const double*)zeta_row, status, sync, zmod, n_cols);
        else launch((k_update<double, false>), g, b, lds, st, reps, blocks, (const double*)zeta_row, status, sync, zmod, n_cols);
    } else {
        if (pair) launch((k_update<float, true>), g, b, lds, st, reps, blocks, (const float*)zeta_row, status, sync, zmod, n_cols);
        else launch((k_update<float, false>), g, b, lds, st, reps, blocks, (const float*)zeta_row, status, sync, zmod, n_cols);
    }
}

}  // namespace qtb
