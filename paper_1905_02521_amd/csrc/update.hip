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
//
// One thread owns one atom with all its beads in registers (P <= 8), so the
// P x P transforms never leave the register file; larger P uses LDS.
// The pair potential also needs the positions relative to the neighbour
// list reference (FP32 in FP32 mode): they are written here, and the
// largest component decides whether the list must be rebuilt.
#include "qtb_internal.h"

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

template <int P, typename T, bool PAIR>
__global__ void __launch_bounds__(256) k_update(const RepDev* __restrict__ reps,
                                                const BlockEntry* __restrict__ blocks,
                                                const T* __restrict__ zeta_row,
                                                int32_t* __restrict__ status)
{
    using T4 = typename Vec4<T>::type;
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int i = be.atom0 + threadIdx.x;
    const int N = R.N, dims = R.dims;
    if (i >= N) return;
    const int sp = R.species[i];
    const double kick = R.kick[sp], sig = R.sigma[sp], c1 = R.c1;
    const T* __restrict__ force = (const T*)R.force;
    const T* __restrict__ z = zeta_row + R.dof_off;
    const double* __restrict__ C = R.nm;
    const double* __restrict__ ring = R.ring;
    double umax = 0.0;
    T uc[3][P];
    bool finite = true;
    for (int a = 0; a < dims; ++a) {
        double r[P], v[P], q[P], p[P];
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const size_t idx = ((size_t)s * dims + a) * N + i;
            r[s] = R.pos[idx];
            v[s] = R.vel[idx] + kick * (double)force[idx];
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double qa = 0.0, pa = 0.0;
#pragma unroll
            for (int s = 0; s < P; ++s) {
                qa += C[s * P + k] * r[s];
                pa += C[s * P + k] * v[s];
            }
            q[k] = qa;
            p[k] = pa;
        }
        const int64_t dof0 = ((int64_t)dims * i + a) * P;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double cw = ring[k], sw = ring[P + k], ws = ring[2 * P + k];
            double q1 = cw * q[k] + sw * p[k];
            double p1 = ws * q[k] + cw * p[k];
            p1 = c1 * p1 + sig * (double)z[dof0 + k];
            q[k] = cw * q1 + sw * p1;
            p[k] = ws * q1 + cw * p1;
        }
#pragma unroll
        for (int s = 0; s < P; ++s) {
            double ra = 0.0, va = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                ra += C[s * P + k] * q[k];
                va += C[s * P + k] * p[k];
            }
            const size_t idx = ((size_t)s * dims + a) * N + i;
            R.pos[idx] = ra;
            R.vel[idx] = va;
            finite = finite && __builtin_isfinite(ra) && __builtin_isfinite(va);
            if (PAIR) {
                const double du = ra - R.rref[(size_t)a * N + i];
                uc[a][s] = (T)du;
                umax = fmax(umax, fabs(du));
            }
        }
    }
    if (PAIR) {
        T4* __restrict__ u = (T4*)R.u;
        const T spb = bits_as<T>(sp);
#pragma unroll
        for (int s = 0; s < P; ++s) {
            T4 val;
            val.x = uc[0][s];
            val.y = uc[1][s];
            val.z = uc[2][s];
            val.w = spb;
            u[(size_t)s * N + i] = val;
        }
        if (!(umax <= R.u_lim)) atomicOr(R.rebuild, 1);
    }
    if (!finite) atomicOr(status, kStatusNonfinite);
}

// Any P: per-thread bead arrays in LDS (64 threads per block).
template <typename T, bool PAIR>
__global__ void __launch_bounds__(64) k_update_lds(const RepDev* __restrict__ reps,
                                                   const BlockEntry* __restrict__ blocks,
                                                   const T* __restrict__ zeta_row,
                                                   int32_t* __restrict__ status)
{
    using T4 = typename Vec4<T>::type;
    extern __shared__ double shq[];
    const BlockEntry be = blocks[blockIdx.x];
    const RepDev& R = reps[__builtin_amdgcn_readfirstlane(be.rep)];
    const int P = R.P;
    double* r = shq + (size_t)threadIdx.x * 4 * P;
    double* v = r + P;
    double* q = v + P;
    double* p = q + P;
    const int i = be.atom0 + threadIdx.x;
    const int N = R.N, dims = R.dims;
    if (i >= N) return;
    const int sp = R.species[i];
    const double kick = R.kick[sp], sig = R.sigma[sp], c1 = R.c1;
    const T* __restrict__ force = (const T*)R.force;
    const T* __restrict__ z = zeta_row + R.dof_off;
    const double* __restrict__ C = R.nm;
    const double* __restrict__ ring = R.ring;
    double umax = 0.0;
    bool finite = true;
    T4* __restrict__ u = (T4*)R.u;
    for (int a = 0; a < dims; ++a) {
        for (int s = 0; s < P; ++s) {
            const size_t idx = ((size_t)s * dims + a) * N + i;
            r[s] = R.pos[idx];
            v[s] = R.vel[idx] + kick * (double)force[idx];
        }
        for (int k = 0; k < P; ++k) {
            double qa = 0.0, pa = 0.0;
            for (int s = 0; s < P; ++s) {
                qa += C[s * P + k] * r[s];
                pa += C[s * P + k] * v[s];
            }
            q[k] = qa;
            p[k] = pa;
        }
        const int64_t dof0 = ((int64_t)dims * i + a) * P;
        for (int k = 0; k < P; ++k) {
            const double cw = ring[k], sw = ring[P + k], ws = ring[2 * P + k];
            double q1 = cw * q[k] + sw * p[k];
            double p1 = ws * q[k] + cw * p[k];
            p1 = c1 * p1 + sig * (double)z[dof0 + k];
            q[k] = cw * q1 + sw * p1;
            p[k] = ws * q1 + cw * p1;
        }
        for (int s = 0; s < P; ++s) {
            double ra = 0.0, va = 0.0;
            for (int k = 0; k < P; ++k) {
                ra += C[s * P + k] * q[k];
                va += C[s * P + k] * p[k];
            }
            const size_t idx = ((size_t)s * dims + a) * N + i;
            R.pos[idx] = ra;
            R.vel[idx] = va;
            finite = finite && __builtin_isfinite(ra) && __builtin_isfinite(va);
            if (PAIR) {
                const double du = ra - R.rref[(size_t)a * N + i];
                umax = fmax(umax, fabs(du));
                T* comp = (T*)&u[(size_t)s * N + i];
                comp[a] = (T)du;
            }
        }
    }
    if (PAIR) {
        const T spb = bits_as<T>(sp);
        for (int s = 0; s < P; ++s) ((T*)&u[(size_t)s * N + i])[3] = spb;
        if (!(umax <= R.u_lim)) atomicOr(R.rebuild, 1);
    }
    if (!finite) atomicOr(status, kStatusNonfinite);
}

template <typename T, bool PAIR>
void launch_T(hipStream_t st, int P, const RepDev* reps, const BlockEntry* blocks, int n_blocks,
              const T* zrow, int32_t* status)
{
    const dim3 g(n_blocks), b(256);
    switch (P) {
#define QTB_UPD(PP) case PP: hipLaunchKernelGGL((k_update<PP, T, PAIR>), g, b, 0, st, reps, blocks, zrow, status); return;
    QTB_UPD(1) QTB_UPD(2) QTB_UPD(3) QTB_UPD(4) QTB_UPD(5) QTB_UPD(6) QTB_UPD(7) QTB_UPD(8)
#undef QTB_UPD
    default: break;
    }
}

}  // namespace

// P <= 8: blocks of 256 atoms.  P > 8: the LDS kernel, whose block table
// holds 64 atoms per entry.
void launch_update(hipStream_t st, bool fp64, bool pair, int P, const RepDev* reps,
                   const BlockEntry* blocks, int n_blocks, const void* zeta_row, int32_t* status)
{
    if (P <= 8) {
        if (fp64) {
            if (pair) launch_T<double, true>(st, P, reps, blocks, n_blocks, (const double*)zeta_row, status);
            else launch_T<double, false>(st, P, reps, blocks, n_blocks, (const double*)zeta_row, status);
        } else {
            if (pair) launch_T<float, true>(st, P, reps, blocks, n_blocks, (const float*)zeta_row, status);
            else launch_T<float, false>(st, P, reps, blocks, n_blocks, (const float*)zeta_row, status);
        }
        return;
    }
    const size_t lds = (size_t)64 * 4 * P * sizeof(double);
    const dim3 g(n_blocks), b(64);
    if (fp64) {
        if (pair) hipLaunchKernelGGL((k_update_lds<double, true>), g, b, lds, st, reps, blocks, (const double*)zeta_row, status);
        else hipLaunchKernelGGL((k_update_lds<double, false>), g, b, lds, st, reps, blocks, (const double*)zeta_row, status);
    } else {
        if (pair) hipLaunchKernelGGL((k_update_lds<float, true>), g, b, lds, st, reps, blocks, (const float*)zeta_row, status);
        else hipLaunchKernelGGL((k_update_lds<float, false>), g, b, lds, st, reps, blocks, (const float*)zeta_row, status);
    }
}

}  // namespace qtb
