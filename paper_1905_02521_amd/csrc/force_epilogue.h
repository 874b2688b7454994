// force_epilogue.h -- end of a force kernel for one (atom, bead): store the
// force -grad V(r^(s)) (the 1/P of eq. 4 is folded into the kick), close the
// step with the second half-kick B(dt/2), and sample the eq. (5) observables.
#pragma once

#include "qtb_internal.h"

namespace qtb {

// State read from global memory (the separate force kernel).
struct GlobalState {
    const RepDev& R;
    int i;
    __device__ __forceinline__ double pos(int b, int a) const
    {
        return R.pos[((size_t)b * 3 + a) * R.N + i];
    }
    __device__ __forceinline__ double vel(int b, int a) const
    {
        return R.vel[((size_t)b * 3 + a) * R.N + i];
    }
};

// The velocity recorder's row [dims][N] that a sampling force pass fills
// (null: none).  Kernels read it before the force loop, so that the two
// dependent loads overlap the force arithmetic instead of the kernel's tail.
__device__ __forceinline__ double* recorder_row(const RepDev& R, int32_t flags)
{
    if (!(flags & kSample) || !R.vt) return nullptr;
    return R.vt + (*R.vt_n % R.vt_cap) * R.dims * R.N;
}

// e_atom: this atom's share of the bead potential V(r^(s)).
// ob (kNobs slots): kinetic, V/P, spring, virial, x^2 in kSample mode
// (kPressure alone: kinetic and spring);
// |F - F_stored|^2 and |F|^2 in kCompare mode (nothing is written then).
// vn receives the velocity after the kick; STORE_V: write it back.  A sample
// also stores vn into the velocity recorder's row vrec (recorder_row).
template <typename T, bool STORE_V = true, typename Src>
__device__ __forceinline__ void force_epilogue_src(const RepDev& R, int i, int s, int spi,
                                                   const double f[3], double e_atom,
                                                   int32_t flags, double* ob, const Src& src,
                                                   double* vn, double* vrec)
{
    const int N = R.N, P = R.P;
    T* __restrict__ force = (T*)R.force;
    if (flags & kCompare) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double d = f[a] - (double)force[((size_t)s * 3 + a) * N + i];
            ob[0] += d * d;
            ob[1] += f[a] * f[a];
        }
        return;
    }
    const double kick = R.kick[spi];
    const double sv2 = R.npt_sv2;  // a barostat's pending scaling after the kick (else 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const size_t idx = ((size_t)s * 3 + a) * N + i;
        force[idx] = (T)f[a];
        double v = src.vel(s, a);
        if (flags & kKick) {
            v = __builtin_fma(kick, f[a], v) * sv2;  // half-kick B(dt/2)
            if (STORE_V) R.vel[idx] = v;
        }
        vn[a] = v;
    }
    if (flags & kEvaluate) R.eatom[(size_t)s * N + i] = e_atom;
    if (flags & kSample) {
        const double m = R.mmu[spi];
        const int sn = (s + 1 == P) ? 0 : s + 1;
        double ke = 0.0, spr = 0.0, vir = 0.0, x2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t idx = ((size_t)s * 3 + a) * N + i;
            const double ra = src.pos(s, a);
            double c = 0.0;
            for (int b = 0; b < P; ++b) c += src.pos(b, a);
            c /= P;
            const double dn = ra - src.pos(sn, a);
            const double d0 = ra - R.r0[idx];
            ke = __builtin_fma(vn[a], vn[a], ke);
            spr = __builtin_fma(dn, dn, spr);
            vir = __builtin_fma(ra - c, f[a], vir);
            x2 = __builtin_fma(d0, d0, x2);
        }
        ob[0] = 0.5 * m * ke;
        ob[1] = e_atom / P;
        ob[2] = (P > 1) ? 0.5 * m * R.omega_P * R.omega_P * spr : 0.0;
        ob[3] = vir;
        ob[4] = x2;
        if (vrec) {  // velocity recorder (P = 1)
#pragma unroll
            for (int a = 0; a < 3; ++a) vrec[(size_t)a * N + i] = vn[a];
        }
    } else if (flags & kPressure) {  // kinetic energy and springs only
        const double m = R.mmu[spi];
        const int sn = (s + 1 == P) ? 0 : s + 1;
        double ke = 0.0, spr = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ke = __builtin_fma(vn[a], vn[a], ke);
            if (P > 1) {
                const double dn = src.pos(s, a) - src.pos(sn, a);
                spr = __builtin_fma(dn, dn, spr);
            }
        }
        ob[0] = 0.5 * m * ke;
        ob[2] = (P > 1) ? 0.5 * m * R.omega_P * R.omega_P * spr : 0.0;
    }
}

template <typename T>
__device__ __forceinline__ void force_epilogue(const RepDev& R, int i, int s, int spi,
                                               const double f[3], double e_atom, int32_t flags,
                                               double* ob, double* vrec)
{
    double vn[3];
    force_epilogue_src<T, true>(R, i, s, spi, f, e_atom, flags, ob, GlobalState{R, i}, vn, vrec);
}

}  // namespace qtb
