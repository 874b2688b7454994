// force_epilogue.h -- end of a force kernel for one (atom, bead): store the
// force -grad V(r^(s)) (the 1/P of eq. 4 is folded into the kick), close the
// step with the second half-kick B(dt/2), and sample the eq. (5) observables.
#pragma once

#include "qtb_internal.h"

namespace qtb {

// e_atom: this atom's share of the bead potential V(r^(s)).
// ob (kNobs slots): kinetic, V/P, spring, virial, x^2 in kSample mode;
// |F - F_stored|^2 and |F|^2 in kCompare mode (nothing is written then).
template <typename T>
__device__ __forceinline__ void force_epilogue(const RepDev& R, int i, int s, int spi,
                                               const double f[3], double e_atom, int32_t flags,
                                               double* ob)
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
    if (flags & kEvaluate) R.eatom[(size_t)s * N + i] = e_atom;
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
        ob[1] = e_atom / P;
        ob[2] = (P > 1) ? 0.5 * m * R.omega_P * R.omega_P * spr : 0.0;
        ob[3] = vir;
        ob[4] = x2;
    }
}

}  // namespace qtb
