// ring_step.h -- arithmetic of the update shared by the separate update
// kernel and the one-kernel step, written with explicit fused multiply-adds
// so that both produce the same bits.
#pragma once

namespace qtb {

// Normal-mode transform term: acc + c x.
__device__ __forceinline__ double nm_acc(double acc, double c, double x)
{
    return __builtin_fma(c, x, acc);
}

// Half-kick B(dt/2): v + kick f.
__device__ __forceinline__ double half_kick(double v, double kick, double f)
{
    return __builtin_fma(kick, f, v);
}

// One normal mode through A(dt/2) O(dt) A(dt/2): the free ring-polymer
// oscillator (cw = cos(w h), sw = sin(w h)/w, ws = -w sin(w h), h = dt/2;
// w = 0 drifts) around the Langevin step p <- c1 p + sig z.
__device__ __forceinline__ void mode_aoa(double& q, double& p, double cw, double sw, double ws,
                                         double c1, double sig, double z)
{
    const double q1 = __builtin_fma(cw, q, sw * p);
    double p1 = __builtin_fma(ws, q, cw * p);
    p1 = __builtin_fma(c1, p1, sig * z);
    q = __builtin_fma(cw, q1, sw * p1);
    p = __builtin_fma(ws, q1, cw * p1);
}

}  // namespace qtb
