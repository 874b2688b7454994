// fft_lds.h -- in-place FP64 FFT of columns held in LDS, shared by the
// velocity-spectrum transform and the block noise generator.
//
// Decimation in frequency on naturally ordered input; two radix-2 stages per
// LDS round trip (a radix-4 butterfly: four loads, the arithmetic of both
// stages in registers, four stores), a single radix-2 stage last when log2 n
// is odd; bin k ends at position bit_reverse(k).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtb {

__device__ __forceinline__ double2 cmul(double2 a, double2 w)
{
    return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

__device__ __forceinline__ int bit_reverse(int k, int L2)
{
    return (int)(__builtin_bitreverse32((uint32_t)k) >> (32 - L2));
}

// Two decimation-in-frequency stages (spans 2 h2 and h2) on the four points
// z[0], z[h2], z[2 h2], z[3 h2]: w1 = W_{4 h2}^pos, w2 = W_{2 h2}^pos.
__device__ __forceinline__ void dif4(double2& a, double2& b, double2& c, double2& d, double2 w1,
                                     double2 w2)
{
    const double2 a1 = make_double2(a.x + c.x, a.y + c.y);
    const double2 c1 = cmul(make_double2(a.x - c.x, a.y - c.y), w1);
    const double2 b1 = make_double2(b.x + d.x, b.y + d.y);
    const double2 e = cmul(make_double2(b.x - d.x, b.y - d.y), w1);
    const double2 d1 = make_double2(e.y, -e.x);  // times W_4 = -i
    a = make_double2(a1.x + b1.x, a1.y + b1.y);
    b = cmul(make_double2(a1.x - b1.x, a1.y - b1.y), w2);
    c = make_double2(c1.x + d1.x, c1.y + d1.y);
    d = cmul(make_double2(c1.x - d1.x, c1.y - d1.y), w2);
}

// Forward DFT X_k = sum_t x_t e^{-2 pi i k t / n}, n = 2^L2 >= 4, of the cw
// columns zb[q n, q n + n), in place; X_k lands at bit_reverse(k, L2).
// tw(k) = e^{-2 pi i k / n} for k < n/2.  Every thread of the block calls
// it after a barrier that publishes the input; it ends with a barrier.
template <typename TW>
__device__ __forceinline__ void fft_dif_lds(double2* zb, int cw, int L2, const TW& tw)
{
    const int seg = 1 << L2, hseg = seg >> 1;
    const int n_b = cw << (L2 - 2);  // radix-4 butterflies per pair of stages
    int s = L2;
    for (; s >= 2; s -= 2) {
        const int lh2 = s - 2, h2 = 1 << lh2;
        // two butterflies per thread and pass: their LDS loads overlap
        for (int b0 = threadIdx.x; b0 < n_b; b0 += 2 * blockDim.x) {
            const int b1 = b0 + blockDim.x;
            const bool two = b1 < n_b;
            double2 *z0, *z1;
            double2 w10, w20, w11, w21;
            {
                const int q = b0 >> (L2 - 2), jb = b0 & ((seg >> 2) - 1), pos = jb & (h2 - 1);
                z0 = zb + (size_t)q * seg + ((jb >> lh2) << s) + pos;
                w10 = tw(pos << (L2 - s));
                w20 = tw(pos << (L2 - s + 1));
            }
            {
                const int bb = two ? b1 : b0;
                const int q = bb >> (L2 - 2), jb = bb & ((seg >> 2) - 1), pos = jb & (h2 - 1);
                z1 = zb + (size_t)q * seg + ((jb >> lh2) << s) + pos;
                w11 = tw(pos << (L2 - s));
                w21 = tw(pos << (L2 - s + 1));
            }
            double2 a0 = z0[0], p0 = z0[h2], c0 = z0[2 * h2], d0 = z0[3 * h2];
            double2 a1 = z1[0], p1 = z1[h2], c1 = z1[2 * h2], d1 = z1[3 * h2];
            dif4(a0, p0, c0, d0, w10, w20);
            dif4(a1, p1, c1, d1, w11, w21);
            z0[0] = a0;
            z0[h2] = p0;
            z0[2 * h2] = c0;
            z0[3 * h2] = d0;
            if (two) {
                z1[0] = a1;
                z1[h2] = p1;
                z1[2 * h2] = c1;
                z1[3 * h2] = d1;
            }
        }
        __syncthreads();
    }
    if (s == 1) {  // odd number of stages: the last one has span 1
        for (int m = threadIdx.x; m < cw * hseg; m += blockDim.x) {
            double2* z = zb + 2 * (size_t)m;
            const double2 a = z[0], b = z[1];
            z[0] = make_double2(a.x + b.x, a.y + b.y);
            z[1] = make_double2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
    }
}

}  // namespace qtb
