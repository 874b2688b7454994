// fir.hip -- coloured noise for K future steps at once.
//
// The QTB random force has the power spectral density 2 m gamma S(omega)
// (eq. 6-7, S = theta of eq. 1; eq. 12, S = kappa_P for QTB-PIMD).  It is
// produced by filtering unit white noise w with the zero-phase FIR taps h
// built on the host: zeta_n = sum_{k=-Nf}^{Nf-1} h_k w_{n-k}.  For a block of
// K steps starting at n_b this is a banded Toeplitz product
//   Z (K x D) = T (K x (K + 2Nf - 1)) . W ((K + 2Nf - 1) x D),
//   T[i][j] = h_{i - j + Nf - 1} on the band j - i in [0, 2Nf - 1],
// with window row j holding step n_b - Nf + 1 + j.  T is never stored: the
// matrix-core A fragments are read straight out of the (zero padded) taps in
// LDS, since an entry depends only on i - j.  B fragments are white-noise
// rows read from the ring buffer in HBM, each element once per block.
//
//  mode 0  FP32:   v_mfma_f32_32x32x2_f32, FP32 accumulation
//  mode 1  BF16x3: v_mfma_f32_32x32x16_bf16 on hi/lo splits of both
//                  operands, hi*hi + hi*lo + lo*hi, FP32 accumulation
//  mode 2  BF16:   hi*hi only
//  mode 3  FP64:   vector FMA, register-blocked over 8 outputs
//
// Ring layouts.  FP32 / FP64 modes: [R][n_cols], row m in slot m mod R.
// BF16 modes: the white noise is stored already split into its BF16 hi and
// lo parts (hi = bf16(w), lo = bf16(w - hi), w the FP32 value), each part a
// plane [R/8][n_cols][8]: the 8 rows of a column that one matrix-core lane
// takes as its B fragment are one aligned 16-byte load.  The window then
// starts at the 8-aligned row J0 = floor8(n_b - Nf + 1); the delta rows
// before the first needed one meet zero taps (the padding).
#include "qtb_internal.h"

namespace qtb {
namespace {

constexpr int kPad = 64;  // zero padding on both sides of the taps in LDS

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t ring_slot(int64_t m, int R)
{
    int64_t s = m % R;
    return s < 0 ? s + R : s;
}

// ------------------------------------------------------------------ FP64
template <int K>
__global__ void __launch_bounds__(256) k_fir_fp64(const FirTile* __restrict__ tiles,
                                                  const double* __restrict__ taps,
                                                  const double* __restrict__ ring,
                                                  double* __restrict__ zeta, int64_t n_cols,
                                                  const int64_t* __restrict__ clock, int R)
{
    extern __shared__ __attribute__((aligned(16))) double sh64[];
    const int64_t nb = *clock;
    const FirTile t = tiles[blockIdx.x];
    const int two_nf = t.two_nf, Nf = two_nf / 2;
    const int L = two_nf + 2 * kPad;
    for (int x = threadIdx.x; x < L; x += blockDim.x) sh64[x] = taps[t.taps_off + x];
    __syncthreads();
    const int64_t col = (int64_t)blockIdx.x * kDofTile + threadIdx.x;
    const int s0 = (int)ring_slot(nb - Nf + 1, R);  // slot of window row 0
    for (int i0 = 0; i0 < K; i0 += 8) {
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        int sl = s0 + i0;
        if (sl >= R) sl -= R;
        for (int j = i0; j < i0 + two_nf + 7; ++j) {
            const double wv = ring[(int64_t)sl * n_cols + col];
            if (++sl == R) sl = 0;
            const int xb = i0 - j + two_nf - 1 + kPad;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = __builtin_fma(sh64[xb + q], wv, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) zeta[(int64_t)(i0 + q) * n_cols + col] = acc[q];
    }
}

// ------------------------------------------------------------------ FP32 MFMA
template <int K>
__global__ void __launch_bounds__(256) k_fir_f32(const FirTile* __restrict__ tiles,
                                                 const float* __restrict__ taps,
                                                 const float* __restrict__ ring,
                                                 float* __restrict__ zeta, int64_t n_cols,
                                                 const int64_t* __restrict__ clock, int R)
{
    extern __shared__ __attribute__((aligned(16))) float sh32[];
    const int64_t nb = *clock;
    constexpr int MT = K / 32;
    const int64_t col0 = (int64_t)blockIdx.x * 128;
    const FirTile t = tiles[col0 / kDofTile];
    const int two_nf = t.two_nf, Nf = two_nf / 2;
    const int L = two_nf + 2 * kPad;
    for (int x = threadIdx.x; x < L; x += blockDim.x) sh32[x] = taps[t.taps_off + x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t col = col0 + 32 * wave + li;
    f32x16 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[mt][r] = 0.0f;
    const int jend = K + two_nf - 1;
    int sl = (int)ring_slot(nb - Nf + 1 + lk, R);  // slot of this lane's row j0 + lk
    for (int j0 = 0; j0 < jend; j0 += 2) {
        const float b = ring[(int64_t)sl * n_cols + col];
        sl += 2;
        if (sl >= R) sl -= R;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int i0 = 32 * mt;
            if (j0 + 1 < i0 || j0 > i0 + 30 + two_nf) continue;
            const float a = sh32[i0 + li - j0 - lk + two_nf - 1 + kPad];
            acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[mt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * mt + 8 * (r >> 2) + 4 * lk + (r & 3);
            zeta[(int64_t)i * n_cols + col] = acc[mt][r];
        }
}

// ------------------------------------------------------------------ BF16 MFMA
__device__ __forceinline__ uint32_t bf16_bits_rn(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

template <int K, bool X3>
__global__ void __launch_bounds__(256) k_fir_bf16(const FirTile* __restrict__ tiles,
                                                  const float* __restrict__ taps,
                                                  const uint16_t* __restrict__ ring_hi,
                                                  const uint16_t* __restrict__ ring_lo,
                                                  float* __restrict__ zeta, int64_t n_cols,
                                                  const int64_t* __restrict__ clock, int R, int LR)
{
    const int64_t nb = *clock;
    // LDS: reversed taps as hi and lo bf16, in 8 copies shifted by 0..7
    // elements so that any 8 consecutive entries are one aligned 16-byte read.
    extern __shared__ __attribute__((aligned(16))) uint16_t shb[];
    uint16_t* Rhi = shb;
    uint16_t* Rlo = shb + 8 * LR;
    constexpr int MT = K / 32;
    const int64_t col0 = (int64_t)blockIdx.x * 128;
    const FirTile t = tiles[col0 / kDofTile];
    const int two_nf = t.two_nf, Nf = two_nf / 2;
    const int Lh = two_nf + 2 * kPad;
    for (int x = threadIdx.x; x < 8 * LR; x += blockDim.x) {
        const int p = x / LR, y = x - p * LR;
        const int yy = y + p;
        float h = 0.0f;
        if (yy < Lh) h = taps[t.taps_off + (Lh - 1 - yy)];
        const uint32_t hi = bf16_bits_rn(h);
        Rhi[x] = (uint16_t)hi;
        Rlo[x] = (uint16_t)bf16_bits_rn(h - bf16_value(hi));
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t col = col0 + 32 * wave + li;
    // window from the 8-aligned row J0 = m0 - delta, m0 = nb - Nf + 1 the
    // first row with a non-zero tap; row J0 + j meets tap index
    // i - j + 2Nf - 1 + delta (zero outside 0 .. 2Nf - 1)
    const int64_t m0 = nb - Nf + 1;
    const int delta = (int)(((m0 % 8) + 8) % 8);
    const int jend = K + two_nf - 1 + delta;
    const int RC = R >> 3;  // 8-row chunks in the ring
    int c = (int)(ring_slot(m0 - delta, R) >> 3) + lk;  // chunk of this lane's rows
    if (c >= RC) c -= RC;
    typedef const __attribute__((address_space(1))) u32x4* gp4;
    const gp4 hp = (gp4)ring_hi + col, lp = (gp4)ring_lo + col;
    f32x16 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[mt][r] = 0.0f;
    for (int j0 = 0; j0 < jend; j0 += 16) {
        const int jb = j0 + 8 * lk;
        const u32x4 ph = hp[(int64_t)c * n_cols];
        const u32x4 pl = lp[(int64_t)c * n_cols];
        c += 2;
        if (c >= RC) c -= RC;
        const bf16x8 Bhi = __builtin_bit_cast(bf16x8, ph);
        const bf16x8 Blo = __builtin_bit_cast(bf16x8, pl);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int i0 = 32 * mt;
            // rows j0 .. j0 + 15 against outputs i0 .. i0 + 31: any tap in band?
            if (j0 + 15 < i0 + delta || j0 > i0 + 30 + delta + two_nf) continue;
            const int X0 = i0 + li - jb + two_nf - 1 + delta + kPad;
            const int s = Lh - 1 - X0;
            const int off = (s & 7) * LR + (s & ~7);
            const bf16x8 Ahi = __builtin_bit_cast(bf16x8, *(const u32x4*)(Rhi + off));
            acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi, Bhi, acc[mt], 0, 0, 0);
            if (X3) {
                const bf16x8 Alo = __builtin_bit_cast(bf16x8, *(const u32x4*)(Rlo + off));
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi, Blo, acc[mt], 0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Alo, Bhi, acc[mt], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * mt + 8 * (r >> 2) + 4 * lk + (r & 3);
            zeta[(int64_t)i * n_cols + col] = acc[mt][r];
        }
}

template <typename F>
void allow_lds(F kernel, size_t bytes)
{
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

template <int K>
void launch_fir_K(hipStream_t st, int mode, const FirTile* tiles, int n_tiles, const void* taps,
                  const void* ring, void* zeta, int64_t n_cols, const int64_t* nb, int R,
                  int max_two_nf)
{
    const int L = max_two_nf + 2 * kPad;
    if (mode == QTB_FIR_FP64) {
        launch(k_fir_fp64<K>, dim3(n_tiles), dim3(256), L * sizeof(double), st,
                           tiles, (const double*)taps, (const double*)ring, (double*)zeta,
                           n_cols, nb, R);
    } else if (mode == QTB_FIR_FP32) {
        launch(k_fir_f32<K>, dim3(n_tiles * 2), dim3(256), L * sizeof(float), st,
                           tiles, (const float*)taps, (const float*)ring, (float*)zeta, n_cols,
                           nb, R);
    } else {
        const int LR = (L + 7) & ~7;
        const size_t lds = (size_t)16 * LR * sizeof(uint16_t);
        allow_lds(k_fir_bf16<K, true>, lds);
        allow_lds(k_fir_bf16<K, false>, lds);
        const uint16_t* hi = (const uint16_t*)ring;
        const uint16_t* lo = hi + (size_t)R * n_cols;
        if (mode == QTB_FIR_BF16X3)
            launch((k_fir_bf16<K, true>), dim3(n_tiles * 2), dim3(256), lds, st,
                               tiles, (const float*)taps, hi, lo, (float*)zeta, n_cols, nb, R, LR);
        else
            launch((k_fir_bf16<K, false>), dim3(n_tiles * 2), dim3(256), lds, st,
                               tiles, (const float*)taps, hi, lo, (float*)zeta, n_cols, nb, R, LR);
    }
}

}  // namespace

int fir_pad() { return kPad; }

size_t fir_lds_bytes(int mode, int max_two_nf)
{
    const int L = max_two_nf + 2 * kPad;
    if (mode == QTB_FIR_FP64) return L * sizeof(double);
    if (mode == QTB_FIR_FP32) return L * sizeof(float);
    return (size_t)16 * ((L + 7) & ~7) * sizeof(uint16_t);
}

void launch_fir(hipStream_t st, int mode, int K, const FirTile* tiles, int n_tiles,
                const void* taps, const void* ring, void* zeta, int64_t n_cols, const int64_t* nb,
                int R, int max_two_nf)
{
    switch (K) {
    case 64: launch_fir_K<64>(st, mode, tiles, n_tiles, taps, ring, zeta, n_cols, nb, R, max_two_nf); break;
    case 128: launch_fir_K<128>(st, mode, tiles, n_tiles, taps, ring, zeta, n_cols, nb, R, max_two_nf); break;
    case 256: launch_fir_K<256>(st, mode, tiles, n_tiles, taps, ring, zeta, n_cols, nb, R, max_two_nf); break;
    default: break;  // rejected at init
    }
}

}  // namespace qtb
