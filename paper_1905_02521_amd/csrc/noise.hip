// noise.hip -- counter-based white noise for the QTB random force.
//
// The paper draws the a_j, b_j of eq. (9) from a normal distribution and
// says no more; this library fixes a reproducible generator: one
// Philox4x32-10 block (Salmon et al., SC'11) per (step, dof) turned into one
// unit Gaussian.  Every operation of the transform is spelled out (no
// library ln / cos, no contraction) so that any implementation of the same
// specification produces the same bits:
//   counter = (lo, hi of n + 2^40, dof, 16 stream + tag), key = seed words
//   u1 = (2 m1 + 1) 2^-53, m1 = (x0 >> 6) 2^26 + (x1 >> 6)      (exact)
//   N2 = 2 m2 + 1,         m2 = (x2 >> 6) 2^26 + (x3 >> 6)
//   w  = sqrt(-2 ln u1) cos(2 pi N2 / 2^53)
// ln: exponent split, f in (1/sqrt2, sqrt2], s = (f-1)/(f+1), Horner in s^2
// of the atanh series to s^22/23, e ln2 with the fdlibm hi/lo split.
// cos: quadrant q = round(4u) taken on the integer, r = 4u - q exact,
// x = r pi/2 (hi/lo), Taylor series of cos and sin to x^18 / x^19.
#include "fft_lds.h"
#include "qtb_internal.h"

#pragma clang fp contract(off)

namespace qtb {
namespace {

__device__ __forceinline__ void philox_4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double spec_log(double u)
{
    const uint64_t bits = __double_as_longlong(u);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    double f = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) |
                                                0x3FF0000000000000ull));
    if (f > 1.4142135623730951) {
        f = f * 0.5;
        e = e + 1;
    }
    const double s = (f - 1.0) / (f + 1.0);
    const double z = s * s;
    double q = 1.0 / 23.0;
    q = __builtin_fma(q, z, 1.0 / 21.0);
    q = __builtin_fma(q, z, 1.0 / 19.0);
    q = __builtin_fma(q, z, 1.0 / 17.0);
    q = __builtin_fma(q, z, 1.0 / 15.0);
    q = __builtin_fma(q, z, 1.0 / 13.0);
    q = __builtin_fma(q, z, 1.0 / 11.0);
    q = __builtin_fma(q, z, 1.0 / 9.0);
    q = __builtin_fma(q, z, 1.0 / 7.0);
    q = __builtin_fma(q, z, 1.0 / 5.0);
    q = __builtin_fma(q, z, 1.0 / 3.0);
    q = __builtin_fma(q, z, 1.0);
    const double t = s * q;
    const double lnf = t + t;
    const double de = (double)e;
    const double hi = de * 6.93147180369123816490e-01;
    const double lo = __builtin_fma(de, 1.90821492927058770002e-10, lnf);
    return hi + lo;
}

__device__ __forceinline__ double spec_cos2pi(uint64_t N)
{
    const uint64_t q = (N + (1ull << 50)) >> 51;
    const int64_t rem = (int64_t)N - (int64_t)(q << 51);
    const double r = (double)rem * 4.4408920985006262e-16;  // 2^-51
    const double xh = r * 1.5707963267948966;
    const double x = __builtin_fma(r, 6.123233995736766e-17, xh);
    const double z = x * x;
    double c = -1.0 / 6402373705728000.0;
    c = __builtin_fma(c, z, 1.0 / 20922789888000.0);
    c = __builtin_fma(c, z, -1.0 / 87178291200.0);
    c = __builtin_fma(c, z, 1.0 / 479001600.0);
    c = __builtin_fma(c, z, -1.0 / 3628800.0);
    c = __builtin_fma(c, z, 1.0 / 40320.0);
    c = __builtin_fma(c, z, -1.0 / 720.0);
    c = __builtin_fma(c, z, 1.0 / 24.0);
    c = __builtin_fma(c, z, -1.0 / 2.0);
    const double cosx = __builtin_fma(c, z, 1.0);
    double p = -1.0 / 121645100408832000.0;
    p = __builtin_fma(p, z, 1.0 / 355687428096000.0);
    p = __builtin_fma(p, z, -1.0 / 1307674368000.0);
    p = __builtin_fma(p, z, 1.0 / 6227020800.0);
    p = __builtin_fma(p, z, -1.0 / 39916800.0);
    p = __builtin_fma(p, z, 1.0 / 362880.0);
    p = __builtin_fma(p, z, -1.0 / 5040.0);
    p = __builtin_fma(p, z, 1.0 / 120.0);
    p = __builtin_fma(p, z, -1.0 / 6.0);
    const double xz = x * z;
    const double sinx = __builtin_fma(xz, p, x);
    const uint32_t quad = (uint32_t)q & 3u;
    const double v = (quad & 1u) ? sinx : cosx;
    return (quad == 1u || quad == 2u) ? -v : v;
}

}  // namespace

__device__ __forceinline__ double white_gauss(uint64_t seed, int64_t n, uint32_t d,
                                              uint32_t stream, uint32_t tag)
{
    const uint64_t cnt = (uint64_t)(n + ((int64_t)1 << 40));
    uint32_t c[4] = {(uint32_t)cnt, (uint32_t)(cnt >> 32), d, stream * 16u + tag};
    philox_4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t m1 = ((uint64_t)(c[0] >> 6) << 26) | (uint64_t)(c[1] >> 6);
    const uint64_t m2 = ((uint64_t)(c[2] >> 6) << 26) | (uint64_t)(c[3] >> 6);
    const double u1 = (double)(2 * m1 + 1) * 1.1102230246251565e-16;  // 2^-53
    const double a = -2.0 * spec_log(u1);
    return __builtin_sqrt(a) * spec_cos2pi(2 * m2 + 1);
}

namespace {

__global__ void k_gaussian(uint64_t seed, uint32_t stream, uint32_t tag, int64_t n0,
                           int64_t n_rows, uint32_t d0, uint32_t n_dof, double* __restrict__ out)
{
    const int64_t total = n_rows * (int64_t)n_dof;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = id / n_dof;
        const uint32_t j = (uint32_t)(id - r * n_dof);
        out[id] = white_gauss(seed, n0 + r, d0 + j, stream, tag);
    }
}

// White-noise rows m0 .. m0+rows-1 (global step index) for every column of
// the concatenated replica dof ranges, stored at ring row m mod R.
template <typename T>
__global__ void k_gen_white(const RepDev* __restrict__ reps, const FirTile* __restrict__ tiles,
                            T* __restrict__ ring, const int64_t* __restrict__ clock, int64_t off,
                            int R, int64_t n_cols)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = *clock + off + blockIdx.y;
    if (col >= n_cols) return;
    const int tile = (int)(col / kDofTile);
    const int rep = __builtin_amdgcn_readfirstlane(tiles[tile].rep);
    const RepDev& Rp = reps[rep];
    const int64_t d = col - Rp.dof_off;
    const int64_t D = (int64_t)Rp.dims * Rp.N * Rp.P;
    T w = T(0);
    if (d < D) w = (T)white_gauss(Rp.seed, m + Rp.step_off, (uint32_t)d, Rp.stream, 0);
    int64_t slot = m % R;
    if (slot < 0) slot += R;
    ring[slot * n_cols + col] = w;
}

__device__ __forceinline__ uint32_t bf16_rn_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

// The same rows for the BF16 matrix-core FIR: each FP32 value w split into
// hi = bf16(w) and lo = bf16(w - hi), stored in two planes [R/8][n_cols][8]
// (R a multiple of 8): one thread per column and aligned group of 8 rows,
// blockIdx.y the group; rows of the group outside m0 .. m0+rows-1 are left
// alone.  A full group is one 16-byte store per plane.
__global__ void k_gen_white_split(const RepDev* __restrict__ reps,
                                  const FirTile* __restrict__ tiles, uint16_t* __restrict__ hi,
                                  uint16_t* __restrict__ lo, const int64_t* __restrict__ clock,
                                  int64_t off, int rows, int R, int64_t n_cols)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n_cols) return;
    const int64_t m0 = *clock + off, m1 = m0 + rows;
    const int64_t g0 = m0 - (((m0 % 8) + 8) % 8);  // first row of the first group
    const int64_t gm = g0 + 8 * (int64_t)blockIdx.y;
    const int tile = (int)(col / kDofTile);
    const int rep = __builtin_amdgcn_readfirstlane(tiles[tile].rep);
    const RepDev& Rp = reps[rep];
    const int64_t d = col - Rp.dof_off;
    const int64_t D = (int64_t)Rp.dims * Rp.N * Rp.P;
    uint32_t h[8], l[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t m = gm + q;
        float w = 0.0f;
        if (m >= m0 && m < m1 && d < D)
            w = (float)white_gauss(Rp.seed, m + Rp.step_off, (uint32_t)d, Rp.stream, 0);
        h[q] = bf16_rn_bits(w);
        l[q] = bf16_rn_bits(w - __uint_as_float(h[q] << 16));
    }
    int64_t slot = gm % R;
    if (slot < 0) slot += R;
    const size_t base = ((size_t)(slot >> 3) * n_cols + col) * 8;
    if (gm >= m0 && gm + 8 <= m1) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        u4 ph, pl;
        ph[0] = h[0] | (h[1] << 16); ph[1] = h[2] | (h[3] << 16);
        ph[2] = h[4] | (h[5] << 16); ph[3] = h[6] | (h[7] << 16);
        pl[0] = l[0] | (l[1] << 16); pl[1] = l[2] | (l[3] << 16);
        pl[2] = l[4] | (l[5] << 16); pl[3] = l[6] | (l[7] << 16);
        *(u4*)(hi + base) = ph;
        *(u4*)(lo + base) = pl;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t m = gm + q;
            if (m >= m0 && m < m1) {
                hi[base + q] = (uint16_t)h[q];
                lo[base + q] = (uint16_t)l[q];
            }
        }
    }
}

}  // namespace

void launch_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, uint32_t tag, int64_t n0,
                     int64_t n_rows, uint32_t d0, uint32_t n_dof, double* out)
{
    const int64_t total = n_rows * (int64_t)n_dof;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return;
    launch(k_gaussian, dim3((unsigned)blocks), dim3(256), 0, st, seed, stream, tag,
                       n0, n_rows, d0, n_dof, out);
}

void launch_gen_white(hipStream_t st, const RepDev* reps, const FirTile* tiles, void* ring,
                      int fir_mode, const int64_t* clock, int64_t off, int rows, int R,
                      int64_t n_cols)
{
    if (rows <= 0) return;
    if (fir_mode == QTB_FIR_BF16X3 || fir_mode == QTB_FIR_BF16) {
        // groups of 8 rows touched by rows clock+off .. clock+off+rows-1
        // (the clock's alignment mod 8 is unknown here: one group spare)
        dim3 grid((unsigned)((n_cols + 255) / 256), (unsigned)((rows + 7) / 8 + 1));
        uint16_t* hi = (uint16_t*)ring;
        launch(k_gen_white_split, grid, dim3(256), 0, st, reps, tiles, hi, hi + (size_t)R * n_cols,
               clock, off, rows, R, n_cols);
        return;
    }
    dim3 grid((unsigned)((n_cols + 255) / 256), (unsigned)rows);
    if (fir_mode == QTB_FIR_FP64)
        launch(k_gen_white<double>, grid, dim3(256), 0, st, reps, tiles,
                           (double*)ring, clock, off, R, n_cols);
    else
        launch(k_gen_white<float>, grid, dim3(256), 0, st, reps, tiles,
                           (float*)ring, clock, off, R, n_cols);
}

namespace {

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b)
{
    const int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// The paper's generator (eq. 9): one block of n steps of coloured noise per
// dof from random Fourier amplitudes on the grid omega_j = 2 pi j / (n dt),
// then an inverse transform.  Mode j of a dof has the amplitude
// A_j (a_j + i b_j), A_j = sqrt(n S_j / 2), and its mirror n - j the complex
// conjugate, so the noise is real (the paper leaves this implicit); the
// self-conjugate modes 0 and n/2 are real, A_j a_j with A_j = sqrt(n S_j).
// a_j, b_j: the library's unit Gaussians at (replica step of the block's
// first step + j, dof, tags 1 and 2).  Noise block B (global steps
// B n .. B n + n - 1) lives in half B mod 2 of the [2 n][n_cols] buffer, so a
// K-step noise block that crosses a boundary finds both; blockIdx.y = 0 / 1
// makes the block of the K-step block's first / last step, unless the marker
// of its half says it is there already (the launch then costs one early
// exit per block: the grid is capped and strides over the column groups).
// Two real dofs share one complex transform (x + i y), computed as
// conj(FFT(conj Z)) / n in LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_eq9(const RepDev* __restrict__ reps,
                                             const FirTile* __restrict__ tiles,
                                             const double* __restrict__ amp, int amp_stride,
                                             const double* __restrict__ tw_g, int L2, int cw,
                                             T* __restrict__ zeta, int64_t n_cols,
                                             const int64_t* __restrict__ clock,
                                             const int64_t* __restrict__ marker, int K,
                                             int64_t n_groups)
{
    extern __shared__ double2 zb[];  // [cw][n]
    const int n = 1 << L2, h = n >> 1;
    const int64_t s0 = *clock;
    const int64_t B = floor_div(s0 + (blockIdx.y ? K - 1 : 0), n);
    if (blockIdx.y == 1 && B == floor_div(s0, n)) return;
    const int half = (int)(B & 1);
    if (marker[half] == B) return;
    for (int64_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const int64_t c0 = g * 2 * cw;  // first real column of the group
        const int rep = __builtin_amdgcn_readfirstlane(tiles[c0 / kDofTile].rep);
        const RepDev& R = reps[rep];
        const double* __restrict__ A = amp + (size_t)rep * amp_stride;
        const int64_t D = (int64_t)R.dims * R.N * R.P;
        const int64_t row0 = B * n + R.step_off;
        for (int e = threadIdx.x; e < cw * (h + 1); e += blockDim.x) {
            const int q = e / (h + 1), j = e - q * (h + 1);
            const int64_t dx = c0 + 2 * q - R.dof_off, dy = dx + 1;
            const bool inner = j > 0 && j < h;
            double ax = 0.0, bx = 0.0, ay = 0.0, by = 0.0;
            if (dx < D) {
                ax = white_gauss(R.seed, row0 + j, (uint32_t)dx, R.stream, 1);
                if (inner) bx = white_gauss(R.seed, row0 + j, (uint32_t)dx, R.stream, 2);
            }
            if (dy < D) {
                ay = white_gauss(R.seed, row0 + j, (uint32_t)dy, R.stream, 1);
                if (inner) by = white_gauss(R.seed, row0 + j, (uint32_t)dy, R.stream, 2);
            }
            const double Aj = A[j];
            const double xr = Aj * ax, xi = Aj * bx, yr = Aj * ay, yi = Aj * by;
            // Z_j = X_j + i Y_j and Z_{n-j} = conj(X_j) + i conj(Y_j), stored conjugated
            double2* z = zb + (size_t)q * n;
            z[j] = make_double2(xr - yi, -(xi + yr));
            if (inner) z[n - j] = make_double2(xr + yi, xi - yr);
        }
        __syncthreads();
        auto tw = [&](int k) -> double2 { return reinterpret_cast<const double2*>(tw_g)[k]; };
        fft_dif_lds(zb, cw, L2, tw);
        const double inv = 1.0 / (double)n;
        T* __restrict__ out = zeta + (size_t)half * n * n_cols + c0;
        for (int e = threadIdx.x; e < n * cw; e += blockDim.x) {
            const int t = e / cw, q = e - t * cw;
            const double2 F = zb[(size_t)q * n + bit_reverse(t, L2)];
            out[(size_t)t * n_cols + 2 * q] = (T)(F.x * inv);
            out[(size_t)t * n_cols + 2 * q + 1] = (T)(-F.y * inv);
        }
        __syncthreads();  // the next group overwrites the LDS columns
    }
}

// Isotropic barostats, one block per replica, after the step of replica step
// n closed (its force pass sampled): the ring polymer's primitive pressure
//   p = (2K - 2 U_spring + W / P) / (3V)
// from the force pass's block sums (the order of the observables'
// reduction), K and U_spring over all beads, W the pair virial summed over
// the beads (P = 1: the virial pressure), and g the unit Gaussian at
// (replica step n, dof 0, tag 4).
//
// Stochastic cell rescaling (after Bernetti and Bussi, J. Chem. Phys. 153,
// 114107 (2020)), one Euler-Maruyama (Ito) step of eps = ln V:
//   d eps = -(beta_T / tau_p) (P0 - p) dt + sqrt(2 k_B T beta_T dt / (V tau_p)) g,
//   s = e^{d eps / 3},  s_v1 = 1 / s,  s_v2 = 1.
// With the diffusion in eps proportional to 1/V this samples
// V^N e^{-P0 V / k_B T} for an ideal gas.
//
// Langevin piston (Quigley and Probert, J. Chem. Phys. 120, 11432 (2004),
// isotropic, in the Martyna-Tobias-Klein form): the strain ln(V) / 3 has a
// momentum p_e of mass W_p, driven by G = 3V (p - P0) + (3 / N_f) 2K,
// N_f = 3 N P, with friction gamma_p at temperature T:
//   p_e <- c_p (p_e + dt G / 2) + sqrt((1 - c_p^2) W_p k_B T) g + dt G / 2,
//   s = e^{dt p_e / W_p},  s_v1 = s_v2 = e^{-(1 + 3 / N_f) dt p_e / (2 W_p)}.
//
// The next step applies s_v1 to the velocities before its first kick,
// sqrt(s) to the normal-mode positions before and after its A-O-A (update
// kernel) and s_v2 after its closing kick (force epilogue); its force pass
// and sample take box and list scale times s, and this kernel, at the end of
// that step, first commits s to them.  Between steps box and positions so
// agree, and force passes there see the system as it is.  The neighbour
// lists follow the box through npt_S (below) until a compression eats into
// the skin.  A replica whose barostat is off has its pending factors
// committed and reset to 1 here, after the step that applied them.
// Block of 320 threads: the first four wavefronts sum the block partials,
// the fifth draws the Gaussian meanwhile (both feed thread 0's update).
constexpr int kBaroThreads = 320;

__global__ void __launch_bounds__(kBaroThreads) k_barostat(RepDev* __restrict__ reps, int n_rep,
                                                           const double* __restrict__ partials,
                                                           const StepRef sync,
                                                           int32_t* __restrict__ status)
{
    __shared__ double red[3][256];
    __shared__ double gsh;
    const int r = blockIdx.x;
    if (r >= n_rep) return;
    RepDev& R = reps[r];
    const int t = threadIdx.x;
    // Every value of the replica is read before the first store to it: the
    // stores would otherwise hold back the loads that follow them.
    const int64_t n = (sync.clk ? *sync.clk : 0) + sync.off;
    int64_t f1 = (n + 1) % 3, f2 = (n + 2) % 3;
    if (f1 < 0) f1 += 3;
    if (f2 < 0) f2 += 3;
    const int npt = R.npt;
    const int nblk = R.obs_nblocks;
    const int64_t blk0 = R.obs_block0;
    const double sr = R.npt_sr;
    // the factor this step applied: box and list scale follow.  This step
    // rebuilt the lists (in the force pass, whose flag stays set, or in the
    // list kernel, which marks its builds): entries in its geometry
    const double box0 = R.box[0] * sr, box1 = R.box[1] * sr, box2 = R.box[2] * sr;
    const double S0 = (R.rflag[f1] != 0 || R.list_built != 0) ? 1.0 : R.npt_S * sr;
    const int P = R.P, N = R.N;
    const double dt = R.dt, kT = R.kT, P0 = R.npt_P0;
    const double beta = R.npt_beta, tau = R.npt_tau, gp = R.npt_gp, Wp = R.npt_W;
    const double pe0 = R.npt_pe, hs0 = R.half_skin0, rcs = R.r_cs;
    const uint64_t seed = R.seed;
    const int64_t step_off = R.step_off;
    const uint32_t stream = R.stream;
    if (t == 0) {
        R.box[0] = box0;
        R.box[1] = box1;
        R.box[2] = box2;
        R.npt_S = S0;
        R.list_built = 0;
    }
    if (!npt) {
        if (t == 0) R.npt_sr = R.npt_sv1 = R.npt_sv2 = 1.0;
        return;
    }
    if (t >= 256) {
        if (t == 256) gsh = white_gauss(seed, n + step_off, 0u, stream, 4);
    } else {
        // partials t, t + 256, ... added in that order; loads four at a time
        double ke = 0.0, spr = 0.0, w = 0.0;
        int b = t;
        for (; b + 768 < nblk; b += 1024) {
            double k4[4], s4[4], w4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double* q = partials + (size_t)(blk0 + b + 256 * u) * kNobs;
                k4[u] = q[0];
                s4[u] = q[2];
                w4[u] = q[5];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ke += k4[u];
                spr += s4[u];
                w += w4[u];
            }
        }
        for (; b < nblk; b += 256) {
            const double* q = partials + (size_t)(blk0 + b) * kNobs;
            ke += q[0];
            spr += q[2];
            w += q[5];
        }
        red[0][t] = ke;
        red[1][t] = spr;
        red[2][t] = w;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] += red[1][t + h];
            red[2][t] += red[2][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double V = box0 * box1 * box2;  // committed above
        const double K = red[0][0];
        const double p = (2.0 * K - 2.0 * red[1][0] + red[2][0] / P) / (3.0 * V);
        const double g = gsh;
        double sc, sv1, sv2;
        if (npt == 1) {
            const double deps = -(beta / tau) * (P0 - p) * dt +
                                sqrt(2.0 * kT * beta * dt / (V * tau)) * g;
            sc = exp(deps / 3.0);
            sv1 = 1.0 / sc;
            sv2 = 1.0;
        } else {
            const double Nf = 3.0 * N * P;
            const double G = 3.0 * V * (p - P0) + (3.0 / Nf) * 2.0 * K;
            const double cp = exp(-gp * dt);
            double pe = pe0 + 0.5 * dt * G;
            pe = cp * pe + sqrt((1.0 - cp * cp) * Wp * kT) * g;
            pe += 0.5 * dt * G;
            R.npt_pe = pe;
            const double ve = pe / Wp;
            sc = exp(dt * ve);
            sv1 = sv2 = exp(-(1.0 + 3.0 / Nf) * 0.5 * dt * ve);
        }
        R.npt_sr = sc;
        R.npt_sv1 = sv1;
        R.npt_sv2 = sv2;
        // The lists keep the geometry of their build, scaled by npt_S.  A pair
        // left out at the build lay beyond r_c + skin + dev_i + dev_j, and
        // lies beyond S = npt_S s times that when the next force pass runs:
        // while S < 1 the displacement allowed before a rebuild shrinks by
        // (1 - S)(r_c + skin) / 2 here and by (1 - S) dev_i in the update
        // kernel's test.  Past half of the skin the next step's force pass
        // rebuilds.
        const double S = S0 * sc;
        const double hs = hs0 - fmax(0.0, 1.0 - S) * 0.5 * rcs;
        R.half_skin = hs;
        if (hs < 0.5 * hs0) {  // (the list kernel reads the context-wide flag)
            R.rflag[f2] = 1;
            atomicOr(status + kAnyRebuild + f2, 1);
        }
    }
}

// After k_eq9: record which noise block each half holds (invalidate: none).
__global__ void k_eq9_mark(const int64_t* __restrict__ clock, int64_t* __restrict__ marker, int n,
                           int K, int invalidate)
{
    if (threadIdx.x != 0) return;
    if (invalidate) {
        marker[0] = marker[1] = INT64_MIN;
        return;
    }
    const int64_t s0 = *clock;
    for (int y = 0; y < 2; ++y) {
        const int64_t B = floor_div(s0 + (y ? K - 1 : 0), n);
        marker[B & 1] = B;
    }
}

}  // namespace

namespace {
// Initial surrogate weights: N(0, 1/fan_in) from the same generator (tag 3,
// step 0, dof = parameter index); biases zero.
__global__ void k_ml_init(float* __restrict__ master, uint64_t seed)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlParams) return;
    const int off = p % kMlParamsSp;
    double scale = 0.0;
    if (off < kMlOffB1) scale = 1.0 / sqrt((double)kMlFeat);
    else if (off >= kMlOffW2 && off < kMlOffB2) scale = 1.0 / sqrt((double)kMlHidden);
    else if (off >= kMlOffW3 && off < kMlOffB3) scale = 1.0 / sqrt((double)kMlHidden);
    master[p] = scale == 0.0 ? 0.0f : (float)(scale * white_gauss(seed, 0, (uint32_t)p, 0, 3));
}

__global__ void k_clock(int64_t* clock, int64_t v, int add)
{
    if (threadIdx.x == 0) *clock = add ? *clock + v : v;
}
}  // namespace

void launch_ml_init(hipStream_t st, float* master, uint64_t seed)
{
    launch(k_ml_init, dim3((kMlParams + 255) / 256), dim3(256), 0, st, master, seed);
}

void launch_eq9(hipStream_t st, bool fp64, const RepDev* reps, const FirTile* tiles,
                const double* amp, int amp_stride, const double* tw, int n, void* zeta,
                int64_t n_cols, const int64_t* clock, int64_t* marker, int K)
{
    const int L2 = __builtin_ctz((unsigned)n);
    const int cw = eq9_columns(n);
    const int64_t n_groups = n_cols / (2 * cw);
    const dim3 grid((unsigned)(n_groups < 2048 ? n_groups : 2048), 2u), block(256);
    const uint32_t lds = (uint32_t)(sizeof(double2) * (size_t)cw * n);
    if (fp64)
        launch(k_eq9<double>, grid, block, lds, st, reps, tiles, amp, amp_stride, tw, L2, cw,
               (double*)zeta, n_cols, (const int64_t*)clock, (const int64_t*)marker, K, n_groups);
    else
        launch(k_eq9<float>, grid, block, lds, st, reps, tiles, amp, amp_stride, tw, L2, cw,
               (float*)zeta, n_cols, (const int64_t*)clock, (const int64_t*)marker, K, n_groups);
    launch(k_eq9_mark, dim3(1), dim3(64), 0, st, clock, marker, n, K, 0);
}

void launch_barostat(hipStream_t st, RepDev* reps, int n_rep, const double* partials,
                     StepRef sync, int32_t* status)
{
    launch(k_barostat, dim3(n_rep), dim3(kBaroThreads), 0, st, reps, n_rep, partials, sync,
           status);
}

void launch_eq9_invalidate(hipStream_t st, int64_t* marker)
{
    launch(k_eq9_mark, dim3(1), dim3(64), 0, st, (const int64_t*)nullptr, marker, 1, 1, 1);
}

int eq9_columns(int n)
{
    // complex columns per block: 2048 points (32 KiB of LDS), within one
    // 256-column tile of a replica
    const int cw = 2048 / n;
    return cw < 1 ? 1 : (cw > kDofTile / 2 ? kDofTile / 2 : cw);
}

void launch_clock(hipStream_t st, int64_t* clock, int64_t v, bool add)
{
    launch(k_clock, dim3(1), dim3(64), 0, st, clock, v, add ? 1 : 0);
}

}  // namespace qtb
