// vdos.hip -- velocity density of states.  Sec. 3 names direct access to
// time-correlation functions as the advantage of QTB-MD over (QTB-)PIMD, and
// recommends checking the vibrational density of states whenever the
// friction gamma is raised against zero-point-energy leakage.  By the
// Wiener-Khinchin theorem the Fourier transform of the velocity
// autocorrelation is the power spectrum of the velocity series, estimated
// here by segment periodograms:
//   S_k = (1/n_seg) sum_segments sum_j w_j |sum_t v_{t,j} e^{-2 pi i k t/seg}|^2 / seg,
// k = 0 .. seg/2, with w_j the mass of dof j (S then averages to twice the
// kinetic energy over all seg frequencies).
//
// The series sits in HBM one sample per row ([t][n_dof], the order the step
// kernels write it, one coalesced row per sample).  A block transforms
// groups of CW complex columns in LDS: complex column q packs the real dofs
// 2q and 2q + 1, each scaled by the square root of its weight, so that
// w_a |A_k|^2 + w_b |B_k|^2 = (|Z_k|^2 + |Z_{-k}|^2) / 2 gives two real
// spectra from one complex FFT.  Radix-2 decimation in time, FP64, the
// input loaded in bit-reversed order; twiddles from a table computed once.
// Each block keeps the sum of its groups' periodograms in its own row of
// partials, summed over blocks in a fixed order by k_vdos_reduce: the result
// does not depend on scheduling.
#include "qtb_internal.h"

namespace qtb {

namespace {

// complex points per block (64 KiB of LDS)
constexpr int kVdosPoints = 4096;
constexpr int kVdosMaxGrid = 2048;

__global__ void __launch_bounds__(256) k_vdos_twiddle(double2* __restrict__ tw, int seg)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < seg / 2) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)seg, &s, &c);  // exp(-2 pi i k / seg)
        tw[k] = make_double2(c, s);
    }
}

__global__ void __launch_bounds__(256) k_vdos_fft(const double* __restrict__ v, int n_dof,
                                                  const double* __restrict__ weight,
                                                  const double2* __restrict__ tw, int L2, int cw,
                                                  int n_groups, double* __restrict__ partials)
{
    extern __shared__ double2 zb[];  // [cw][seg]
    const int seg = 1 << L2, hseg = seg >> 1, ncol = 2 * cw;
    const int lc = __builtin_ctz(ncol);
    double* __restrict__ prow = partials + (size_t)blockIdx.x * (hseg + 1);
    for (int g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const int c0 = g * ncol;
        // rows of ncol consecutive dofs (one coalesced segment per sample)
        for (int e = threadIdx.x; e < seg * ncol; e += blockDim.x) {
            const int t = e >> lc, c = e & (ncol - 1), j = c0 + c;
            double x = 0.0;
            if (j < n_dof) x = v[(size_t)t * n_dof + j] * sqrt(weight[j]);
            const int rt = (int)(__builtin_bitreverse32((uint32_t)t) >> (32 - L2));
            reinterpret_cast<double*>(zb + (size_t)(c >> 1) * seg + rt)[c & 1] = x;
        }
        __syncthreads();
        for (int s = 0; s < L2; ++s) {
            const int half = 1 << s;
            for (int b = threadIdx.x; b < cw * hseg; b += blockDim.x) {
                const int q = b >> (L2 - 1), jb = b & (hseg - 1), pos = jb & (half - 1);
                const int i0 = ((jb >> s) << (s + 1)) + pos, i1 = i0 + half;
                const double2 w = tw[pos << (L2 - 1 - s)];
                double2* z = zb + (size_t)q * seg;
                const double2 a = z[i0], u = z[i1];
                const double tr = w.x * u.x - w.y * u.y, ti = w.x * u.y + w.y * u.x;
                z[i0] = make_double2(a.x + tr, a.y + ti);
                z[i1] = make_double2(a.x - tr, a.y - ti);
            }
            __syncthreads();
        }
        for (int k = threadIdx.x; k <= hseg; k += blockDim.x) {
            const int km = (seg - k) & (seg - 1);
            double p = 0.0;
            for (int q = 0; q < cw; ++q) {
                const double2 a = zb[(size_t)q * seg + k], u = zb[(size_t)q * seg + km];
                p += a.x * a.x + a.y * a.y + u.x * u.x + u.y * u.y;
            }
            prow[k] = (g == (int)blockIdx.x) ? 0.5 * p : prow[k] + 0.5 * p;
        }
        __syncthreads();  // the next group overwrites the LDS columns
    }
}

// spec[k] = (accumulate ? spec[k] : 0) + scale * sum over rows of partials
__global__ void __launch_bounds__(256) k_vdos_reduce(const double* __restrict__ partials, int rows,
                                                     int nk, double* __restrict__ spec, double scale,
                                                     int accumulate)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += partials[(size_t)r * nk + k];
    spec[k] = (accumulate ? spec[k] : 0.0) + scale * s;
}

// w[a N + i] = m mu of atom i's species (the recorder's trace layout)
__global__ void __launch_bounds__(256) k_vdos_weights(const RepDev* __restrict__ reps, int r,
                                                      double* __restrict__ w)
{
    const RepDev& R = reps[r];
    const int n = R.dims * R.N;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        w[j] = R.mmu[R.species[j % R.N]];
}

}  // namespace

VdosPlan vdos_plan(int n_dof, int seg)
{
    VdosPlan p{};
    p.seg = seg;
    p.L2 = __builtin_ctz((unsigned)seg);
    p.cw = kVdosPoints / seg < 1 ? 1 : kVdosPoints / seg;
    const int n_pairs = (n_dof + 1) / 2;
    // no more complex columns per group than the dofs fill
    while (p.cw > 1 && p.cw / 2 >= n_pairs) p.cw /= 2;
    p.n_groups = (n_pairs + p.cw - 1) / p.cw;
    p.grid = p.n_groups < kVdosMaxGrid ? p.n_groups : kVdosMaxGrid;
    p.nk = seg / 2 + 1;
    return p;
}

void launch_vdos_twiddle(hipStream_t st, double* tw, int seg)
{
    launch(k_vdos_twiddle, dim3((seg / 2 + 255) / 256), dim3(256), 0, st,
           reinterpret_cast<double2*>(tw), seg);
}

void launch_vdos_segment(hipStream_t st, const VdosPlan& p, const double* v, int n_dof,
                         const double* weight, const double* tw, double* partials, double* spec,
                         double scale, bool accumulate)
{
    const uint32_t lds = (uint32_t)(sizeof(double2) * (size_t)p.cw * p.seg);
    launch(k_vdos_fft, dim3(p.grid), dim3(256), lds, st, v, n_dof, weight,
           reinterpret_cast<const double2*>(tw), p.L2, p.cw, p.n_groups, partials);
    launch(k_vdos_reduce, dim3((p.nk + 255) / 256), dim3(256), 0, st, (const double*)partials,
           p.grid, p.nk, spec, scale, accumulate ? 1 : 0);
}

void launch_vdos_weights(hipStream_t st, const RepDev* reps, int r, int n_dof, double* w)
{
    int blocks = (n_dof + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    launch(k_vdos_weights, dim3(blocks), dim3(256), 0, st, reps, r, w);
}

}  // namespace qtb
