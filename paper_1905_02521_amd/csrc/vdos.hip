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
// The series is read with a sample stride and a dof stride.  The recorder
// keeps one row of dofs per sample ([samples][dof], the row a step writes
// with coalesced stores); a block reads rows of its 2 CW dofs.  A block
// transforms groups of CW complex columns in LDS: complex column q packs the
// real dofs 2q and 2q + 1, each scaled by the square root of its weight, so
// that w_a |A_k|^2 + w_b |B_k|^2 = (|Z_k|^2 + |Z_{-k}|^2) / 2 gives two real
// spectra from one complex FFT.  FP64, in place, decimation in frequency on
// the naturally ordered input, two radix-2 stages at a time (a radix-4
// butterfly with one LDS round trip per pair of stages), the bins then read
// in bit-reversed order; twiddles from a table computed once.  Each block
// keeps the sum of its groups' periodograms in its own row of partials; two
// fixed-order passes sum the rows: the result does not depend on scheduling.
#include <mutex>

#include "fft_lds.h"
#include "qtb_internal.h"

namespace qtb {

namespace {

// complex points per block: 32 KiB of LDS (four blocks per CU) up to
// segments of 2048 samples, one 4096-point column (64 KiB) above
constexpr int kVdosPoints = 2048;
constexpr size_t kVdosLdsBytes = 65536;
constexpr int kVdosBatch = 8;
constexpr int kVdosMaxGrid = 1024;
constexpr int kVdosStageRows = 32;

__global__ void __launch_bounds__(256) k_vdos_twiddle(double2* __restrict__ tw, int seg)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < seg / 2) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)seg, &s, &c);  // exp(-2 pi i k / seg)
        tw[k] = make_double2(c, s);
    }
}

// LDS_TW: the twiddle table is copied into LDS behind the columns.  Groups
// follow the XCD-aware block order: groups g and g + 1, which share the HBM
// lines of a row of samples, run on one XCD at the same time.
template <bool LDS_TW>
__global__ void __launch_bounds__(256) k_vdos_fft(const double* __restrict__ v, int64_t ts,
                                                  int64_t js, int n_dof,
                                                  const double* __restrict__ tw_g, int L2, int cw,
                                                  int n_groups, const double* __restrict__ sqrt_w,
                                                  double* __restrict__ partials)
{
    extern __shared__ double2 zb[];  // [cw][seg], then the twiddles if LDS_TW
    const int seg = 1 << L2, hseg = seg >> 1, ncol = 2 * cw;
    const int lc = __builtin_ctz(ncol);
    const bool time_major = ts == 1;  // each dof's samples contiguous
    const int lb = xcd_block();
    const double2* __restrict__ twg = reinterpret_cast<const double2*>(tw_g);
    const size_t tw_off = (size_t)cw * seg;
    if (LDS_TW)  // made visible by the barrier after the first group's load
        for (int k = threadIdx.x; k < hseg; k += blockDim.x) zb[tw_off + k] = twg[k];
    auto tw = [&](int k) -> double2 {
        if constexpr (LDS_TW) return zb[tw_off + k];
        else return twg[k];
    };
    double* __restrict__ prow = partials + (size_t)lb * (hseg + 1);
    for (int g = lb; g < n_groups; g += gridDim.x) {
        const int c0 = g * ncol;
        // batches of kVdosBatch loads in flight per thread, then the LDS stores
        const int total = seg * ncol;
        for (int e0 = threadIdx.x; e0 < total; e0 += kVdosBatch * blockDim.x) {
            // unconditional loads (indices clamped into range), all in flight
            // together; out-of-range elements are zeroed afterwards
            double x[kVdosBatch], wj[kVdosBatch];
#pragma unroll
            for (int u = 0; u < kVdosBatch; ++u) {
                const int e = min(e0 + u * (int)blockDim.x, total - 1);
                const int t = time_major ? (e & (seg - 1)) : (e >> lc);
                const int c = time_major ? (e >> L2) : (e & (ncol - 1));
                const int j = min(c0 + c, n_dof - 1);
                x[u] = v[(int64_t)t * ts + (int64_t)j * js];
                wj[u] = sqrt_w[j];
            }
#pragma unroll
            for (int u = 0; u < kVdosBatch; ++u) {
                const int e = e0 + u * blockDim.x;
                if (e < total) {
                    const int t = time_major ? (e & (seg - 1)) : (e >> lc);
                    const int c = time_major ? (e >> L2) : (e & (ncol - 1));
                    reinterpret_cast<double*>(zb + (size_t)(c >> 1) * seg + t)[c & 1] =
                        (c0 + c < n_dof) ? x[u] * wj[u] : 0.0;
                }
            }
        }
        __syncthreads();
        fft_dif_lds(zb, cw, L2, tw);
        // bin k sits at the bit reverse of k
        for (int k = threadIdx.x; k <= hseg; k += blockDim.x) {
            const int rk = bit_reverse(k, L2), rm = bit_reverse((seg - k) & (seg - 1), L2);
            double p = 0.0;
            for (int q = 0; q < cw; ++q) {
                const double2 a = zb[(size_t)q * seg + rk], u = zb[(size_t)q * seg + rm];
                p += a.x * a.x + a.y * a.y + u.x * u.x + u.y * u.y;
            }
            prow[k] = (g == lb) ? 0.5 * p : prow[k] + 0.5 * p;
        }
        __syncthreads();  // the next group overwrites the LDS columns
    }
}

// Rows r = y, y + n_out, y + 2 n_out, ... of in [rows][nk], summed in that
// order: out[y][k] for n_out > 1; for n_out = 1 the final spectrum,
// spec[k] = (accumulate ? spec[k] : 0) + scale * sum.
__global__ void __launch_bounds__(256) k_vdos_reduce(const double* __restrict__ in, int rows,
                                                     int nk, double* __restrict__ out, int n_out,
                                                     double scale, int accumulate)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (k >= nk) return;
    double s = 0.0;
#pragma unroll 8
    for (int r = y; r < rows; r += n_out) s += in[(size_t)r * nk + k];
    if (n_out > 1) out[(size_t)y * nk + k] = s;
    else out[k] = (accumulate ? out[k] : 0.0) + scale * s;
}

// sw[a N + i] = sqrt(m mu) of atom i's species (the recorder's trace layout)
__global__ void __launch_bounds__(256) k_vdos_weights(const RepDev* __restrict__ reps, int r,
                                                      double* __restrict__ sw)
{
    const RepDev& R = reps[r];
    const int n = R.dims * R.N;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        sw[j] = sqrt(R.mmu[R.species[j % R.N]]);
}

__global__ void __launch_bounds__(256) k_vdos_sqrt(const double* __restrict__ w, int n,
                                                   double* __restrict__ sw)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        sw[j] = sqrt(w[j]);
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
    p.stage_rows = p.grid > kVdosStageRows ? kVdosStageRows : 0;
    return p;
}

void launch_vdos_twiddle(hipStream_t st, double* tw, int seg)
{
    launch(k_vdos_twiddle, dim3((seg / 2 + 255) / 256), dim3(256), 0, st,
           reinterpret_cast<double2*>(tw), seg);
}

void launch_vdos_segment(hipStream_t st, const VdosPlan& p, const double* v, int64_t ts,
                         int64_t js, int n_dof, const double* sqrt_w, const double* tw,
                         double* partials, double* stage, double* spec, double scale,
                         bool accumulate)
{
    const size_t cols = sizeof(double2) * (size_t)p.cw * p.seg, tws = sizeof(double2) * (p.seg / 2);
    if (cols + tws <= kVdosLdsBytes)
        launch(k_vdos_fft<true>, dim3(p.grid), dim3(256), (uint32_t)(cols + tws), st, v, ts, js,
               n_dof, tw, p.L2, p.cw, p.n_groups, sqrt_w, partials);
    else
        launch(k_vdos_fft<false>, dim3(p.grid), dim3(256), (uint32_t)cols, st, v, ts, js, n_dof,
               tw, p.L2, p.cw, p.n_groups, sqrt_w, partials);
    const unsigned bx = (unsigned)((p.nk + 255) / 256);
    const double* rows = partials;
    int n_rows = p.grid;
    if (p.stage_rows > 0) {
        launch(k_vdos_reduce, dim3(bx, (unsigned)p.stage_rows), dim3(256), 0, st, rows, n_rows,
               p.nk, stage, p.stage_rows, 1.0, 0);
        rows = stage;
        n_rows = p.stage_rows;
    }
    launch(k_vdos_reduce, dim3(bx, 1u), dim3(256), 0, st, rows, n_rows, p.nk, spec, 1, scale,
           accumulate ? 1 : 0);
}

void launch_vdos_weights(hipStream_t st, const RepDev* reps, int r, int n_dof, double* sw)
{
    int blocks = (n_dof + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    launch(k_vdos_weights, dim3(blocks), dim3(256), 0, st, reps, r, sw);
}

void launch_vdos_sqrt(hipStream_t st, const double* w, int n, double* sw)
{
    int blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    launch(k_vdos_sqrt, dim3(blocks), dim3(256), 0, st, w, n, sw);
}

}  // namespace qtb

// ------------------------------------------------- allocation-free spectrum
namespace qtb {
namespace {
// The scratch of qtb_vdos_spectrum_noalloc: a file-scope device array, one
// copy per GPU, alive until the process ends.  In host code its name stands
// for a host-side shadow, so the device address of each GPU's copy is looked
// up once (hipGetSymbolAddress, with that GPU current) and used instead.
constexpr size_t kVdosScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kVdosScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch (null on failure).
void* scratch_address(hipError_t& err)
{
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    err = hipSuccess;
    return g_scratch_ptr[dev];
}
}  // namespace

}  // namespace qtb

extern "C" qtb_status qtb_vdos_spectrum_noalloc(const double* d_v, int64_t n_samples,
                                                int32_t n_dof, int64_t sample_stride,
                                                int64_t dof_stride, const double* d_weight,
                                                int32_t seg, double* d_spec, void* hip_stream)
{
    if (!d_v || !d_weight || !d_spec || n_samples < 0 || sample_stride < 1 || dof_stride < 1) {
        qtb::set_static_error("bad spectrum arguments");
        return QTB_E_INVALID;
    }
    const size_t need = qtb_vdos_workspace_bytes(n_dof, seg, 0);
    if (need == 0) {
        qtb::set_static_error("n_dof >= 1 and seg a power of two in [16, 4096]");
        return QTB_E_INVALID;
    }
    if (need > qtb::kVdosScratchBytes) {
        qtb::set_static_error("qtb_vdos_spectrum_noalloc: the sizes need more scratch than its "
                              "static 16 MiB (qtb_vdos_workspace_bytes(n_dof, seg, 0)); use "
                              "qtb_vdos_spectrum with a workspace");
        return QTB_E_INVALID;
    }
    hipError_t err = hipSuccess;
    void* ws = qtb::scratch_address(err);
    if (!ws) {
        qtb::set_static_error(std::string("scratch address: ") + hipGetErrorString(err));
        return QTB_E_DEVICE;
    }
    return qtb_vdos_spectrum(d_v, n_samples, n_dof, sample_stride, dof_stride, d_weight, seg,
                             d_spec, ws, qtb::kVdosScratchBytes, hip_stream);
}
